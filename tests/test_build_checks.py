"""The build's refusal of kernels that spill vector registers: the parser of
the compiler's resource-usage remarks (no GPU, no compile)."""
from paper_1304_3992_amd import build

REMARKS = """\
x.h:519:1: remark: Function Name: _ZN5logfx4kern12pass1_kernelIiLi1ELi1ELi0ELb1EE [-Rpass-analysis=kernel-resource-usage]
x.h:519:1: remark:     VGPRs: 128 [-Rpass-analysis=kernel-resource-usage]
x.h:519:1: remark:     SGPRs Spill: 2 [-Rpass-analysis=kernel-resource-usage]
x.h:519:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
x.h:519:1: remark: Function Name: _ZN5logfx4kern12pass2_kernelIiLi4ELi4ELi5ELb0EE [-Rpass-analysis=kernel-resource-usage]
x.h:519:1: remark:     SGPRs Spill: 38 [-Rpass-analysis=kernel-resource-usage]
x.h:519:1: remark:     VGPRs Spill: 25 [-Rpass-analysis=kernel-resource-usage]
"""


def test_vgpr_spills_found_per_kernel():
    assert build._vgpr_spills(REMARKS) == ["_ZN5logfx4kern12pass2_kernelIiLi4ELi4ELi5ELb0EE (25)"]


def test_no_spills_no_names():
    assert build._vgpr_spills(REMARKS.replace("VGPRs Spill: 25", "VGPRs Spill: 0")) == []
    assert build._vgpr_spills("") == []
