"""The binding's ctypes structures against the C header: size and every
field offset of each public struct, as the system C compiler lays them out
from include/logfx.h.  Host only."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1304_3992_amd import logfx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {
    "logfx_image": logfx.logfx_image,
    "logfx_mask": logfx.logfx_mask,
    "logfx_params": logfx.logfx_params,
    "logfx_report": logfx.logfx_report,
    "logfx_tune_result": logfx.logfx_tune_result,
}


def test_ctypes_layout_matches_header(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "logfx.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", exe], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([exe], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for name, cls in STRUCTS.items():
        assert int(got[f"{name} size"]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)
