"""The benchmark's command line, without a GPU: more than one GPU is
refused with a message, and the hash that ties the traffic figures to the
kernel sources is stable."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_kernel_source_hash_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 16
    assert len(bench.TRAFFIC_SOURCE_HASH) == 16
    assert set(bench.TRAFFIC_BYTES) == {"pass1_kernel", "pass2z_kernel"}
    # every kernel source outside the gate network's files takes part
    import glob
    csrc = os.path.join(ROOT, "paper_1304_3992_amd", "csrc")
    kernel_files = {os.path.basename(f) for f in glob.glob(os.path.join(csrc, "*.h")) + glob.glob(os.path.join(csrc, "*.hip"))}
    assert set(bench.PIPELINE_SOURCES) == {f for f in kernel_files if not f.startswith("logfx_gate")}
