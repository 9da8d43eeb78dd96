"""LOGFX_LOG=1: liblogfx writes every error (and one line per pipeline
call) to stderr.  Checked on the host-only entry points, in a child
process so that the setting, read once, does not leak into other tests."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, %r)
from paper_1304_3992_amd import logfx
lib = logfx.load()
rc = lib.logfx_make_log_mask(4, 1.0, 16, None, None)
print("rc", rc)
""" % ROOT


def _run(env_value):
    env = dict(os.environ)
    env.pop("LOGFX_LOG", None)
    if env_value is not None:
        env["LOGFX_LOG"] = env_value
    return subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True, timeout=120)


def test_errors_logged_when_enabled():
    r = _run("1")
    assert r.returncode == 0 and "rc 1" in r.stdout
    assert "[liblogfx] error 1:" in r.stderr and "taps_out is NULL" in r.stderr


def test_silent_by_default():
    for v in (None, "0"):
        r = _run(v)
        assert r.returncode == 0 and "[liblogfx]" not in r.stderr
