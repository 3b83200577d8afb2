"""The library's diagnostics (smf_set_log_level, the SMF_LOG environment variable): the reason
for a rejected setup argument on stderr, the level taken from the environment, the setter's
contract.  No device is needed: a rejected argument is reported before any HIP call.  Each case
runs in a fresh process, whose stderr (written by the C library) the test reads."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1709_10314_amd", "libsmf.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsmf.so is not built")

SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
from paper_1709_10314_amd import smf
lvl = {level}
if lvl is not None:
    print("previous", smf.smf_set_log_level(lvl), flush=True)
rc, _ = smf.smf_setup(2, 8, 48, 15, kappa=[9.0, 16.0], flags=smf.SMF_FP64, stream=0)
print("rc", rc, flush=True)
rc, _ = smf.smf_setup(5, 8, 32, 15, kappa=[9.0, 16.0], flags=smf.SMF_FP64, stream=0)
print("rc", rc, flush=True)
print("negative", smf.smf_set_log_level(-1), flush=True)
"""


def _run(level=None, env_level=None):
    env = dict(os.environ)
    env.pop("SMF_LOG", None)
    if env_level is not None:
        env["SMF_LOG"] = str(env_level)
    p = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT, level=level)], env=env, capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    return p.stdout, p.stderr


def test_rejected_arguments_are_explained_at_level_1():
    out, err = _run(level=1)
    assert "previous 0" in out and out.count("rc -1") == 2 and "negative -1" in out
    assert "[smf] smf_setup: invalid argument: n_phi must be a power of two in [4, 16384]" in err
    assert "[smf] smf_setup: invalid argument: order must be 1, 2, 3 or 4" in err


def test_silent_by_default():
    out, err = _run()
    assert out.count("rc -1") == 2
    assert "[smf]" not in err


def test_level_from_the_environment():
    out, err = _run(level=0, env_level=2)
    assert "previous 2" in out
    assert "[smf]" not in err          # the setter replaced the environment's level before the calls
    out, err = _run(env_level=1)
    assert err.count("[smf] smf_setup: invalid argument") == 2
