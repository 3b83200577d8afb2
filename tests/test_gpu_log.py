"""The library's diagnostics on a device: with SMF_LOG=2, a plan's setup, a ring plan's
transform classes and each sampling call's launch shape are reported on stderr (read from a
fresh process, where the C library writes it)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
import torch
from paper_1709_10314_amd import Plan, RingPlan, workloads
p = Plan(2, 64, 128, 63, kappa=[400.0, 400.0], precision="fp32")
p.sample(1, 2)
p.close()
z, n_ring, phi0 = workloads.healpix_rings(16)
r = RingPlan(2, n_ring, phi0, 47, kappa=[400.0, 400.0], precision="fp32", z=z)
r.sample_rings(1, 2)
r.close()
torch.cuda.synchronize()
print("done", flush=True)
"""


def test_setups_and_calls_are_reported_at_level_2():
    env = dict(os.environ)
    env["SMF_LOG"] = "2"
    p = subprocess.run([sys.executable, "-u", "-c", SCRIPT.format(root=ROOT)], env=env, capture_output=True, text=True,
                       timeout=300)
    print(p.stderr[-3000:], flush=True)
    assert p.returncode == 0 and "done" in p.stdout
    err = p.stderr
    assert "[smf] setup: order 2, 64 x 128 rings x longitudes, ell_max 63" in err
    assert "[smf] sample: 2 fields" in err and "then the transform" in err
    assert "[smf] setup_rings: 63 rings, 3072 pixels per field" in err
    assert "[smf] synthesize_rings: 2 fields" in err
