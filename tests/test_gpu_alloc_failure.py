"""Allocation failures (smf_debug_fail_alloc): every setup entry point, with its k-th device
or pinned allocation made to fail for every k until the setup gets through, returns
SMF_ENOMEM, creates no plan and keeps no memory; the setup that then succeeds works."""
import numpy as np
import pytest

from gpu_helpers import log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def _sweep(make, destroy):
    """Runs make() with the k-th allocation failing, k = 0, 1, ...; returns how many
    allocations the setup makes."""
    from paper_1709_10314_amd import smf

    lib = smf.load()
    k = 0
    while True:
        assert lib.smf_debug_fail_alloc(k) == smf.SMF_OK
        try:
            rc, h = make()
        finally:
            lib.smf_debug_fail_alloc(-1)
        if rc == smf.SMF_OK:
            destroy(h)
            return k
        assert rc == smf.SMF_ENOMEM, (k, rc)
        assert not h.value, k
        k += 1
        assert k < 64


CASES = {
    "setup-fp32-scan": lambda smf: smf.smf_setup(2, 64, 128, 63, kappa=[100.0, 100.0], flags=smf.SMF_FP32),
    "setup-fp64-no-mirror": lambda smf: smf.smf_setup(1, 33, 64, 32, kappa=[50.0],
                                                      flags=smf.SMF_FP64 | smf.SMF_NO_MIRROR),
    "setup-green": lambda smf: smf.smf_setup(1, 32, 64, 0, kappa=[64.0], flags=smf.SMF_FP32 | smf.SMF_GREEN),
    "setup-explicit-c": lambda smf: smf.smf_setup(2, 16, 32, 15, c_ell=1.0 / (10.0 + np.arange(16.0) ** 4),
                                                  flags=smf.SMF_FP64),
    "setup-batch": lambda smf: smf.smf_setup_batch(
        [dict(n_theta=16, n_phi=32, order=1, kappa=[9.0], ell_max=15),
         dict(n_theta=33, n_phi=64, order=2, kappa=[40.0, 40.0], ell_max=32)]),
    "setup-rings": lambda smf: smf.smf_setup_rings(2, np.array([4, 8, 8, 4], dtype=np.int32),
                                                   np.zeros(4), 5, kappa=[30.0, 30.0], flags=smf.SMF_FP64),
    # rings of the power-of-two and Bluestein transform classes (their tables and kernels' transforms)
    "setup-rings-classes": lambda smf: smf.smf_setup_rings(1, np.array([1024, 2042, 2042, 1024], dtype=np.int32),
                                                           np.zeros(4), 5, kappa=[30.0], flags=smf.SMF_FP32),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_every_allocation_failure_is_clean(name):
    from paper_1709_10314_amd import smf

    make = lambda: CASES[name](smf)   # noqa: E731
    n_alloc = _sweep(make, smf.smf_destroy)          # warm-up: library and runtime state settle
    before = _free()
    for _ in range(3):
        assert _sweep(make, smf.smf_destroy) == n_alloc
    after = _free()
    log(f"{name}: {n_alloc} allocations, each failed once; free memory {before} -> {after}")
    assert n_alloc >= 3
    assert after >= before - (4 << 20)


def test_plan_works_after_failures():
    from paper_1709_10314_amd import Plan, smf

    lib = smf.load()
    lib.smf_debug_fail_alloc(2)
    with pytest.raises(smf.SmfError):
        Plan(1, 16, 32, 15, kappa=[9.0], precision="fp64")
    lib.smf_debug_fail_alloc(-1)
    p = Plan(1, 16, 32, 15, kappa=[9.0], precision="fp64")
    T = p.sample(1, 2)
    torch.cuda.synchronize()
    assert torch.isfinite(T).all() and float(T.abs().max()) > 0
    p.close()
    assert lib.smf_debug_fail_alloc(-2) == smf.SMF_EINVAL
