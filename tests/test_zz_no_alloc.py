"""The allocation-free ring sampling call (smf_sample_rings_noalloc) through the C ABI against
smf_sample_rings with a caller-given work buffer: equal pixels on two calls in a row, the
second with fewer fields, for FP32 and FP64 HEALPix plans; a request beyond the library's
64 MiB array is rejected."""
import numpy as np
import pytest

from gpu_helpers import log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,nside,order", [("fp32", 16, 2), ("fp64", 8, 1), ("fp32", 64, 2)])
def test_noalloc_equals_work_buffer_form(precision, nside, order):
    from paper_1709_10314_amd import RingPlan, smf, workloads

    z, n_ring, phi0 = workloads.healpix_rings(nside)
    plan = RingPlan(order, n_ring, phi0, 3 * nside - 1, kappa=[400.0] * order, precision=precision, z=z)
    for seed, count in ((5, 4), (9, 2)):          # the second call is smaller
        ref = plan.sample_rings(seed, count)
        out = plan.empty_rings(count)
        out.fill_(float("nan"))
        got = plan.sample_rings_noalloc(seed, count, out)
        torch.cuda.synchronize()
        log(f"noalloc {precision} nside {nside} seed {seed} x{count}: "
            f"max |diff| {float((got - ref).abs().max()):.3e}")
        assert torch.equal(got, ref)
    elem = 8 if precision == "fp64" else 4
    too_many = (64 << 20) // (plan.n_theta * plan.n_phi * elem) + 1
    out = plan.empty_rings(1)
    assert smf.smf_sample_rings_noalloc(plan.handle, 1, too_many, out.data_ptr()) == smf.SMF_EINVAL
    assert smf.smf_sample_rings_noalloc(plan.handle, 1, 0, out.data_ptr()) == smf.SMF_OK
    plan.close()
