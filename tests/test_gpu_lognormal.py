"""The lognormal field exp(mu + sigma T) (the application named at the end of Sec. 4),
mapped by the FFT as it stores T: against exp of the same call's Gaussian field from
smf_sample (FP64 to 1e-14, FP32 within expf's own error plus the rounding of
fmaf(sigma, T, mu)), against exp(mu + sigma T_oracle) at the parity bars, and the argument
checks."""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}


def _plan(order, n, nphi, lmax, kap, precision):
    from paper_1709_10314_amd import Plan

    return Plan(order, n, nphi, lmax, kappa=[kap] * order, precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", [(1, 64, 128, 63, 64.0, 0.0, 1.0), (2, 130, 256, 200, 700.0, -1.5, 40.0),
                                  (2, 256, 1024, 255, 2500.0, 0.3, 400.0)],
                         ids=lambda c: "M%d-%dx%d-l%d-k%g-mu%g-s%g" % c)
def test_lognormal_is_exp_of_the_field(case, precision):
    order, n, nphi, lmax, kap, mu, sig = case
    count, seed = 3, 41
    plan = _plan(order, n, nphi, lmax, kap, precision)
    T = plan.sample(seed, count).clone()
    L = plan.sample_lognormal(seed, count, mu, sig)
    torch.cuda.synchronize()
    T = T.cpu().numpy()
    L = L.cpu().numpy()
    plan.close()
    if precision == "fp64":
        ref = np.exp(mu + sig * T)
        e = float(np.max(np.abs(L - ref) / ref))
        bound = 1e-14
    else:
        y = np.float32(mu) + np.float32(sig) * T.astype(np.float64)
        ref = np.exp(y)
        e = float(np.max(np.abs(L.astype(np.float64) - ref) / ref))
        # expf to a few ulps, plus the rounding of the fused y (|y| 2^-24 relative in exp)
        bound = 4 * 2.0 ** -24 + float(np.max(np.abs(y))) * 2.0 ** -24 * 2
    ymax = float(np.max(np.abs(mu + sig * T)))
    log(f"{case} {precision}: max |y| {ymax:.2f}, max rel err vs exp(field) {e:.2e} (bound {bound:.2e})")
    assert e <= bound
    # end to end against the oracle field
    C = oracle.spectrum([kap] * order, lmax)
    A, B = oracle.setup(order, C, n, nphi)
    To, _ = oracle.sample(order, n, nphi, A, B, seed, count)
    for f in range(count):
        Lo = np.exp(mu + sig * To[f])
        el = rel_rms(L[f].astype(np.float64), Lo)
        eT = rel_rms(T[f].astype(np.float64), To[f])
        # exp turns an absolute error d in y into a relative one; sigma |T| scales T's error
        lim = TOL[precision] * max(1.0, sig * float(np.max(np.abs(To[f]))))
        log(f"  field {f}: lognormal rel RMS {el:.2e} (field {eT:.2e}, limit {lim:.2e})")
        assert el <= lim


def test_lognormal_rejects_bad_arguments():
    from paper_1709_10314_amd import smf

    plan = _plan(1, 8, 16, 7, 30.0, "fp64")
    out = plan.empty(1)
    for mu, sig in ((math.nan, 1.0), (0.0, math.inf)):
        assert smf.smf_sample_lognormal(plan.handle, 1, 1, mu, sig, out.data_ptr()) == smf.SMF_EINVAL
    assert smf.smf_sample_lognormal(plan.handle, 1, -1, 0.0, 1.0, out.data_ptr()) == smf.SMF_EINVAL
    assert smf.smf_sample_lognormal(plan.handle, 1, 0, 0.0, 1.0, 0) == smf.SMF_OK
    plan.close()
