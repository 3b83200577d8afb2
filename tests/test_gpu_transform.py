"""GPU parity of the C2R transform on its own (Alg. 2, last step): seeded random modes,
with garbage in the slots the transform must ignore (m > m_top and the imaginary part of
g_0), against the oracle's naive DFT for every FFT size the library builds (n_phi = 4 ..
16384); and smf_sample = smf_sample_modes then smf_transform, bit for bit."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# the FFT's own rounding: a few eps times log2(n_phi) relative RMS
TOL = {"fp64": 1e-13, "fp32": 2e-6}


def _plan(order, n_theta, n_phi, ell_max, precision):
    from paper_1709_10314_amd import Plan

    return Plan(order, n_theta, n_phi, ell_max, kappa=[50.0] * order, precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("log2n", list(range(2, 15)))
def test_transform_random_modes_matches_oracle_dft(log2n, precision):
    nphi = 1 << log2n
    n = 6 if nphi >= 4096 else 9
    lmax = max(1, nphi // 2 - 1 - (nphi // 8))          # m_top below n_phi/2 - 1: ignored tail
    count = 2
    plan = _plan(1, n, nphi, lmax, precision)
    mt = plan.m_top
    rng = np.random.default_rng(1000 + log2n)
    g = rng.standard_normal((count, n, nphi // 2, 2))    # garbage above m_top and in Im g_0
    dt = torch.float64 if precision == "fp64" else torch.float32
    data = torch.from_numpy(g).to(dt).cuda().contiguous()
    T = plan.transform(data, count)
    torch.cuda.synchronize()
    T = T.double().cpu().numpy()
    plan.close()
    gr = g.astype(np.float32).astype(np.float64) if precision == "fp32" else g
    go = gr[:, :, : mt + 1, 0] + 1j * gr[:, :, : mt + 1, 1]
    go[:, :, 0] = go[:, :, 0].real
    To = oracle.dft(go, nphi)
    e = max(rel_rms(T[f], To[f]) for f in range(count))
    log(f"n_phi {nphi} {precision}: m_top {mt}, rel RMS {e:.2e}")
    assert e <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sample_is_modes_then_transform(precision):
    plan = _plan(2, 130, 256, 200, precision)
    T = plan.sample(4, 3).clone()
    g = plan.sample_modes(4, 3)
    T2 = plan.transform(g, 3)
    torch.cuda.synchronize()
    assert torch.equal(T, T2)
    plan.close()


def test_transform_rejects_bad_arguments():
    from paper_1709_10314_amd import smf

    plan = _plan(1, 8, 16, 7, "fp64")
    assert smf.smf_transform(plan.handle, -1, 0) == smf.SMF_EINVAL
    assert smf.smf_transform(plan.handle, 1, 0) == smf.SMF_EINVAL
    assert smf.smf_transform(plan.handle, 0, 0) == smf.SMF_OK
    plan.close()
