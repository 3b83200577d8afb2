"""The paper's convergence experiment (Sec. 5, Fig. 3) on the GPU path.

Spectrum C_l = (10 + l^2 (l+1)^2)^-1 (order 2), grids n_theta in {4, 8, 16, 32} with
n_phi = 2 n_theta (m_max = n_theta), N = 320,000 samples per grid; the error is the largest
|Cov_hat(x, y) - C_T(x, y)| over the point pairs of a set S, once the equator and once a
meridian.  Readings: the infinite spectrum is summed to ell_max = 4095 in the setup (the tail
beyond is below 1e-7 of C_T(0)); the ring-centre grids have no equator ring, so the equator
set is the ring next to it (z = sin(pi / (2 n))); the meridian set is the great circle
phi in {0, pi}; the Nyquist mode is not sampled, so m_top = n_theta - 1.

Beside the empirical covariance of GPU samples, the sampler's exact covariance (its factors'
chain covariances, summed over the sampled modes) separates the method's error from the
sampling noise: the empirical covariance must agree with it within the sampling error, and
the exact error must fall as n_theta^-2 (the oracle-only test of the same experiment also
takes the paper's reading with the Nyquist term kept, and finds the same rate)."""
import numpy as np
import pytest

import oracle
from fig3 import GRIDS, LMAX, chain_field_covariance, cos_gamma, covariance_CT, point_sets, slope, spectrum
from gpu_helpers import log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_PAPER = 320_000


def empirical(plan, n, nsamp, batch=32_000, seed=1):
    """N^-1 sum_j T_j(x) T_j(y) over both point sets, from GPU samples in batches (the
    Gram matrices accumulate in FP64 on the GPU)."""
    s = n // 2 - 1
    Ge = torch.zeros(2 * n, 2 * n, dtype=torch.float64, device="cuda")
    Gm = torch.zeros(2 * n, 2 * n, dtype=torch.float64, device="cuda")
    out = plan.empty(batch)
    done = 0
    while done < nsamp:
        c = min(batch, nsamp - done)
        T = plan.sample(seed + done, c, out)[:c]
        Xe = T[:, s, :].double()
        Xm = torch.cat([T[:, :, 0], T[:, :, n]], dim=1).double()
        Ge += Xe.T @ Xe
        Gm += Xm.T @ Xm
        done += c
    torch.cuda.synchronize()
    return (Ge / nsamp).cpu().numpy(), (Gm / nsamp).cpu().numpy()


def run_experiment(nsamp, precision="fp32"):
    from paper_1709_10314_amd import Plan

    C = spectrum(LMAX)
    rows = []
    for n in GRIDS:
        plan = Plan(2, n, 2 * n, LMAX, c_ell=C, precision=precision)
        m_top = plan.m_top
        Ce, Cm = empirical(plan, n, nsamp)
        plan.close()
        A, B = oracle.setup(2, C, n, 2 * n)
        res = {"n_theta": n, "m_top": m_top}
        for name, pts, Cemp in (("equator", point_sets(n)[0], Ce), ("meridian", point_sets(n)[1], Cm)):
            CT = covariance_CT(cos_gamma(pts, n))
            Cex = chain_field_covariance(A, B, n, m_top, pts)
            # sampling standard error of each entry (Isserlis): sqrt((C_xx C_yy + C_xy^2) / N)
            d = np.diag(Cex)
            se = np.sqrt((d[:, None] * d[None, :] + Cex ** 2) / nsamp)
            res[name] = {"err_empirical": float(np.max(np.abs(Cemp - CT))),
                         "err_exact": float(np.max(np.abs(Cex - CT))),
                         "max_z_empirical_vs_exact": float(np.max(np.abs(Cemp - Cex) / se)),
                         "CT0": float(CT[0, 0])}
        rows.append(res)
        log(f"n_theta {n:2d} (m_top {m_top:2d}): equator exact {res['equator']['err_exact']:.3e} "
            f"empirical {res['equator']['err_empirical']:.3e}; meridian exact {res['meridian']['err_exact']:.3e} "
            f"empirical {res['meridian']['err_empirical']:.3e}; max |z| {max(res['equator']['max_z_empirical_vs_exact'], res['meridian']['max_z_empirical_vs_exact']):.2f}")
    return rows


def test_covariance_convergence_paper_experiment():
    rows = run_experiment(N_PAPER)
    for key in ("equator", "meridian"):
        ex = [r[key]["err_exact"] for r in rows]
        log(f"{key}: exact-error slope {slope(rows, key, 'err_exact'):.2f}, "
            f"empirical-error slope {slope(rows, key, 'err_empirical'):.2f}")
        # the method's error falls with the resolution, as n_theta^-2 (-2.02 fitted) ...
        assert all(b < a for a, b in zip(ex, ex[1:])), ex
        assert -2.1 <= slope(rows, key, "err_exact") <= -1.9
        # ... and with the paper's N the sampling error flattens the empirical curve at the
        # finer grids (the paper's m_max^-3/2 lies in this band; measured -1.2 and -1.05)
        assert -2.1 <= slope(rows, key, "err_empirical") <= -0.9
        # ... and the GPU samples have the sampler's covariance within the sampling error
        for r in rows:
            assert r[key]["max_z_empirical_vs_exact"] < 6.0, (key, r)
