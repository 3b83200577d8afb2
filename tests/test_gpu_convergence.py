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
the exact error must fall with n_theta."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LMAX = 4095
GRIDS = (4, 8, 16, 32)
N_PAPER = 320_000


def spectrum(lmax):
    ell = np.arange(lmax + 1, dtype=np.float64)
    return 1.0 / (10.0 + ell ** 2 * (ell + 1.0) ** 2)


def covariance_CT(cosg, lmax=20000):
    """C_T = sum_l (2l+1)/(4 pi) C_l P_l(cos gamma), Legendre polynomials by their
    three-term recurrence, summed to lmax (the remainder is below 1e-9 of C_T(0))."""
    x = np.asarray(cosg, dtype=np.float64)
    C = spectrum(lmax)
    p_prev, p = np.ones_like(x), x.copy()
    acc = C[0] / (4 * np.pi) * p_prev + 3 * C[1] / (4 * np.pi) * p
    for ell in range(1, lmax):
        p_prev, p = p, ((2 * ell + 1) * x * p - ell * p_prev) / (ell + 1)
        acc += (2 * ell + 3) / (4 * np.pi) * C[ell + 1] * p
    return acc


def chain_field_covariance(A, B, n, m_top, pts):
    """Exact covariance of the sampled field between the points pts = [(ring, phi)], from
    the chains' joint covariances (propagated through the factors in generation order, the
    southern steps mirrored) summed over the sampled modes with weights 1 (m = 0), 2."""
    s = n // 2 - 1 if n % 2 == 0 else (n - 1) // 2
    even = n % 2 == 0
    D = np.diag([1.0, -1.0])
    rings = np.array([p[0] for p in pts])
    phis = np.array([p[1] for p in pts])
    out = np.zeros((len(pts), len(pts)))
    for m in range(m_top + 1):
        steps = [(s, None, None, B[0, m])]
        for j in range(2 if even else 1, A.shape[0]):
            b = s - j + 1 if even else s - j
            steps.append((b, b + 1, A[j, m], B[j, m]))
        prev, j0 = s, 1
        if even:
            steps.append((s + 1, s, A[1, m], B[1, m]))
            prev, j0 = s + 1, 2
        for j in range(j0, A.shape[0]):
            steps.append((prev + 1, prev, D @ A[j, m] @ D, D @ B[j, m] @ D))
            prev += 1
        cov, done = {}, []
        for r, parent, P, Q in steps:
            if parent is None:
                cov[(r, r)] = Q @ Q.T
            else:
                for k in done:
                    cov[(r, k)] = P @ cov[(parent, k)]
                    cov[(k, r)] = cov[(r, k)].T
                cov[(r, r)] = P @ cov[(parent, parent)] @ P.T + Q @ Q.T
            done.append(r)
        K = np.array([[cov[(a, b)][0, 0] for b in rings] for a in rings])
        w = 1.0 if m == 0 else 2.0
        out += w * K * np.cos(m * (phis[:, None] - phis[None, :]))
    return out


def point_sets(n):
    s = n // 2 - 1
    nphi = 2 * n
    equator = [(s, 2 * np.pi * k / nphi) for k in range(nphi)]
    meridian = [(i, 0.0) for i in range(n)] + [(i, np.pi) for i in range(n)]
    return equator, meridian


def cos_gamma(pts, n):
    th = np.pi * (np.arange(n) + 0.5) / n
    t = th[[p[0] for p in pts]]
    ph = np.array([p[1] for p in pts])
    return np.cos(t)[:, None] * np.cos(t)[None, :] + np.sin(t)[:, None] * np.sin(t)[None, :] * np.cos(
        ph[:, None] - ph[None, :])


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


def slope(rows, key, kind):
    x = np.log([r["n_theta"] for r in rows])
    y = np.log([r[key][kind] for r in rows])
    return float(np.polyfit(x, y, 1)[0])


def test_covariance_convergence_paper_experiment():
    rows = run_experiment(N_PAPER)
    for key in ("equator", "meridian"):
        ex = [r[key]["err_exact"] for r in rows]
        log(f"{key}: exact-error slope {slope(rows, key, 'err_exact'):.2f}, "
            f"empirical-error slope {slope(rows, key, 'err_empirical'):.2f}")
        # the method's error falls with the resolution ...
        assert all(b < a for a, b in zip(ex, ex[1:])), ex
        # ... and the GPU samples have the sampler's covariance within the sampling error
        for r in rows:
            assert r[key]["max_z_empirical_vs_exact"] < 6.0, (key, r)
