"""Pieces of the paper's convergence experiment (Sec. 5, Fig. 3) shared by its CPU and GPU
tests: the spectrum of eq. (sample_spec), the field covariance C_T of Sec. 5, the point sets
(equator, meridian), and the exact covariance of the sampled field from the chains' factors.
Plain numpy; no part of the sampling path."""
import numpy as np

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


def chain_mode_covariance(A, B, n, m, pts):
    """K^m between the rings of the points pts = [(ring, phi)]: the value component of the
    chain's joint covariance, propagated exactly through the factors of mode m in
    generation order (start, crossing, outward both ways, the southern steps mirrored)."""
    s = n // 2 - 1 if n % 2 == 0 else (n - 1) // 2
    even = n % 2 == 0
    M = A.shape[-1]
    D = np.diag([(-1.0) ** p for p in range(M)])
    rings = np.array([p[0] for p in pts])
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
    return np.array([[cov[(a, b)][0, 0] for b in rings] for a in rings])


def chain_field_covariance(A, B, n, m_top, pts):
    """Exact covariance of the sampled field between the points pts = [(ring, phi)], the
    modes' chain covariances summed over m <= m_top with weights 1 (m = 0), 2."""
    phis = np.array([p[1] for p in pts])
    out = np.zeros((len(pts), len(pts)))
    for m in range(m_top + 1):
        w = 1.0 if m == 0 else 2.0
        out += w * chain_mode_covariance(A, B, n, m, pts) * np.cos(m * (phis[:, None] - phis[None, :]))
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



def exact_errors(A, B, n, m_top, nyquist=False):
    """Largest |Cov(x, y) - C_T(x, y)| over the equator and the meridian point sets of the
    exact covariance of the sampled field, modes m <= m_top with weights 1 (m = 0) and 2
    (every other mode: the real part of g_m e^{i m phi} taken twice).  nyquist=True adds the
    paper's reading of Alg. 2's last step with m_max = n_theta and n_phi = 2 n_theta: the sum
    runs to m = m_max, whose term g_{m_max} e^{i pi j} has no conjugate partner and keeps its
    real part, Re(g_{m_max}) (-1)^j, of covariance K^{m_max}(x, y) / 2 cos(m phi_x) cos(m phi_y).
    A and B must then hold the factors of mode m_top + 1 = m_max as well."""
    out = {}
    for name, pts in zip(("equator", "meridian"), point_sets(n)):
        CT = covariance_CT(cos_gamma(pts, n))
        K = chain_field_covariance(A, B, n, m_top, pts)
        if nyquist:
            mx = m_top + 1
            Kn = chain_mode_covariance(A, B, n, mx, pts)
            ph = np.array([p[1] for p in pts])
            K = K + 0.5 * Kn * np.cos(mx * ph)[:, None] * np.cos(mx * ph)[None, :]
        out[name] = float(np.max(np.abs(K - CT)))
    return out


def slope(rows, key, kind):
    """Least-squares slope of log(error) against log(n_theta)."""
    x = np.log([r["n_theta"] for r in rows])
    y = np.log([r[key][kind] for r in rows])
    return float(np.polyfit(x, y, 1)[0])


