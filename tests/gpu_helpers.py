"""Shared helpers of the GPU tests (comparison metrics; no method arithmetic)."""
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(x, ref):
    """sqrt(sum (x - ref)^2 / sum ref^2) over all elements."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.sum(ref * ref)
    return float(np.sqrt(np.sum((x - ref) ** 2) / den)) if den > 0 else float(np.sqrt(np.sum(x * x)))


def marginal_sd(A, B, n_theta):
    """Marginal standard deviations (per state component) before and after each factor
    set, from exact covariance propagation of the northern chain through (A, B); these
    equal sqrt(diag J) at the rings (the chain reproduces J at each ring).
    Returns sd_a, sd_b of shape [sets, modes, order]."""
    ns, nm, M, _ = A.shape
    even = n_theta % 2 == 0
    sig = {}
    sd_a = np.zeros((ns, nm, M))
    sd_b = np.zeros((ns, nm, M))
    S0 = np.einsum("mpk,mqk->mpq", B[0], B[0])
    sd_a[0] = sd_b[0] = np.sqrt(np.maximum(np.einsum("mpp->mp", S0), 0))
    prev = S0
    for j in range(1, ns):
        Sa = S0 if (j == 1 or (even and j == 2)) else prev
        Sb = np.einsum("mpk,mkl,mql->mpq", A[j], Sa, A[j]) + np.einsum("mpk,mqk->mpq", B[j], B[j])
        sd_a[j] = np.sqrt(np.maximum(np.einsum("mpp->mp", Sa), 0))
        sd_b[j] = np.sqrt(np.maximum(np.einsum("mpp->mp", Sb), 0))
        if not (even and j == 1):
            prev = Sb
    return sd_a, sd_b


def factor_errors(Ag, Bg, Ao, Bo, n_theta):
    """Errors of device factors against oracle factors in units of the marginal standard
    deviations: |dA_pq| sd_a,q / sd_b,p and |dB_pq| / sd_b,p (rows with sd_b = 0 must be
    zero on both sides).  Returns (max dA, max dB)."""
    sd_a, sd_b = marginal_sd(Ao, Bo, n_theta)
    live = sd_b > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        dA = np.abs(Ag - Ao) * sd_a[:, :, None, :] / sd_b[:, :, :, None]
        dB = np.abs(Bg - Bo) / sd_b[:, :, :, None]
    dA = np.where(live[..., None], dA, np.abs(Ag - Ao))
    dB = np.where(live[..., None], dB, np.abs(Bg - Bo))
    return float(np.nanmax(dA)), float(np.nanmax(dB))
