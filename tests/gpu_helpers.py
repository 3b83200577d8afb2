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


def max_rel_err(x, ref):
    """max |x - ref| over all elements, relative to the RMS of ref (the element-wise
    companion of rel_rms: a few large local errors that an RMS would average away show)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = np.sqrt(np.mean(ref * ref))
    d = float(np.max(np.abs(x - ref))) if x.size else 0.0
    return d / rms if rms > 0 else d


def chain_covariances(A, B, n_theta):
    """Covariance of the state before (Sa) and after (Sb) each factor set, by exact
    propagation of the northern chain through (A, B) from the start factor; the chain
    reproduces J at each ring, so these are J(a,a) and J(b,b).  Shapes [sets, modes, M, M]."""
    ns, nm, M, _ = A.shape
    even = n_theta % 2 == 0
    Sa = np.zeros((ns, nm, M, M))
    Sb = np.zeros((ns, nm, M, M))
    S0 = np.einsum("mpk,mqk->mpq", B[0], B[0])
    Sa[0] = Sb[0] = S0
    prev = S0
    for j in range(1, ns):
        Sa[j] = S0 if (j == 1 or (even and j == 2)) else prev
        Sb[j] = np.einsum("mpk,mkl,mql->mpq", A[j], Sa[j], A[j]) + np.einsum("mpk,mqk->mpq", B[j], B[j])
        if not (even and j == 1):
            prev = Sb[j]
    return Sa, Sb


def _sqrtm_psd(S):
    w, V = np.linalg.eigh(S)
    return np.einsum("...ij,...j,...kj->...ik", V, np.sqrt(np.clip(w, 0, None)), V)


def threshold_ambiguous(Ao, Bo, n_theta, lo=1e-14, hi=1e-10):
    """Steps whose factorisation sits near the 1e-12 thresholds, from the oracle's chain:
    the smaller pivot 1 - rho^2 of the equilibrated J(a,a) (order 2; every pivot for orders 3
    and 4) or a relative
    conditional variance diag(B B^T) / diag J(b,b) within [lo, hi].  There keeping or
    dropping a pivot changes the conditional law discontinuously, and two FP64 roundings
    of J may fall on different sides.  Returns a [sets, modes] bool mask."""
    Sa, Sb = chain_covariances(Ao, Bo, n_theta)
    M = Ao.shape[-1]
    amb = np.zeros(Ao.shape[:2], dtype=bool)
    with np.errstate(divide="ignore", invalid="ignore"):
        if M == 2:
            d = Sa[..., 0, 0] * Sa[..., 1, 1]
            piv = np.where(d > 0, 1 - Sa[..., 0, 1] ** 2 / d, 1.0)
            amb |= (piv >= lo) & (piv <= hi)
        elif M > 2:
            # every pivot of the thresholded Cholesky of the equilibrated J(a,a)
            dg = np.sqrt(np.clip(np.einsum("...pp->...p", Sa), 0, None))
            inv = np.where(dg > 0, 1.0 / np.where(dg > 0, dg, 1.0), 0.0)
            R = Sa * inv[..., :, None] * inv[..., None, :]
            L = np.zeros_like(R)
            for j in range(M):
                piv = R[..., j, j] - np.sum(L[..., j, :j] ** 2, axis=-1)
                if j > 0:
                    amb |= (piv >= lo) & (piv <= hi)
                keep = piv > 1e-12
                g = np.sqrt(np.where(keep, piv, 1.0))
                for i in range(j + 1, M):
                    v = R[..., i, j] - np.sum(L[..., i, :j] * L[..., j, :j], axis=-1)
                    L[..., i, j] = np.where(keep, v / g, 0.0)
                L[..., j, j] = np.where(keep, g, 0.0)
        S = np.einsum("...pk,...pk->...p", Bo, Bo)
        Kd = np.einsum("...pp->...p", Sb)
        rel = np.where(Kd > 0, S / Kd, 1.0)
        amb |= np.any((rel >= lo) & (rel <= hi), axis=-1)
    amb[0] = False
    return amb


def factor_errors(Ag, Bg, Ao, Bo, n_theta, skip_ambiguous=True):
    """Errors of device factors against oracle factors, measured on what the factors do
    to the chain's law rather than entry by entry (the entries of A are ill-determined
    along near-null directions of J(a,a), and those of B = chol(S) when S is nearly
    singular):
      dA = max |(A_dev - A_orc) J(a,a)^{1/2}|_pq / sd_b,p   (conditional-mean map on a
                                                             unit-variance input)
      dS = max |B_dev B_dev^T - B_orc B_orc^T|_pq / (sd_b,p sd_b,q)   (conditional covariance)
    with sd_b = sqrt(diag J(b,b)); rows with sd_b = 0 must be zero on both sides.  Steps
    next to a threshold (threshold_ambiguous) are left out when skip_ambiguous is set.
    Returns (max dA, max dS, number of steps left out)."""
    Sa, Sb = chain_covariances(Ao, Bo, n_theta)
    sd_b = np.sqrt(np.clip(np.einsum("...pp->...p", Sb), 0, None))
    R = _sqrtm_psd(Sa)
    eA = np.abs(np.einsum("...pk,...kq->...pq", Ag - Ao, R))
    eS = np.abs(np.einsum("...pk,...qk->...pq", Bg, Bg) - np.einsum("...pk,...qk->...pq", Bo, Bo))
    live = sd_b > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        dA = np.where(live[..., None], eA / sd_b[..., :, None], np.abs(Ag - Ao))
        den = sd_b[..., :, None] * sd_b[..., None, :]
        dS = np.where(den > 0, eS / den, eS)
    amb = threshold_ambiguous(Ao, Bo, n_theta) if skip_ambiguous else np.zeros(Ao.shape[:2], bool)
    keep = ~amb
    dA = dA[keep]
    dS = dS[keep]
    return (float(np.nanmax(dA)) if dA.size else 0.0, float(np.nanmax(dS)) if dS.size else 0.0,
            int(amb.sum()))


def threshold_decisions(Ag, Bg, Ao, Bo, n_theta):
    """For the steps next to a threshold (threshold_ambiguous), whether the device and the
    oracle took the same keep/drop decisions: a dropped pivot of J(a,a) leaves its column of
    A exactly zero, and a conditional variance at or below the threshold leaves its diagonal
    entry of B exactly zero, so the decision of a step is the pattern of zero columns of A
    and zero diagonal entries of B.  Returns (number of ambiguous steps, list of (set, mode)
    where the patterns differ)."""
    amb = threshold_ambiguous(Ao, Bo, n_theta)
    M = Ao.shape[-1]

    def pattern(A, B):
        cols = np.all(A == 0.0, axis=-2)                     # [sets, modes, M]
        diag = np.einsum("...pp->...p", B) == 0.0             # [sets, modes, M]
        return np.concatenate([cols, diag], axis=-1)

    pg, po = pattern(Ag, Bg), pattern(Ao, Bo)
    differ = np.any(pg != po, axis=-1) & amb
    del M
    return int(amb.sum()), [tuple(int(x) for x in ij) for ij in np.argwhere(differ)]
