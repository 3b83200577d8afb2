"""GPU tests of the Green's-function setup of Sec. 3 (SMF_GREEN): at order 1 C_l =
1/(kappa + l(l+1)) for every l, J^m from eq. (Jmatrix_efficient) with P^m_lambda of complex
(or, for kappa <= 1/4, real) degree; at order 2 two distinct kappa through the partial
fractions of eq. (C_ell_efficient), in the basis (g, U g).  The device factors against the oracle's Green's-function
setup by their action on the chain's law, the fields against the oracle's chains and DFT on
the same Philox normals (FP64 1e-10, FP32 1e-4 per field, with element-wise maxima), and the
property the band-limited setup lacks: the device chain reproduces the closed-form J^m between
rings far apart (no Markov defect).  Also on a ring plan (HEALPix rings): the factors of the
modes up to the plan's ell_max on the HEALPix latitudes, then the synthesis at each ring's
pixels."""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import factor_errors, log, max_rel_err, rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (n_theta, n_phi, kappa): the 64 x 128 grid of the order-1 workload with its kappa = 8^2,
# the 1024 x 2048 grid with kappa = 20^2, an odd grid with a real degree, a finer one
CASES = [(64, 128, 64.0), (1024, 2048, 400.0), (33, 64, 0.2), (256, 512, 2500.0)]


def _plan(n, nphi, kappa, precision, **kw):
    from paper_1709_10314_amd import Plan

    return Plan(1, n, nphi, 0, kappa=[kappa], precision=precision, green=True, **kw)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-k{c[2]:g}")
def test_green_factors_match_oracle(case):
    n, nphi, kappa = case
    p = _plan(n, nphi, kappa, "fp64")
    assert p.m_top == nphi // 2 - 1
    Ag, Bg = p.factors()
    p.close()
    Ao, Bo = oracle.setup_green(kappa, n, nphi)
    dA, dS, amb = factor_errors(Ag, Bg, Ao, Bo, n, skip_ambiguous=False)
    log(f"green {n}x{nphi} kappa {kappa}: factor errors dA {dA:.2e} dS {dS:.2e}")
    assert dA <= 1e-9 and dS <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES[:3], ids=lambda c: f"{c[0]}x{c[1]}-k{c[2]:g}")
def test_green_fields_match_oracle(case, precision):
    n, nphi, kappa = case
    count = 3 if n <= 256 else 1
    p = _plan(n, nphi, kappa, precision)
    T = p.sample(11, count).double().cpu().numpy()
    torch.cuda.synchronize()
    p.close()
    Ao, Bo = oracle.setup_green(kappa, n, nphi)
    if n <= 256:
        To, _ = oracle.sample(1, n, nphi, Ao, Bo, 11, count)
        rows = slice(None)
    else:   # the rings around the equator: every mode from the factor sets near the start
        sets = 17
        s = oracle.start_ring(n)
        g = oracle.sample_modes(1, n, Ao[:sets], Bo[:sets], 11, count, sets=sets)
        r0, r1 = s - sets + 2, s + sets
        To = oracle.dft(g, nphi, r0, r1)
        rows = slice(r0, r1)
    bar = 1e-10 if precision == "fp64" else 1e-4
    for f in range(count):
        e, emax = rel_rms(T[f][rows], To[f]), max_rel_err(T[f][rows], To[f])
        log(f"green {n}x{nphi} kappa {kappa} {precision} field {f}: rel RMS {e:.2e}, max {emax:.2e}")
        assert e <= bar and emax <= 10 * bar


@pytest.mark.parametrize("case", [CASES[0], CASES[3]], ids=lambda c: f"{c[0]}x{c[1]}-k{c[2]:g}")
def test_green_chain_has_no_markov_defect(case):
    """Covariances propagated through the device's FP64 factors along the northern walk
    reproduce the closed-form J^m(z_r, z_s) between every ring r and the start ring s."""
    n, nphi, kappa = case
    p = _plan(n, nphi, kappa, "fp64")
    A, B = p.factors()
    p.close()
    _, z = oracle.grid(n)
    s = oracle.start_ring(n)
    worst = 0.0
    for m in (0, 1, 5, nphi // 8):
        var, cross, prev = {s: B[0, m, 0, 0] ** 2}, {s: B[0, m, 0, 0] ** 2}, s
        for j in range(2, A.shape[0]):
            r = s - j + 1
            var[r] = A[j, m, 0, 0] ** 2 * var[prev] + B[j, m, 0, 0] ** 2
            cross[r] = A[j, m, 0, 0] * cross[prev]
            prev = r
        for r in list(var)[::5]:
            Jrs = oracle.jblock_green(m, kappa, z[r], z[s])
            sd = math.sqrt(var[r] * var[s])
            worst = max(worst, abs(cross[r] - Jrs) / sd)
    log(f"green {n}x{nphi}: largest chain-vs-closed-form cross covariance error {worst:.2e} of the sd product")
    assert worst <= 1e-10


def test_green_rejects_what_it_does_not_cover():
    from paper_1709_10314_amd import smf

    for kw in (dict(order=3, kappa=[64.0, 9.0, 4.0]), dict(order=1, kappa=[64.0, 9.0]), dict(order=1, kappa=[-1.0]),
               dict(order=1, kappa=[1e-6]), dict(order=1, kappa=[2e4])):
        rc, _ = smf.smf_setup(kw["order"], 16, 32, 15, kappa=kw["kappa"], flags=smf.SMF_FP64 | smf.SMF_GREEN)
        assert rc == smf.SMF_EINVAL, kw
    rc, _ = smf.smf_setup(1, 16, 32, 15, c_ell=np.ones(16), flags=smf.SMF_FP64 | smf.SMF_GREEN)
    assert rc == smf.SMF_EINVAL
    rc, _ = smf.smf_setup(1, 16, 32, 15, kappa=[4.0], flags=smf.SMF_FP64 | smf.SMF_GREEN | smf.SMF_UBASIS)
    assert rc == smf.SMF_EINVAL


# ---------------------------------------------------------------- order 2, two distinct kappa
CASES2 = [(64, 128, [100.0, 900.0]), (256, 512, [64.0, 2500.0]), (33, 64, [0.2, 3.0])]


def _plan2(n, nphi, kappas, precision):
    from paper_1709_10314_amd import Plan

    return Plan(2, n, nphi, 0, kappa=kappas, precision=precision, green=True)


@pytest.mark.parametrize("case", CASES2, ids=lambda c: f"{c[0]}x{c[1]}-k{c[2][0]:g}-{c[2][1]:g}")
def test_green2_factors_and_fields_match_oracle(case):
    n, nphi, kappas = case
    p = _plan2(n, nphi, kappas, "fp64")
    Ag, Bg = p.factors()
    T = p.sample(13, 2).double().cpu().numpy()
    torch.cuda.synchronize()
    p.close()
    Ao, Bo = oracle.setup_green2(kappas, n, nphi)
    dA, dS, amb = factor_errors(Ag, Bg, Ao, Bo, n)
    # The factor bar is the conditioning of the problem, measured on the oracle alone: its own
    # factors move this far when each kappa moves by one unit in the last place.  The partial
    # fractions of eq. (C_ell_efficient) (weights 1/(kappa_2 - kappa_1)) and the Schur
    # complement of Alg. 1 (conditional variances of the value a small power of the ring
    # spacing below the marginal ones) both amplify FP64 rounding.
    Ap, Bp = oracle.setup_green2([kappas[0] * (1 + 2.0 ** -52), kappas[1] * (1 - 2.0 ** -52)], n, nphi)
    sA, sS, _ = factor_errors(Ap, Bp, Ao, Bo, n)
    To, _ = oracle.sample(2, n, nphi, Ao, Bo, 13, 2)
    e = max(rel_rms(T[f], To[f]) for f in range(2))
    emax = max(max_rel_err(T[f], To[f]) for f in range(2))
    log(f"green2 {n}x{nphi} kappa {kappas}: factors dA {dA:.2e} dS {dS:.2e} ({amb} steps next to a threshold), "
        f"oracle's one-ulp sensitivity dA {sA:.2e} dS {sS:.2e}; fields rel RMS {e:.2e}, max {emax:.2e}")
    assert dA <= 10 * sA + 1e-13 and dS <= 10 * sS + 1e-13
    assert e <= 1e-10 and emax <= 1e-9
    p32 = _plan2(n, nphi, kappas, "fp32")
    T32 = p32.sample(13, 2).double().cpu().numpy()
    torch.cuda.synchronize()
    p32.close()
    e32 = max(rel_rms(T32[f], To[f]) for f in range(2))
    log(f"  fp32 fields rel RMS {e32:.2e}")
    assert e32 <= 1e-4


@pytest.mark.parametrize("case", CASES2[:2], ids=lambda c: f"{c[0]}x{c[1]}")
def test_green2_chain_has_no_markov_defect(case):
    """All four components of J^m between the start ring and rings far from it, from the
    device's FP64 factors, against the closed form, to 1e-10 of the standard deviations."""
    n, nphi, kappas = case
    p = _plan2(n, nphi, kappas, "fp64")
    A, B = p.factors()
    p.close()
    _, z = oracle.grid(n)
    s = oracle.start_ring(n)
    worst = 0.0
    for m in (0, 1, 7, nphi // 8):
        S = B[0, m] @ B[0, m].T
        V, X = S.copy(), S.copy()
        for j in range(2, A.shape[0]):
            r = s - j + 1
            V = A[j, m] @ V @ A[j, m].T + B[j, m] @ B[j, m].T
            X = A[j, m] @ X
            if (s - r) % 7 == 0:
                J = oracle.jblock_green2(m, kappas, z[r], z[s])
                sd = np.sqrt(np.outer(np.diag(V), np.diag(S)))
                worst = max(worst, float(np.max(np.abs(X - J) / sd)))
    log(f"green2 {n}x{nphi}: largest cross-covariance error {worst:.2e} of the sd products")
    assert worst <= 1e-10


def test_green2_rejects_repeated_or_missing_kappa():
    from paper_1709_10314_amd import smf

    for kw in (dict(order=2, kappa=[50.0, 50.0]), dict(order=2, kappa=[50.0]), dict(order=3, kappa=[1.0, 2.0, 3.0]),
               dict(order=2, kappa=[50.0, 0.0]), dict(order=2, kappa=[50.0, 50.0 * (1 + 1e-4)])):
        rc, _ = smf.smf_setup(kw["order"], 16, 32, 15, kappa=kw["kappa"], flags=smf.SMF_FP64 | smf.SMF_GREEN)
        assert rc == smf.SMF_EINVAL, kw


# ---------------------------------------------------------------- order 2, complex-conjugate kappa pair
# (alpha, beta): kappa = alpha +- i beta; (0, sqrt 10) is the Sec. 5 spectrum 1/((l(l+1))^2 + 10)
CASES2C = [(64, 128, (0.0, float(np.sqrt(10.0)))), (256, 512, (0.0, float(np.sqrt(10.0)))), (33, 64, (2.0, 5.0)),
           (128, 256, (-3.0, 1.5))]


def _plan2c(n, nphi, ab, precision):
    from paper_1709_10314_amd import Plan

    return Plan(2, n, nphi, 0, kappa=list(ab), precision=precision, green=True, kappa_pair=True)


@pytest.mark.parametrize("case", CASES2C, ids=lambda c: f"{c[0]}x{c[1]}-a{c[2][0]:g}-b{c[2][1]:.3g}")
def test_green_pair_factors_and_fields_match_oracle(case):
    """The GPU setup for the conjugate pair against the oracle's: factors by their action on the
    chain's law within ten times the oracle's own movement when alpha and beta move by one unit
    in the last place (of beta's size), FP64 fields to 1e-10 relative RMS (1e-9 element-wise),
    FP32 fields to 1e-4."""
    n, nphi, (alpha, beta) = case
    p = _plan2c(n, nphi, (alpha, beta), "fp64")
    Ag, Bg = p.factors()
    T = p.sample(17, 2).double().cpu().numpy()
    torch.cuda.synchronize()
    p.close()
    Ao, Bo = oracle.setup_green2c(alpha, beta, n, nphi)
    dA, dS, amb = factor_errors(Ag, Bg, Ao, Bo, n)
    ulp = 2.0 ** -52 * max(abs(alpha), beta)
    Ap, Bp = oracle.setup_green2c(alpha + ulp, beta - ulp, n, nphi)
    sA, sS, _ = factor_errors(Ap, Bp, Ao, Bo, n)
    To, _ = oracle.sample(2, n, nphi, Ao, Bo, 17, 2)
    e = max(rel_rms(T[f], To[f]) for f in range(2))
    emax = max(max_rel_err(T[f], To[f]) for f in range(2))
    log(f"green pair {n}x{nphi} alpha {alpha} beta {beta:.4g}: factors dA {dA:.2e} dS {dS:.2e} ({amb} near a "
        f"threshold), oracle's one-ulp sensitivity dA {sA:.2e} dS {sS:.2e}; fields rel RMS {e:.2e}, max {emax:.2e}")
    assert dA <= 10 * sA + 1e-13 and dS <= 10 * sS + 1e-13
    assert e <= 1e-10 and emax <= 1e-9
    p32 = _plan2c(n, nphi, (alpha, beta), "fp32")
    T32 = p32.sample(17, 2).double().cpu().numpy()
    torch.cuda.synchronize()
    p32.close()
    e32 = max(rel_rms(T32[f], To[f]) for f in range(2))
    log(f"  fp32 fields rel RMS {e32:.2e}")
    assert e32 <= 1e-4


@pytest.mark.parametrize("case", CASES2C[:2], ids=lambda c: f"{c[0]}x{c[1]}")
def test_green_pair_chain_has_no_markov_defect(case):
    """All four components of J^m between the start ring and rings far from it, from the device's
    FP64 factors for the Sec. 5 spectrum, against the closed form, to 1e-10 of the standard
    deviations: the band-limit defect the Legendre-sum setup leaves for this spectrum is gone."""
    n, nphi, (alpha, beta) = case
    p = _plan2c(n, nphi, (alpha, beta), "fp64")
    A, B = p.factors()
    p.close()
    _, z = oracle.grid(n)
    s = oracle.start_ring(n)
    worst = 0.0
    for m in (0, 1, 7, nphi // 8):
        S = B[0, m] @ B[0, m].T
        V, X = S.copy(), S.copy()
        for j in range(2, A.shape[0]):
            r = s - j + 1
            V = A[j, m] @ V @ A[j, m].T + B[j, m] @ B[j, m].T
            X = A[j, m] @ X
            if (s - r) % 7 == 0:
                J = oracle.jblock_green2c(m, alpha, beta, z[r], z[s])
                sd = np.sqrt(np.outer(np.diag(V), np.diag(S)))
                worst = max(worst, float(np.max(np.abs(X - J) / sd)))
    log(f"green pair {n}x{nphi}: largest cross-covariance error {worst:.2e} of the sd products")
    assert worst <= 1e-10


def test_green_pair_rejects_what_it_does_not_cover():
    from paper_1709_10314_amd import smf

    F = smf.SMF_FP64 | smf.SMF_GREEN | smf.SMF_KAPPA_PAIR
    for order, kap, flags in ((2, [0.0, 0.0], F), (2, [0.0, -1.0], F), (1, [3.0], F), (2, [float("nan"), 1.0], F),
                              (2, [0.0, 3.0], smf.SMF_FP64 | smf.SMF_KAPPA_PAIR), (2, [9.99e3, 999.0], F),
                              (2, [-100.0, 1.0], F), (2, [0.0, 2000.0], F)):
        rc, _ = smf.smf_setup(order, 16, 32, 15, kappa=kap, flags=flags)
        assert rc == smf.SMF_EINVAL, (order, kap, flags)


# ---------------------------------------------------------------- ring plans (HEALPix rings)
def _green_factors(order, kap, n, nphi, modes, z):
    if order == 1:
        return oracle.setup_green(kap[0], n, nphi, modes=modes, z=z)
    return oracle.setup_green2c(kap[0], kap[1], n, nphi, modes=modes, z=z)


@pytest.mark.parametrize("case", [(1, (400.0,)), (2, (0.0, float(np.sqrt(10.0))))], ids=["order1-k400", "pair-i-sqrt10"])
def test_green_on_healpix_rings_matches_oracle(case):
    """SMF_GREEN on a ring plan (HEALPix nside 16, 63 rings of 4 to 64 pixels, ell_max 47):
    the chains run the Sec. 3 factors of the modes up to ell_max on the HEALPix latitudes (for
    the pair, the Sec. 5 spectrum), and each ring is synthesised at its own pixels; against the
    oracle's factors on the same latitudes, its chains and its ring sum on the same normals.
    FP64 within 1e-10 relative RMS, or 20 times the oracle's own movement when the northern
    latitudes move by a relative 2.2e-16 if that is larger (HEALPix's uneven polar rings);
    FP32 within 1e-4."""
    from paper_1709_10314_amd import RingPlan, workloads

    order, kap = case
    z, n_ring, phi0 = workloads.healpix_rings(16)
    n, lmax, seed, count = len(z), 47, 7, 2
    md = np.arange(lmax + 1)
    for precision in ("fp64", "fp32"):
        plan = RingPlan(order, n_ring, phi0, lmax, kappa=list(kap), precision=precision, z=z, green=True,
                        kappa_pair=order == 2)
        assert plan.m_top == lmax
        A, B = _green_factors(order, kap, n, plan.n_phi, md, z)
        To = oracle.dft_rings(oracle.sample_modes(order, n, A, B, seed, count), n_ring, phi0)
        T = plan.sample_rings(seed, count).double().cpu().numpy()
        torch.cuda.synchronize()
        plan.close()
        bar = 1e-4
        if precision == "fp64":
            h = (n + 1) // 2
            sens = 0.0
            for d in range(2):
                zn = z[:h] * (1 + 2.2e-16 * np.random.default_rng(d).standard_normal(h))
                zp = np.concatenate([zn, -zn[: n - h][::-1]])
                Ap, Bp = _green_factors(order, kap, n, plan.n_phi, md, zp)
                Tp = oracle.dft_rings(oracle.sample_modes(order, n, Ap, Bp, seed, count), n_ring, phi0)
                sens = max(sens, max(rel_rms(Tp[f], To[f]) for f in range(count)))
            bar = max(1e-10, 20 * sens)
            log(f"green on HEALPix {case} fp64: oracle's latitude sensitivity {sens:.2e}, bar {bar:.2e}")
        e = max(rel_rms(T[f], To[f]) for f in range(count))
        emax = max(max_rel_err(T[f], To[f]) for f in range(count))
        log(f"green on HEALPix {case} {precision}: fields rel RMS {e:.2e}, max {emax:.2e}")
        assert e <= bar


# ---------------------------------------------------------------- the southern walk's own factor sets
@pytest.mark.parametrize("grid", [(64, 128), (33, 64)], ids=["64x128", "33x64"])
@pytest.mark.parametrize("case", [(1, (400.0,)), (2, (100.0, 900.0)), (2, (0.0, float(np.sqrt(10.0))))],
                         ids=["order1", "order2-real", "pair"])
def test_green_southern_sets_equal_the_mirror(grid, case):
    """SMF_NO_MIRROR with SMF_GREEN: the southern walk's factor sets computed on their own (the
    Green's-function kernels' southern form) against the mirrored northern sets on a symmetric
    grid; the fields must agree to rounding (the mirrored path is the one pinned to the oracle)."""
    from paper_1709_10314_amd import Plan

    n, nphi = grid
    order, kap = case
    pair = order == 2 and kap[0] == 0.0
    for precision, bar in (("fp64", 1e-12), ("fp32", 1e-6)):
        plans = [Plan(order, n, nphi, 0, kappa=list(kap), precision=precision, green=True, kappa_pair=pair,
                      mirror=mirror) for mirror in (True, False)]
        T = [p.sample(5, 2).double().cpu().numpy() for p in plans]
        torch.cuda.synchronize()
        for p in plans:
            p.close()
        e = max(rel_rms(T[1][f], T[0][f]) for f in range(2))
        log(f"green {case} {grid} {precision}: own southern sets against the mirror, rel RMS {e:.2e}")
        assert e <= bar


# ---------------------------------------------------------------- the corners of the accepted kappa domain
@pytest.mark.parametrize("case", [(1, (1e-5,)), (1, (1e4,)), (2, (-50.0, 0.1)), (2, (-50.0, 1000.0)),
                                  (2, (9000.0, 1000.0)), ("real2", (1e-5, 1e4)), ("real2", (100.0, 100.0 * (1 + 2e-3)))],
                         ids=lambda c: f"{c[0]}-{c[1]}")
def test_green_domain_corners_match_oracle(case):
    """The Green's-function setups at the edges of the kappa domain they accept (|kappa| from 1e-5
    to 1e4; for the pair alpha >= -50, beta <= 1000; two real roots a relative distance of at
    least 1e-3 apart), 64 x 128, FP64: fields against the oracle's factors and chains on the same
    normals within 1e-10 relative RMS, or ten times the oracle's own movement when kappa moves by
    one unit in the last place if that is larger."""
    from paper_1709_10314_amd import Plan

    kind, kap = case
    order = 1 if kind == 1 else 2
    n, nphi, seed, count = 64, 128, 23, 2

    def oracle_factors(k):
        if kind == 1:
            return oracle.setup_green(k[0], n, nphi)
        return oracle.setup_green2(list(k), n, nphi) if kind == "real2" else oracle.setup_green2c(k[0], k[1], n, nphi)

    p = Plan(order, n, nphi, 0, kappa=list(kap), precision="fp64", green=True, kappa_pair=kind == 2)
    T = p.sample(seed, count).double().cpu().numpy()
    torch.cuda.synchronize()
    p.close()
    Ao, Bo = oracle_factors(kap)
    To, _ = oracle.sample(order, n, nphi, Ao, Bo, seed, count)
    # one unit in the last place, into the domain
    kp = tuple(k * (1 + 2.0 ** -52) if abs(k) <= 1e-5 else k * (1 - 2.0 ** -52) for k in kap)
    Ap, Bp = oracle_factors(kp)
    Tp, _ = oracle.sample(order, n, nphi, Ap, Bp, seed, count)   # (for two real roots both move inward)
    sens = max(rel_rms(Tp[f], To[f]) for f in range(count))
    e = max(rel_rms(T[f], To[f]) for f in range(count))
    bar = max(1e-10, 10 * sens)
    log(f"green domain corner {case}: fields rel RMS {e:.2e}, oracle's one-ulp sensitivity {sens:.2e}, bar {bar:.2e}")
    assert np.isfinite(T).all() and e <= bar


@pytest.mark.parametrize("case", [(1, (400.0,)), (2, (0.0, float(np.sqrt(10.0))))], ids=["order1", "pair"])
def test_green_on_an_explicit_grid_matches_oracle(case):
    """SMF_GREEN on an explicit grid (smf_setup_grid): 48 Gauss-Legendre latitudes, 128 longitudes,
    every mode up to n_phi / 2 - 1; FP64 fields against the oracle's factors on the same latitudes
    within 1e-10 relative RMS (or ten times the oracle's own movement when the northern latitudes
    move by a relative 2.2e-16, if larger), FP32 within 1e-4."""
    from paper_1709_10314_amd import Plan

    order, kap = case
    n, nphi, seed, count = 48, 128, 31, 2
    z = np.sort(np.polynomial.legendre.leggauss(n)[0])[::-1].copy()
    z[n // 2:] = -z[: n // 2][::-1]   # symmetric to the bit

    def factors(zz):
        if order == 1:
            return oracle.setup_green(kap[0], n, nphi, z=zz)
        return oracle.setup_green2c(kap[0], kap[1], n, nphi, z=zz)

    A, B = factors(z)
    To, _ = oracle.sample(order, n, nphi, A, B, seed, count)
    zp = z.copy()
    zp[: n // 2] *= 1 + 2.2e-16 * np.random.default_rng(0).standard_normal(n // 2)
    zp[n // 2:] = -zp[: n // 2][::-1]
    Ap, Bp = factors(zp)
    Tp, _ = oracle.sample(order, n, nphi, Ap, Bp, seed, count)
    sens = max(rel_rms(Tp[f], To[f]) for f in range(count))
    for precision, bar in (("fp64", max(1e-10, 10 * sens)), ("fp32", 1e-4)):
        p = Plan(order, n, nphi, 0, kappa=list(kap), precision=precision, z=z, green=True, kappa_pair=order == 2)
        T = p.sample(seed, count).double().cpu().numpy()
        torch.cuda.synchronize()
        p.close()
        e = max(rel_rms(T[f], To[f]) for f in range(count))
        log(f"green on Gauss-Legendre latitudes {case} {precision}: fields rel RMS {e:.2e} (oracle's sensitivity {sens:.2e})")
        assert e <= bar
