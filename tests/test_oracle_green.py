"""Pins of the oracle's Green's-function setup (Sec. 3): at order 1 C_l = 1/(kappa + l(l+1))
for every l, kappa = -lambda(lambda+1), J^m from eq. (Jmatrix_efficient) with P^m_lambda of
eq. (Legendre_hypergeometric) and no sum over l; at order 2 the partial fractions of eq.
(C_ell_efficient) over two distinct real kappa or a complex-conjugate pair (the Sec. 5
spectrum's kappa = +- i sqrt 10) in the basis (g, U g).  Each check compares with something other
than the oracle's own formula: mpmath's Gauss hypergeometric function and Ferrers function
of complex degree, scipy's hypergeometric function for real degree (0 < kappa <= 1/4), the
value at z = 1, the Wronskian of DLMF 14.2.3 as the paper quotes it, the associated Legendre
equation, the brute-force Legendre sums of Lemma 2.1 as ell_max grows, and the Markov
property that the Green's function gives the chain exactly (no band-limit defect)."""
import math

import numpy as np
import pytest
import scipy.special as ss

mp = pytest.importorskip("mpmath")

KAPPAS = [0.2, 3.0, 64.0, 400.0]


def _lam(kappa):
    return (-1 + mp.sqrt(1 - 4 * mp.mpf(kappa))) / 2


@pytest.mark.parametrize("kappa", KAPPAS)
def test_G_matches_mpmath_hypergeometric(orc, kappa):
    """G_m(x) = 2F1(-lambda, lambda+1; 1+m; (1-x)/2) on both sides of the equator and near
    the south pole (the continuation about t = 1 and the recurrence in m), to 1e-13."""
    mp.mp.dps = 25
    lam = _lam(kappa)
    a, b = -lam, lam + 1
    for m in (0, 1, 2, 7, 40, 300):
        for x in (0.95, 0.3, 0.0, -0.02, -0.3, -0.7, -0.97):
            ref = float(mp.re(mp.hyp2f1(a, b, 1 + m, (1 - mp.mpf(x)) / 2)))
            assert orc.green_G(m, kappa, x) == pytest.approx(ref, rel=1e-13), (m, x)


@pytest.mark.parametrize("kappa", [64.0, 400.0])
def test_P_matches_mpmath_ferrers_function(orc, kappa):
    """P^m_lambda of eq. (Legendre_hypergeometric) is the Ferrers function of the first kind
    (mpmath legenp, type 2) of complex degree lambda = -1/2 + i tau."""
    mp.mp.dps = 25
    lam = _lam(kappa)
    for m in (0, 1, 3, 12):
        for x in (0.8, 0.2, -0.1, -0.6):
            ref = float(mp.re(mp.legenp(lam, m, x, type=2)))
            assert orc.green_P(m, kappa, x) == pytest.approx(ref, rel=1e-12), (m, x)


def test_real_degree_matches_scipy_near_the_pole(orc):
    """0 < kappa <= 1/4 gives a real degree lambda in (-1/2, 0]; then scipy's hyp2f1 (real
    parameters) pins G_m up to the ring next to the south pole of a 1024-ring grid, where
    the oracle takes the logarithmic continuation about t = 1."""
    kappa = 0.2
    lam = (-1 + math.sqrt(1 - 4 * kappa)) / 2
    for m in (0, 1, 2, 5, 30):
        for x in (-0.9, -0.999, -math.cos(math.pi / 2048)):
            t = (1 - x) / 2
            ref = ss.hyp2f1(-lam, lam + 1, 1 + m, t)
            assert orc.green_G(m, kappa, x) == pytest.approx(ref, rel=1e-9), (m, x)


@pytest.mark.parametrize("kappa", KAPPAS)
def test_P_at_the_north_pole_is_delta(orc, kappa):
    """P^m_lambda(1) = delta_m0 (stated after eq. (Legendre_hypergeometric))."""
    for m in range(6):
        assert orc.green_P(m, kappa, 1.0, 0.0) == (1.0 if m == 0 else 0.0)


@pytest.mark.parametrize("kappa", [3.0, 64.0])
@pytest.mark.parametrize("m", [0, 1, 4])
def test_wronskian(orc, kappa, m):
    """W{P^m(z), P^m(-z)} = 2 (1 - z^2)^-1 / (Gamma(lambda+1-m) Gamma(-lambda-m)) (the
    Wronskian the paper quotes from DLMF 14.2.3), by central differences (h = 1e-5)."""
    mp.mp.dps = 25
    lam = _lam(kappa)
    gam = complex(mp.gamma(lam + 1 - m) * mp.gamma(-lam - m)).real
    h = 1e-5
    for z in (-0.5, 0.1, 0.6):
        P = orc.green_P(m, kappa, z)
        dP = (orc.green_P(m, kappa, z + h) - orc.green_P(m, kappa, z - h)) / (2 * h)
        Q = orc.green_P(m, kappa, -z)
        dQ = (orc.green_P(m, kappa, -z - h) - orc.green_P(m, kappa, -z + h)) / (2 * h)    # d/dz P(-z)
        W = P * dQ - dP * Q
        want = 2.0 / (1 - z * z) / gam
        assert W == pytest.approx(want, rel=1e-7), (z, W, want)


@pytest.mark.parametrize("kappa", [3.0, 64.0])
def test_associated_legendre_equation(orc, kappa):
    """(1-z^2) P'' - 2 z P' + (lambda(lambda+1) - m^2/(1-z^2)) P = 0 with lambda(lambda+1) =
    -kappa, by central differences."""
    h = 1e-4
    for m in (0, 2, 5):
        for z in (-0.7, -0.2, 0.4):
            f = [orc.green_P(m, kappa, z + k * h) for k in (-1, 0, 1)]
            d1 = (f[2] - f[0]) / (2 * h)
            d2 = (f[2] - 2 * f[1] + f[0]) / (h * h)
            res = (1 - z * z) * d2 - 2 * z * d1 + (-kappa - m * m / (1 - z * z)) * f[1]
            scale = abs(kappa * f[1]) + abs(m * m / (1 - z * z) * f[1])
            assert abs(res) < 1e-5 * scale, (m, z, res, scale)


@pytest.mark.parametrize("kappa", [64.0, 400.0])
def test_legendre_sums_converge_to_the_green_function(orc, kappa):
    """The brute-force sums of Lemma 2.1 approach J^m of eq. (Jmatrix_efficient) as ell_max
    grows (errors relative to sqrt(J(z1,z1) J(z2,z2))): off the diagonal to 5e-5 at
    ell_max = 16000 with the error falling at every step; on the diagonal (where the sum converges like 1/ell_max) with ell_max times
    the error settling to a constant."""
    for m in (0, 3, 20):
        for z1, z2 in ((0.2, 0.35), (-0.3, 0.1), (0.5, 0.5)):
            Jg = orc.jblock_green(m, kappa, z1, z2)
            sd = math.sqrt(orc.jblock_green(m, kappa, z1, z1) * orc.jblock_green(m, kappa, z2, z2))
            errs = []
            for lmax in (2000, 8000, 16000):
                C = orc.spectrum([kappa], lmax)
                errs.append(abs(orc.jblock_z(1, m, lmax, C, z1, z2)[0, 0] - Jg) / sd)
            if z1 != z2:
                assert errs[2] < errs[1] < errs[0] and errs[-1] < 5e-5, (m, z1, z2, errs)
            else:
                assert errs[2] < errs[1] < errs[0], errs
                assert 16000 * errs[2] == pytest.approx(8000 * errs[1], rel=0.1), errs


@pytest.mark.parametrize("kappa,n", [(64.0, 64), (400.0, 256), (0.2, 33)])
def test_green_chain_is_exactly_markov(orc, kappa, n):
    """With the whole spectrum the mode is an exact Gauss-Markov chain: covariances
    propagated through the factors reproduce J^m of eq. (Jmatrix_efficient) between any two
    rings of a hemisphere, not only neighbours, to 1e-12 (a band-limited spectrum leaves a
    defect of percents there), and at every ring of both hemispheres."""
    nphi = 2 * n if n % 2 == 0 else 2 * (n + 1)
    A, B = orc.setup_green(kappa, n, nphi)
    _, z = orc.grid(n)
    s = orc.start_ring(n)
    even = n % 2 == 0
    for m in (0, 1, 7, n // 2):
        # northern walk: rings s, (s+1 for even n), s-1, ..., 0 with their factor sets
        cov = {s: B[0, m, 0, 0] ** 2}
        cross = {s: cov[s]}                                  # Cov(x_r, x_s)
        prev = s
        for j in range(2 if even else 1, A.shape[0]):
            r = s - j + 1 if even else s - j
            a_, b_ = A[j, m, 0, 0], B[j, m, 0, 0]
            cov[r] = a_ * a_ * cov[prev] + b_ * b_
            cross[r] = a_ * cross[prev]
            prev = r
        for r in list(cov)[::7]:
            Jrr = orc.jblock_green(m, kappa, z[r], z[r])
            Jrs = orc.jblock_green(m, kappa, z[r], z[s])
            assert cov[r] == pytest.approx(Jrr, rel=1e-12, abs=1e-300), (m, r)
            assert cross[r] == pytest.approx(Jrs, rel=1e-10, abs=1e-14 * math.sqrt(Jrr * cov[s])), (m, r)


# ---------------------------------------------------------------- order 2, two distinct kappa
K2 = [[100.0, 900.0], [3.0, 64.0]]


@pytest.mark.parametrize("kappas", K2)
def test_order2_green_matches_u_basis_sums(orc, kappas):
    """Order 2 in the basis (g, U g): the partial fractions of eq. (C_ell_efficient) and
    eq. (Jmatrix_efficient) with P^m and P^{m+1} against the brute-force sums of
    U^p L_lm U^q L_lm (the U basis of eq. (Jmatrix_more_efficient), Legendre sums with
    C_l = 1/((kappa_1 + l(l+1))(kappa_2 + l(l+1)))) as ell_max grows; errors relative to the
    standard deviations of the two components; off the diagonal to 1e-6 at ell_max = 16000,
    every component falling with ell_max."""
    for m in (0, 2, 11):
        for z1, z2 in ((0.2, 0.35), (-0.3, 0.1), (0.6, 0.1), (0.45, 0.45)):
            Jg = orc.jblock_green2(m, kappas, z1, z2)
            sd = np.sqrt(np.outer(np.diag(orc.jblock_green2(m, kappas, z1, z1)),
                                  np.diag(orc.jblock_green2(m, kappas, z2, z2))))
            errs = []
            for lmax in (2000, 8000, 16000):
                C = orc.spectrum(kappas, lmax)
                errs.append(np.abs(orc.jblock_u(m, lmax, C, z1, z2) - Jg) / sd)
            worst = [float(e.max()) for e in errs]
            assert worst[2] < worst[1] < worst[0], (m, z1, z2, worst)
            if z1 != z2:
                assert worst[2] < 1e-6, (m, z1, z2, worst)
            else:   # the U U component converges like 1 / ell_max on the diagonal
                assert worst[2] < 5e-3 and 16000 * worst[2] == pytest.approx(8000 * worst[1], rel=0.15), worst


@pytest.mark.parametrize("kappas,n", [([100.0, 900.0], 64), ([3.0, 64.0], 33)])
def test_order2_green_chain_is_exactly_markov(orc, kappas, n):
    """The order-2 chain on the Green's-function factors reproduces the closed-form J^m
    (all four components) between the start ring and rings far from it, to 1e-10 of the
    standard deviations."""
    nphi = 2 * n if n % 2 == 0 else 2 * (n + 1)
    A, B = orc.setup_green2(kappas, n, nphi)
    _, z = orc.grid(n)
    s = orc.start_ring(n)
    even = n % 2 == 0
    for m in (0, 1, 5, n // 2):
        S = B[0, m] @ B[0, m].T
        V, X, prev = S.copy(), S.copy(), s
        for j in range(2 if even else 1, A.shape[0]):
            r = s - j + 1 if even else s - j
            V = A[j, m] @ V @ A[j, m].T + B[j, m] @ B[j, m].T
            X = A[j, m] @ X
            if (s - r) % 5 == 0:
                J = orc.jblock_green2(m, kappas, z[r], z[s])
                sd = np.sqrt(np.outer(np.diag(V), np.diag(S)))
                assert np.max(np.abs(X - J) / sd) < 1e-10, (m, r)
                Jrr = orc.jblock_green2(m, kappas, z[r], z[r])
                assert np.max(np.abs(V - Jrr) / np.sqrt(np.outer(np.diag(V), np.diag(V)))) < 1e-10, (m, r)


# ---------------------------------------------------------------- order 2, complex-conjugate kappa
# The Sec. 5 spectrum C_l = 1/((l(l+1))^2 + 10): kappa = +- i sqrt(10).
BETA = np.sqrt(10.0)


def test_complex_kappa_G_matches_mpmath(orc):
    """G_m of complex degree for complex kappa = i sqrt(10) against mpmath's hyp2f1, on both
    sides of the equator and next to the south pole (the continuation about t = 1)."""
    mpmath = pytest.importorskip("mpmath")
    kappa = 1j * BETA
    lam = -0.5 + np.sqrt(0.25 - kappa + 0j)
    worst = 0.0
    for m in (0, 1, 5, 30, 120):
        for x in (0.9, 0.3, -0.2, -0.7, -0.97, -0.9995):
            g = orc.greenc_G(m, kappa, x)
            ref = complex(mpmath.hyp2f1(-lam, lam + 1, 1 + m, (1 - x) / 2))
            worst = max(worst, abs(g - ref) / abs(ref))
    assert worst < 1e-13, worst


def test_complex_kappa_with_real_part_G_matches_mpmath(orc):
    """G_m for kappa = alpha + i beta with alpha != 0 (the pairs 2 +- 5i and -3 +- 1.5i, the
    second with Re kappa < 0) against mpmath's hyp2f1, on both sides of the equator."""
    mpmath = pytest.importorskip("mpmath")
    worst = 0.0
    for kappa in (2.0 + 5.0j, -3.0 + 1.5j, -3.0 - 1.5j):
        lam = -0.5 + np.sqrt(0.25 - kappa + 0j)
        for m in (0, 1, 6, 40):
            for x in (0.8, 0.1, -0.5, -0.95, -0.999):
                g = orc.greenc_G(m, kappa, x)
                ref = complex(mpmath.hyp2f1(-lam, lam + 1, 1 + m, (1 - x) / 2))
                worst = max(worst, abs(g - ref) / abs(ref))
    assert worst < 1e-12, worst


def test_complex_kappa_G_reduces_to_the_real_case(orc):
    """With a real kappa the complex-kappa path gives the real path's G_m (both degrees of the
    real case: complex lambda for kappa > 1/4, real lambda below)."""
    for kappa in (0.2, 40.0):
        for m in (0, 3, 17):
            for x in (0.5, -0.4, -0.99):
                assert orc.greenc_G(m, kappa, x) == pytest.approx(orc.green_G(m, kappa, x), rel=1e-13)


def test_conjugate_pair_green_matches_u_basis_sums(orc):
    """Order 2 for kappa = +- i sqrt(10) (the partial fractions with b_1 = i / (2 sqrt 10) = -b_2,
    whose two terms are complex conjugates) against the brute-force U-basis Legendre sums of
    the same spectrum (C_l from the complex factors) as ell_max grows: off the diagonal to 1e-6
    of the standard deviations at ell_max = 16000, the U U entry on it at the 1/ell_max rate."""
    for m in (0, 2, 11):
        for z1, z2 in ((0.2, 0.35), (-0.3, 0.1), (0.6, 0.1), (0.45, 0.45)):
            Jg = orc.jblock_green2c(m, 0.0, BETA, z1, z2)
            sd = np.sqrt(np.outer(np.diag(orc.jblock_green2c(m, 0.0, BETA, z1, z1)),
                                  np.diag(orc.jblock_green2c(m, 0.0, BETA, z2, z2))))
            worst = []
            for lmax in (2000, 8000, 16000):
                C = orc.spectrum_complex([1j * BETA, -1j * BETA], lmax)
                worst.append(float((np.abs(orc.jblock_u(m, lmax, C, z1, z2) - Jg) / sd).max()))
            assert worst[2] < worst[1] < worst[0], (m, z1, z2, worst)
            if z1 != z2:
                assert worst[2] < 1e-6, (m, z1, z2, worst)
            else:
                assert worst[2] < 1e-3 and 16000 * worst[2] == pytest.approx(8000 * worst[1], rel=0.15), worst


@pytest.mark.parametrize("alpha,beta", [(2.0, 5.0), (-3.0, 1.5)])
def test_conjugate_pair_with_real_part_matches_u_basis_sums(orc, alpha, beta):
    """The same check for pairs alpha +- i beta with alpha != 0, C_l = 1/((l(l+1) + alpha)^2 +
    beta^2), off the diagonal: the sums approach the closed form as ell_max grows."""
    for m in (0, 3):
        for z1, z2 in ((-0.3, 0.1), (0.6, 0.1)):
            Jg = orc.jblock_green2c(m, alpha, beta, z1, z2)
            sd = np.sqrt(np.outer(np.diag(orc.jblock_green2c(m, alpha, beta, z1, z1)),
                                  np.diag(orc.jblock_green2c(m, alpha, beta, z2, z2))))
            worst = []
            for lmax in (2000, 8000):
                C = orc.spectrum_complex([alpha + 1j * beta, alpha - 1j * beta], lmax)
                worst.append(float((np.abs(orc.jblock_u(m, lmax, C, z1, z2) - Jg) / sd).max()))
            assert worst[1] < worst[0] and worst[1] < 1e-6, (m, z1, z2, worst)


@pytest.mark.parametrize("n", [64, 33])
def test_conjugate_pair_chain_is_exactly_markov(orc, n):
    """The order-2 chain on the conjugate-pair factors reproduces the closed-form J^m (all four
    components) between the start ring and rings far from it, to 1e-10 of the standard
    deviations."""
    nphi = 2 * n if n % 2 == 0 else 2 * (n + 1)
    A, B = orc.setup_green2c(0.0, BETA, n, nphi)
    _, z = orc.grid(n)
    s = orc.start_ring(n)
    even = n % 2 == 0
    for m in (0, 1, 5, n // 2):
        S = B[0, m] @ B[0, m].T
        V, X = S.copy(), S.copy()
        for j in range(2 if even else 1, A.shape[0]):
            r = s - j + 1 if even else s - j
            V = A[j, m] @ V @ A[j, m].T + B[j, m] @ B[j, m].T
            X = A[j, m] @ X
            if (s - r) % 5 == 0:
                J = orc.jblock_green2c(m, 0.0, BETA, z[r], z[s])
                sd = np.sqrt(np.outer(np.diag(V), np.diag(S)))
                assert np.max(np.abs(X - J) / sd) < 1e-10, (m, r)
                Jrr = orc.jblock_green2c(m, 0.0, BETA, z[r], z[r])
                assert np.max(np.abs(V - Jrr) / np.sqrt(np.outer(np.diag(V), np.diag(V)))) < 1e-10, (m, r)


def test_green_setups_hold_kappa_to_their_fp64_range(orc):
    """G_m and sin(pi lambda) grow like exp(pi sqrt|kappa|) in FP64: the Green's-function setups
    take |kappa| <= 1e4 (there the values stay below about 1e137; near 1e5 the closed-form J^m
    of nearby rings already underflows to zero, which a setup must not pass on silently)."""
    assert orc.jblock_green(0, 1e5, 0.1, 0.2) == 0.0   # the failure the bound keeps out
    A, B = orc.setup_green(1e4, 8, 16)
    assert np.isfinite(A).all() and np.isfinite(B).all()
    for bad in (lambda: orc.setup_green(2e4, 8, 16), lambda: orc.setup_green2([100.0, 2e4], 8, 16),
                lambda: orc.setup_green2c(9.99e3, 999.0, 8, 16)):
        with pytest.raises(ValueError):
            bad()
    A, B = orc.setup_green2c(5e3, 1e3, 8, 16)
    assert np.isfinite(A).all() and np.isfinite(B).all()


def test_conjugate_pair_domain_keeps_G_accurate(orc):
    """The pair's series of G_m cancels where its terms n^2 + n + kappa turn sign (alpha well
    below zero: at alpha = -1000 the sum is wrong by orders of magnitude) or rotate (beta in the
    thousands), so the setup takes alpha >= -50 and beta <= 1000 (|kappa| <= 1e4): at the corners
    of that domain G_m is within 1e-10 of mpmath's hyp2f1 at 40 digits; outside it is rejected."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    worst = 0.0
    for kappa in (complex(-50.0, 0.1), complex(-50.0, 1000.0), complex(0.0, 1000.0), complex(9000.0, 1000.0)):
        lam = -mpmath.mpf(1) / 2 + mpmath.sqrt(mpmath.mpf(1) / 4 - mpmath.mpc(kappa))
        for m in (0, 1, 10):
            for x in (0.9, 0.0, -0.5, -0.9, -0.999):
                ref = complex(mpmath.hyp2f1(-lam, lam + 1, 1 + m, (1 - mpmath.mpf(x)) / 2))
                worst = max(worst, abs(orc.greenc_G(m, kappa, x) - ref) / abs(ref))
    mpmath.mp.dps = 15
    assert worst < 1e-10, worst
    for alpha, beta in ((-100.0, 1.0), (0.0, 2000.0), (9e3, 5e3), (0.0, 1e-6)):
        with pytest.raises(ValueError):
            orc.setup_green2c(alpha, beta, 8, 16)


def test_green_setups_hold_small_kappa_off(orc):
    """As kappa -> 0 (lambda -> 0) the continuation about t = 1 loses digits (against mpmath at
    40 digits: 5e-11 at kappa = 1e-7, 6e-10 at 1e-8): the setups take |kappa| >= 1e-5, where G_m
    is within 1e-11, real or complex."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    worst = 0.0
    for kappa in (1e-5, 1e-5j, complex(1e-5, 1e-5)):
        lam = -mpmath.mpf(1) / 2 + mpmath.sqrt(mpmath.mpf(1) / 4 - mpmath.mpc(kappa))
        for m in (0, 1, 100):
            for x in (0.9, -0.5, -0.999, -0.99999):
                ref = complex(mpmath.hyp2f1(-lam, lam + 1, 1 + m, (1 - mpmath.mpf(x)) / 2))
                worst = max(worst, abs(orc.greenc_G(m, complex(kappa), x) - ref) / abs(ref))
    mpmath.mp.dps = 15
    assert worst < 1e-11, worst
    orc.setup_green(1e-5, 8, 16)
    for bad in (lambda: orc.setup_green(1e-6, 8, 16), lambda: orc.setup_green2([1e-6, 1.0], 8, 16)):
        with pytest.raises(ValueError):
            bad()


def test_green2_holds_its_real_roots_apart(orc):
    """Two real roots lose about log10(kappa / |kappa_2 - kappa_1|) digits to the partial
    fractions (against the U-basis Legendre sums at ell_max = 16000: 3e-7 of the standard
    deviations, the sums' own truncation, at a relative distance of 1e-8, 3.6e-3 at 1e-12; a
    64 x 128 field moves by 5e-11 when kappa moves by one unit in the last place at 1e-3, by
    1e-9 at 1e-4): the setup takes a relative distance of at least 1e-3, which keeps FP64 fields
    reproducible to 1e-10; a conjugate pair has no such loss (its second term is the conjugate of
    the first, not subtracted from it)."""
    orc.setup_green2([100.0, 100.0 * (1 + 2e-3)], 8, 16)
    with pytest.raises(ValueError):
        orc.setup_green2([100.0, 100.0 * (1 + 1e-4)], 8, 16)
    k = [100.0, 100.0 + 1e-10]
    Jg = orc.jblock_green2(3, k, 0.2, 0.35)
    Ju = orc.jblock_u(3, 16000, orc.spectrum(k, 16000), 0.2, 0.35)
    sd = np.sqrt(np.outer(np.diag(orc.jblock_green2(3, k, 0.2, 0.2)), np.diag(orc.jblock_green2(3, k, 0.35, 0.35))))
    assert np.max(np.abs(Jg - Ju) / sd) > 1e-4   # the loss the bound keeps out
