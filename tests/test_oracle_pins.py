"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Every check compares the oracle with something other than itself: scipy's associated
Legendre functions, closed forms (sectoral values, Unsold's theorem, the addition
theorem for the field covariance C_T of Sec. 5), two independent Philox headers,
numpy's inverse real FFT, finite differences, and exact covariance propagation.
"""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.special as ss

TORCH_INC = None
try:
    import torch.utils.cpp_extension as _ce

    TORCH_INC = _ce.include_paths()[0]
except Exception:  # pragma: no cover
    pass


# --------------------------------------------------------------------------- Legendre
@pytest.mark.parametrize("m", [0, 1, 2, 5, 17, 40])
@pytest.mark.parametrize("theta", [0.05, 0.7, 1.5707963, 2.3, 3.1])
def test_legendre_matches_scipy(orc, m, theta):
    """L_lm = P_lm-normalised / sqrt(2 pi) (scipy's norm=True has 1/2 where we have 1/(4 pi));
    derivative d/dz from scipy's diff_n=1.  Products remove the Condon-Shortley sign."""
    lmax = 60
    L, dL = orc.legendre(m, lmax, theta)
    z = math.cos(theta)
    ref = np.array([ss.assoc_legendre_p(l, m, z, norm=True, diff_n=1) for l in range(m, lmax + 1)])
    ref = ref / math.sqrt(2 * math.pi)
    scale = np.max(np.abs(ref[:, 0]))
    np.testing.assert_allclose(np.abs(L), np.abs(ref[:, 0]), rtol=1e-12, atol=1e-14 * max(scale, 1e-300))
    # sign of the derivative relative to the value (Condon-Shortley cancels in L * dL)
    d_scale = np.max(np.abs(ref[:, 0] * ref[:, 1]))
    np.testing.assert_allclose(L * dL, ref[:, 0] * ref[:, 1], rtol=1e-11, atol=1e-13 * d_scale)
    np.testing.assert_allclose(np.abs(dL), np.abs(ref[:, 1]), rtol=1e-11, atol=1e-13 * np.max(np.abs(ref[:, 1])))


def test_legendre_closed_forms(orc):
    th = 0.9
    z, s = math.cos(th), math.sin(th)
    L, dL = orc.legendre(0, 1, th)
    assert abs(L[0] - 1 / math.sqrt(4 * math.pi)) < 1e-16
    assert abs(L[1] - math.sqrt(3 / (4 * math.pi)) * z) < 1e-16
    assert abs(dL[0]) < 1e-16
    assert abs(dL[1] - math.sqrt(3 / (4 * math.pi))) < 1e-15
    L, dL = orc.legendre(1, 1, th)
    assert abs(L[0] - math.sqrt(3 / (8 * math.pi)) * s) < 1e-16
    # d/dz sqrt(1-z^2) = -z / sqrt(1-z^2)
    assert abs(dL[0] + math.sqrt(3 / (8 * math.pi)) * z / s) < 1e-15


@pytest.mark.parametrize("m,theta", [(300, 0.2), (2000, 0.5), (4000, 0.05), (8000, 1.2)])
def test_sectoral_extended_exponent(orc, m, theta):
    """L_mm = sqrt((2m+1)/(4 pi) (2m)!/(4^m (m!)^2)) sin^m(theta), compared in log space;
    these seeds are far below the FP64 range for most of the cases."""
    lmax = m + 3
    L, _ = orc.legendre(m, lmax, theta)
    # (2m)!/(4^m (m!)^2) = prod_k (1 - 1/(2k)); summed with fsum for an accurate log
    log_ref = 0.5 * (math.log((2 * m + 1) / (4 * math.pi))
                     + math.fsum(math.log1p(-0.5 / k) for k in range(1, m + 1))) \
        + m * math.log(math.sin(theta))
    if log_ref > math.log(1e-300):
        assert abs(math.log(abs(L[0])) - log_ref) < 1e-12 * max(1.0, abs(log_ref))
    else:
        assert L[0] == 0.0 or abs(L[0]) < 1e-300


@pytest.mark.parametrize("lmax,z", [(4095, 0.818), (2047, 0.999), (8191, -0.31)])
def test_unsold_at_high_degree(orc, lmax, z):
    """Unsold: L_l0^2 + 2 sum_{m>=1} L_lm^2 = (2l+1)/(4 pi); with the derivative
    identity sum_m w_m L_lm dL_lm/dz = 0 (derivative of a constant)."""
    th = math.acos(z)
    tot = 0.0
    dtot = 0.0
    dabs = 0.0
    for m in range(lmax + 1):
        L, dL = orc.legendre(m, lmax, th)
        w = 1.0 if m == 0 else 2.0
        tot += w * L[-1] ** 2
        dtot += w * L[-1] * dL[-1]
        dabs += w * abs(L[-1] * dL[-1])
    assert abs(tot / ((2 * lmax + 1) / (4 * math.pi)) - 1) < 1e-12
    assert abs(dtot) < 1e-11 * dabs


# --------------------------------------------------------------------------- J blocks
def _addition_target(C, cosg):
    """C_T = sum_l (2l+1)/(4 pi) C_l P_l(cos gamma)  (Sec. 5)."""
    l = np.arange(len(C))
    return np.sum((2 * l + 1) / (4 * np.pi) * C * ss.eval_legendre(l, cosg))


@pytest.mark.parametrize("kappa,lmax", [(64.0, 63), (400.0, 120), (3.0, 40)])
def test_jblock_addition_theorem(orc, kappa, lmax):
    """sum_m w_m J^m_00(a,b) cos(m dphi) = C_T(gamma) for every ring pair and dphi."""
    C = orc.spectrum([kappa], lmax)
    ths = [0.1, 0.8, 1.4, 2.2, 3.0]
    for ta in ths:
        for tb in ths:
            Js = np.array([orc.jblock(1, m, lmax, C, ta, tb)[0, 0] for m in range(lmax + 1)])
            for dphi in [0.0, 0.4, math.pi]:
                w = np.where(np.arange(lmax + 1) == 0, 1.0, 2.0)
                val = np.sum(w * Js * np.cos(np.arange(lmax + 1) * dphi))
                cosg = math.cos(ta) * math.cos(tb) + math.sin(ta) * math.sin(tb) * math.cos(dphi)
                ref = _addition_target(C, cosg)
                assert abs(val - ref) < 1e-12 * _addition_target(C, 1.0)


@pytest.mark.parametrize("m", [0, 3, 11])
def test_jblock_derivatives_finite_difference(orc, m):
    """J_01 = d/dz2 J_00, J_10 = d/dz1 J_00, J_11 = d2/dz1dz2 J_00 (Sec. 2 cross covariances),
    by central differences in z (theta = acos z)."""
    lmax = 50
    C = orc.spectrum([30.0, 30.0], lmax)
    z1, z2, h = 0.31, -0.47, 1e-5

    def J00(a, b):
        return orc.jblock(1, m, lmax, C, math.acos(a), math.acos(b))[0, 0]

    J = orc.jblock(2, m, lmax, C, math.acos(z1), math.acos(z2))
    d2 = (J00(z1, z2 + h) - J00(z1, z2 - h)) / (2 * h)
    d1 = (J00(z1 + h, z2) - J00(z1 - h, z2)) / (2 * h)
    d12 = (J00(z1 + h, z2 + h) - J00(z1 + h, z2 - h) - J00(z1 - h, z2 + h) + J00(z1 - h, z2 - h)) / (4 * h * h)
    sc = abs(J[0, 0]) + abs(J[1, 1]) ** 0.5 * abs(J[0, 0]) ** 0.5 + 1e-30
    assert abs(J[0, 1] - d2) < 1e-6 * sc
    assert abs(J[1, 0] - d1) < 1e-6 * sc
    assert abs(J[1, 1] - d12) < 1e-4 * abs(J[1, 1]) + 1e-6 * sc


@pytest.mark.parametrize("m", [0, 2, 7, 30])
@pytest.mark.parametrize("z", [-0.8, -0.1, 0.3, 0.9])
def test_legendre_higher_derivatives_finite_difference(orc, m, z):
    """Second and third z-derivatives (from the associated Legendre equation) against
    central differences of the next lower derivative, l = m..m+25."""
    lmax, h = m + 25, 1e-5
    F = orc.legendre_derivs(m, lmax, z, 4)
    Fp = orc.legendre_derivs(m, lmax, z + h, 4)
    Fm = orc.legendre_derivs(m, lmax, z - h, 4)
    for k in (1, 2):
        fd = (Fp[k] - Fm[k]) / (2 * h)
        scale = np.max(np.abs(F[k + 1])) + 1e-300
        assert np.max(np.abs(fd - F[k + 1])) < 1e-6 * scale, (k + 1, m, z)


@pytest.mark.parametrize("m", [0, 3, 11])
def test_jblock_order4_derivatives_finite_difference(orc, m):
    """J^m_pq of order 4 are the mixed z-derivatives of J_00: J_{p+1,q} = d/dz1 J_pq and
    J_{p,q+1} = d/dz2 J_pq, by central differences."""
    lmax = 40
    C = orc.spectrum([30.0] * 4, lmax)
    z1, z2, h = 0.31, -0.47, 1e-5
    J = orc.jblock_z(4, m, lmax, C, z1, z2)
    J1p, J1m = orc.jblock_z(4, m, lmax, C, z1 + h, z2), orc.jblock_z(4, m, lmax, C, z1 - h, z2)
    J2p, J2m = orc.jblock_z(4, m, lmax, C, z1, z2 + h), orc.jblock_z(4, m, lmax, C, z1, z2 - h)
    d1 = (J1p - J1m) / (2 * h)
    d2 = (J2p - J2m) / (2 * h)
    for p in range(4):
        for q in range(4):
            sc = math.sqrt(abs(orc.jblock_z(4, m, lmax, C, z1, z1)[p, p]) * abs(orc.jblock_z(4, m, lmax, C, z2, z2)[q, q]))
            if p < 3:
                assert abs(d1[p, q] - J[p + 1, q]) < 1e-6 * sc * (1 + m), (p, q)
            if q < 3:
                assert abs(d2[p, q] - J[p, q + 1]) < 1e-6 * sc * (1 + m), (p, q)


def test_spectrum_rejects_nonpositive(orc):
    with pytest.raises(ValueError):
        orc.spectrum([0.0], 5)          # C_0 = 1/0
    with pytest.raises(ValueError):
        orc.spectrum([-2.0], 5)         # C_1 = 1/0
    C = orc.spectrum([2500.0, 2500.0], 3)
    assert C[0] == 1.0 / 2500.0 ** 2
    with pytest.raises(ValueError):
        orc.spectrum_complex([1j], 3)    # a lone complex kappa gives complex C_l


# eq. (Cl) worked out by hand, l(l+1) = 0, 2, 6, 12, 20, 30, 42, 56, ... :
#   kappa = (64)        C_l = 1/(64 + l(l+1))
#   kappa = (3, 11)     C_l = 1/((3 + l(l+1)) (11 + l(l+1)))    (distinct, Sec. 3)
#   kappa = (2500)^2    C_l = 1/(2500 + l(l+1))^2               (repeated, the bench spectrum)
# Each value is a ratio of integers written out below; l^2 in place of l(l+1), or a sum
# in place of the product over kappa_i, changes every entry with l >= 1.
_CL_HAND = [
    ([64.0], {0: 1 / 64, 1: 1 / 66, 2: 1 / 70, 3: 1 / 76, 7: 1 / 120, 10: 1 / 174}),
    ([3.0, 11.0], {0: 1 / 33, 1: 1 / 65, 2: 1 / 153, 4: 1 / 713, 6: 1 / (45 * 53)}),
    ([2500.0, 2500.0], {1: 1 / 2502 ** 2, 5: 1 / 2530 ** 2, 7: 1 / 2556 ** 2, 49: 1 / 4950 ** 2}),
]


@pytest.mark.parametrize("kappa,want", _CL_HAND)
def test_spectrum_worked_values(orc, kappa, want):
    C = orc.spectrum(kappa, max(want))
    for ell, c in want.items():
        assert C[ell] == pytest.approx(c, rel=1e-15), (kappa, ell)


def test_sample_spectrum_of_sec5_is_the_complex_pair(orc):
    """eq. (sample_spec), C_l = (10 + l^2 (l+1)^2)^-1, is eq. (Cl) with the complex pair
    kappa = +-i sqrt(10) (Sec. 3's example with a^2 = 10): hand values 1/10, 1/14, 1/46,
    1/154, 1/410, 1/910 at l = 0..5, and the explicit spectrum the convergence experiment
    passes as c_ell agrees at every l."""
    C = orc.spectrum_complex([1j * math.sqrt(10.0), -1j * math.sqrt(10.0)], 4095)
    for ell, c in {0: 1 / 10, 1: 1 / 14, 2: 1 / 46, 3: 1 / 154, 4: 1 / 410, 5: 1 / 910}.items():
        assert C[ell] == pytest.approx(c, rel=1e-14), ell
    ell = np.arange(4096, dtype=np.float64)
    explicit = 1.0 / (10.0 + ell ** 2 * (ell + 1.0) ** 2)   # the convergence test's c_ell
    np.testing.assert_allclose(C, explicit, rtol=1e-14)


# --------------------------------------------------------------------------- factors
def _propagate_check(orc, order, kappa, n, lmax, n_phi, z=None):
    """Covariance propagation through the factors (Sigma_b = A Sigma_a A^T + B B^T, cross
    A Sigma_a) reproduces J(b,b) and J(b,a) at every step of both hemispheres, the south
    computed from J at the true southern rings (mirror via D A D, D B D).  z: an explicit
    ring grid (default the ring centres)."""
    C = orc.spectrum([kappa] * order, lmax)
    A, B = orc.setup(order, C, n, n_phi, z=z)
    s = orc.start_ring(n)
    D = np.diag([(-1.0) ** p for p in range(order)])
    even = n % 2 == 0
    worst = 0.0

    def jb(m, i1, i2):
        if z is None:
            return orc.jblock_ring(order, m, lmax, C, n, i1, i2)
        return orc.jblock_z(order, m, lmax, C, z[i1], z[i2])

    def cmp(S, K):
        d = np.sqrt(np.maximum(np.diag(K), 0))
        sc = np.outer(d, d)
        mask = sc > 1e-280
        return np.max(np.abs(S - K)[mask] / sc[mask]) if mask.any() else 0.0

    for m in range(A.shape[1]):
        Ks = jb(m, s, s)
        Ss = B[0, m] @ B[0, m].T
        worst = max(worst, cmp(Ss, Ks))
        # north
        Sig, a = Ss, s
        for j in range(2 if even else 1, A.shape[0]):
            b = s - j + 1 if even else s - j
            Kbb = jb(m, b, b)
            Kba = jb(m, b, a)
            cross = A[j, m] @ Sig
            Sig = A[j, m] @ Sig @ A[j, m].T + B[j, m] @ B[j, m].T
            worst = max(worst, cmp(Sig, Kbb), cmp(cross, Kba))
            a = b
        # south
        Sig, a = Ss, s
        j0 = 1
        if even:
            b = s + 1
            Kbb = jb(m, b, b)
            Kba = jb(m, b, a)
            cross = A[1, m] @ Sig
            Sig = A[1, m] @ Sig @ A[1, m].T + B[1, m] @ B[1, m].T
            worst = max(worst, cmp(Sig, Kbb), cmp(cross, Kba))
            a, j0 = b, 2
        for j in range(j0, A.shape[0]):
            b = a + 1
            Am, Bm = D @ A[j, m] @ D, D @ B[j, m] @ D
            Kbb = jb(m, b, b)
            Kba = jb(m, b, a)
            cross = Am @ Sig
            Sig = Am @ Sig @ Am.T + Bm @ Bm.T
            worst = max(worst, cmp(Sig, Kbb), cmp(cross, Kba))
            a = b
    return worst


@pytest.mark.parametrize("order,kappa,n,lmax,n_phi", [
    (1, 64.0, 64, 63, 128),       # the 64 x 128 plain form
    (1, 400.0, 33, 40, 82),       # odd ring count: equator start
    (2, 2500.0, 16, 15, 32),
    (2, 100.0, 8, 63, 128),
    (2, 9.0, 21, 30, 62),
])
def test_factors_reproduce_ring_covariances(orc, order, kappa, n, lmax, n_phi):
    assert _propagate_check(orc, order, kappa, n, lmax, n_phi) < 1e-11


@pytest.mark.parametrize("order,kappa,n,lmax,n_phi", [
    (3, 30.0, 16, 15, 32),
    (3, 400.0, 33, 40, 82),
    (4, 100.0, 16, 15, 32),
    (4, 900.0, 21, 30, 62),
    (3, 2500.0, 64, 63, 128),
])
def test_factors_reproduce_ring_covariances_high_order(orc, order, kappa, n, lmax, n_phi):
    """Orders 3 and 4: the same propagation check.  The value and its first M-1
    derivatives are strongly correlated, so more pivots fall under the 1e-12 threshold;
    dropping one costs up to sqrt(1e-12) = 1e-6 of a correlation per step, which bounds
    the reproduction at 1e-4 over a walk."""
    assert _propagate_check(orc, order, kappa, n, lmax, n_phi) < 1e-4


def test_factors_lower_triangular_positive(orc):
    C = orc.spectrum([50.0, 50.0], 40)
    A, B = orc.setup(2, C, 24, 82)
    assert np.all(B[..., 0, 1] == 0.0)
    assert np.all(B[..., 0, 0] >= 0.0) and np.all(B[..., 1, 1] >= 0.0)
    assert np.all(A[0] == 0.0)


def test_mirror_factors_match_direct_southern_step(orc):
    """The paper's symmetry remark: the factors of the mirrored (southern) step equal
    D A D and D B D, here against factors built from J at the southern rings."""
    order, lmax, n = 2, 30, 12
    C = orc.spectrum([20.0, 20.0], lmax)
    A, B = orc.setup(order, C, n, 62)
    th, _ = orc.grid(n)
    s = orc.start_ring(n)
    D = np.diag([1.0, -1.0])
    for m in [0, 1, 7, 20]:
        for j in range(2, A.shape[0]):
            a_n, b_n = s - j + 2, s - j + 1
            a_s, b_s = n - 1 - a_n, n - 1 - b_n
            Kaa = orc.jblock_ring(order, m, lmax, C, n, a_s, a_s)
            Kbb = orc.jblock_ring(order, m, lmax, C, n, b_s, b_s)
            Kba = orc.jblock_ring(order, m, lmax, C, n, b_s, a_s)
            As, Bs = _step(orc, order, Kaa, Kbb, Kba)
            # the two sides round their thetas differently, and near-deterministic steps
            # make S = J(b,b) - A J(a,b) a strong cancellation, so errors are measured in
            # units of the marginal standard deviations: dA_pq sqrt(J_aa,qq / J_bb,pp)
            # and dB_pq / sqrt(J_bb,pp)
            sb = np.sqrt(np.diag(Kbb))
            sa = np.sqrt(np.diag(Kaa))
            dA = np.abs(As - D @ A[j, m] @ D) * sa[None, :] / sb[:, None]
            dB = np.abs(Bs - D @ B[j, m] @ D) / sb[:, None]
            # B = chol(S) with S known to ~eps J(b,b): |dB| <~ eps / sqrt(S~), and the
            # threshold keeps S~ > 1e-12, so 1e-8 bounds it with room
            assert np.max(dA) < 1e-10 and np.max(dB) < 1e-8, (m, j, dA, dB)


def _step(orc, order, Kaa, Kbb, Kba):
    import ctypes
    lib = orc._load()
    pd = ctypes.POINTER(ctypes.c_double)
    A = np.zeros(order * order)
    B = np.zeros(order * order)
    Kaa, Kbb, Kba = (np.ascontiguousarray(x, dtype=np.float64).reshape(-1) for x in (Kaa, Kbb, Kba))
    lib.orc_step_factors.argtypes = [ctypes.c_int, pd, pd, pd, pd, pd]
    lib.orc_step_factors(order, Kaa.ctypes.data_as(pd), Kbb.ctypes.data_as(pd), Kba.ctypes.data_as(pd),
                         A.ctypes.data_as(pd), B.ctypes.data_as(pd))
    return A.reshape(order, order), B.reshape(order, order)


def test_step_factors_threshold_cases(orc):
    """Degenerate blocks: an identical next ring (S = 0 -> B = 0, A = identity), a zero
    block (everything zero), and a rank-1 2x2 block (second pivot dropped)."""
    K = np.array([[2.0, 0.3], [0.3, 0.5]])
    A, B = _step(orc, 2, K, K, K)
    np.testing.assert_allclose(A, np.eye(2), atol=1e-14)
    assert np.all(B == 0.0)
    Z = np.zeros((2, 2))
    A, B = _step(orc, 2, Z, Z, Z)
    assert np.all(A == 0.0) and np.all(B == 0.0)
    v = np.array([1.0, 3.0])
    R1 = np.outer(v, v)                          # x_1 = 3 x_0 exactly
    Kbb = np.array([[4.0, 1.0], [1.0, 9.0]])
    Kba = np.array([[0.5, 1.5], [0.1, 0.3]])
    A, B = _step(orc, 2, R1, Kbb, Kba)
    assert np.all(np.isfinite(A)) and np.all(np.isfinite(B))
    assert A[0, 1] == 0.0 and A[1, 1] == 0.0     # dropped pivot: no weight on x_1
    np.testing.assert_allclose(A[:, 0], Kba[:, 0] / R1[0, 0], rtol=1e-14)


# --------------------------------------------------------------------------- Philox
_PHILOX_TORCH = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int i = 1; i + 5 < argc + 0; i += 6) {
    uint64_t key = strtoull(argv[i], 0, 0) | (strtoull(argv[i + 1], 0, 0) << 32);
    uint64_t off = strtoull(argv[i + 2], 0, 0) | (strtoull(argv[i + 3], 0, 0) << 32);
    uint64_t sub = strtoull(argv[i + 4], 0, 0) | (strtoull(argv[i + 5], 0, 0) << 32);
    at::philox_engine e(key, sub, off);
    for (int w = 0; w < 4; ++w) printf("%u ", (unsigned)e());
    printf("\n");
  }
}
"""

_PHILOX_ROCRAND = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
struct Eng : rocrand_device::philox4x32_10_engine {
  Eng() : philox4x32_10_engine(0, 0, 0) {}
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main(int argc, char** argv) {
  Eng e;
  for (int i = 1; i + 5 < argc + 0; i += 6) {
    uint2 k = {(unsigned)strtoul(argv[i], 0, 0), (unsigned)strtoul(argv[i + 1], 0, 0)};
    uint4 c = {(unsigned)strtoul(argv[i + 2], 0, 0), (unsigned)strtoul(argv[i + 3], 0, 0),
               (unsigned)strtoul(argv[i + 4], 0, 0), (unsigned)strtoul(argv[i + 5], 0, 0)};
    uint4 o = e.run(c, k);
    printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
  }
}
"""


def _philox_cases():
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 0, 0, 5, 1, 0), (16, 0, 1023, 4095, 1, 0)]
    for _ in range(40):
        cases.append(tuple(int(x) for x in rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)))
    return cases


def _run_header_program(src, extra):
    with tempfile.TemporaryDirectory() as d:
        cpp, exe = os.path.join(d, "p.cpp"), os.path.join(d, "p")
        open(cpp, "w").write(src)
        subprocess.run(["g++", "-O1", "-std=c++17"] + extra + [cpp, "-o", exe], check=True,
                       capture_output=True)
        args = [str(x) for c in _philox_cases() for x in c]
        out = subprocess.run([exe] + args, check=True, capture_output=True, text=True).stdout
    return [[int(x) for x in line.split()] for line in out.strip().splitlines()]


@pytest.mark.skipif(TORCH_INC is None, reason="torch headers not found")
def test_philox_matches_torch_header(orc):
    ref = _run_header_program(_PHILOX_TORCH, ["-I" + TORCH_INC])
    for (k0, k1, c0, c1, c2, c3), r in zip(_philox_cases(), ref):
        assert orc.philox([c0, c1, c2, c3], [k0, k1]) == r


@pytest.mark.skipif(not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"),
                    reason="rocRAND headers not found")
def test_philox_matches_rocrand_header(orc):
    ref = _run_header_program(_PHILOX_ROCRAND, ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"])
    for (k0, k1, c0, c1, c2, c3), r in zip(_philox_cases(), ref):
        assert orc.philox([c0, c1, c2, c3], [k0, k1]) == r


def test_normals_distribution(orc):
    """Box-Muller output is N(0,1): moments and a KS test over 40k draws."""
    from scipy import stats

    xs = np.array([orc.normal(3, m, p, r, 2, q) for m in range(10) for p in range(2)
                   for r in range(1000) for q in range(2)])
    assert abs(xs.mean()) < 5 / math.sqrt(len(xs))
    assert abs(xs.var() - 1) < 5 * math.sqrt(2 / len(xs))
    assert stats.kstest(xs, "norm").pvalue > 1e-4


def test_normal_counter_map(orc):
    """xi_q of ring r uses word (r M + q) mod 4 of block floor((r M + q)/4); the pair
    (0,1) is (R cos, R sin) of one Box-Muller draw, so the two share a radius."""
    key = 0x1_0000_0005
    for order in (1, 2):
        for r in range(8):
            for q in range(order):
                idx = r * order + q
                w = orc.philox([idx // 4, 9, 1, 0], [key & 0xFFFFFFFF, key >> 32])
                pair = (idx % 4) // 2
                u0 = (w[2 * pair] + 0.5) * 2.0 ** -32
                u1 = (w[2 * pair + 1] + 0.5) * 2.0 ** -32
                rad = math.sqrt(-2 * math.log(u0))
                ang = 2 * math.pi * u1
                ref = rad * (math.cos(ang) if idx % 2 == 0 else math.sin(ang))
                assert abs(orc.normal(key, 9, 1, r, order, q) - ref) < 1e-12
    # the two normals of a pair lie on one circle of radius R
    a, b = orc.normal(5, 2, 0, 6, 2, 0), orc.normal(5, 2, 0, 6, 2, 1)
    w = orc.philox([3, 2, 0, 0], [5, 0])
    assert abs(a * a + b * b - (-2 * math.log((w[0] + 0.5) * 2.0 ** -32))) < 1e-12


# --------------------------------------------------------------------------- DFT, sampling
@pytest.mark.parametrize("n_phi,lmax", [(8, 3), (128, 63), (64, 20), (256, 200)])
def test_dft_matches_numpy_irfft(orc, n_phi, lmax):
    rng = np.random.default_rng(n_phi)
    mt = orc.m_top(lmax, n_phi)
    g = rng.normal(size=(2, 3, mt + 1)) + 1j * rng.normal(size=(2, 3, mt + 1))
    g[..., 0] = g[..., 0].real
    T = orc.dft(g, n_phi)
    X = np.zeros((2, 3, n_phi // 2 + 1), complex)
    X[..., : mt + 1] = g
    ref = np.fft.irfft(X, n=n_phi, axis=-1) * n_phi
    np.testing.assert_allclose(T, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))


def test_constant_field_when_lmax_zero(orc):
    """ell_max = 0: T is one N(0, C_0/(4 pi)) constant over the sphere; the chain has
    A = 1 and B = 0 (degenerate S, threshold path)."""
    for order in (1, 2):
        C = orc.spectrum([3.0] * order, 0)
        n, nphi = 10, 16
        A, B = orc.setup(order, C, n, nphi)
        T, g = orc.sample(order, n, nphi, A, B, 11, 2)
        for f in range(2):
            xi = orc.normal(11 + f, 0, 0, orc.start_ring(n), order, 0)
            np.testing.assert_allclose(T[f], math.sqrt(C[0] / (4 * math.pi)) * xi, rtol=1e-13)


def _chain_variance(orc, order, A, B, n):
    """Var T(z_i, phi) at every ring from exact covariance propagation through the factors
    in both hemispheres (sum over the modes, weight 2 for m > 0)."""
    s = orc.start_ring(n)
    D = np.diag([(-1.0) ** p for p in range(order)])
    even = n % 2 == 0
    var = np.zeros(n)
    for m in range(A.shape[1]):
        w = 1.0 if m == 0 else 2.0
        Sig = B[0, m] @ B[0, m].T
        var[s] += w * Sig[0, 0]
        S0 = Sig
        for j in range(2 if even else 1, A.shape[0]):
            Sig = A[j, m] @ Sig @ A[j, m].T + B[j, m] @ B[j, m].T
            var[s - j + 1 if even else s - j] += w * Sig[0, 0]
        Sig, r, j0 = S0, s, 1
        if even:
            Sig = A[1, m] @ Sig @ A[1, m].T + B[1, m] @ B[1, m].T
            r, j0 = s + 1, 2
            var[r] += w * Sig[0, 0]
        for j in range(j0, A.shape[0]):
            Am, Bm = D @ A[j, m] @ D, D @ B[j, m] @ D
            Sig = Am @ Sig @ Am.T + Bm @ Bm.T
            r += 1
            var[r] += w * Sig[0, 0]
    return var


@pytest.mark.parametrize("order,kappa,n,lmax", [(1, 64.0, 16, 15), (2, 50.0, 11, 10), (1, 5.0, 10, 40),
                                                (3, 50.0, 11, 10), (4, 50.0, 12, 14), (3, 9.0, 16, 40),
                                                (4, 200.0, 17, 30)])
def test_chain_variance_closed_form(orc, order, kappa, n, lmax):
    """Var T(z_i, phi) = sum_l (2l+1) C_l / (4 pi) at every ring, from exact covariance
    propagation through the factors in both hemispheres (no m truncation: n_phi large)."""
    n_phi = 2 * (lmax + 1)
    C = orc.spectrum([kappa] * order, lmax)
    A, B = orc.setup(order, C, n, n_phi)
    var = _chain_variance(orc, order, A, B, n)
    ref = np.sum((2 * np.arange(lmax + 1) + 1) * C) / (4 * math.pi)
    np.testing.assert_allclose(var, ref, rtol=1e-11)


# --------------------------------------------------------------------------- explicit grids
def _grids():
    from paper_1709_10314_amd import workloads as w

    return {"gauss-legendre-12": w.gauss_legendre_z(12), "gauss-legendre-13": w.gauss_legendre_z(13),
            "healpix-nside4": w.healpix_ring_z(4), "random-10": w.random_z(10, 3),
            "random-15": w.random_z(15, 4)}


@pytest.mark.parametrize("grid", sorted(_grids()))
@pytest.mark.parametrize("order,kappa,lmax", [(1, 64.0, 30), (2, 100.0, 25)])
def test_explicit_grid_factors_reproduce_ring_covariances(orc, grid, order, kappa, lmax):
    """Alg. 1 on a grid given as values (Gauss-Legendre nodes, HEALPix ring latitudes, a
    random symmetric grid): covariance propagation through the factors reproduces J at the
    grid's own rings in both hemispheres."""
    z = _grids()[grid]
    assert _propagate_check(orc, order, kappa, len(z), lmax, 2 * (lmax + 1), z=z) < 1e-11


@pytest.mark.parametrize("grid", sorted(_grids()))
@pytest.mark.parametrize("order,kappa,lmax", [(1, 9.0, 24), (2, 50.0, 20)])
def test_explicit_grid_variance_closed_form(orc, grid, order, kappa, lmax):
    """The addition theorem at any latitude: Var T(z_i, phi) = sum_l (2l+1) C_l / (4 pi) at
    every ring of an explicit grid (no m truncation)."""
    z = _grids()[grid]
    n = len(z)
    C = orc.spectrum([kappa] * order, lmax)
    A, B = orc.setup(order, C, n, 2 * (lmax + 1), z=z)
    var = _chain_variance(orc, order, A, B, n)
    ref = np.sum((2 * np.arange(lmax + 1) + 1) * C) / (4 * math.pi)
    np.testing.assert_allclose(var, ref, rtol=1e-11)


# --------------------------------------------------------------------------- U basis (Sec. 3)
@pytest.mark.parametrize("m", [0, 3, 17, 39])
@pytest.mark.parametrize("z1,z2", [(0.3, -0.6), (0.95, 0.9), (0.1, 0.1), (-0.99, -0.97)])
def test_u_basis_is_the_operator_of_sec3(orc, m, z1, z2):
    """The oracle's J in the basis (g, U g), summed over -sqrt((l+m+1)(l-m)) L_{l,m+1}, against
    the operator of Sec. 3 applied by its definition, U_m f = -(1 - z^2)^{(m+1)/2}
    d/dz[(1 - z^2)^{-m/2} f] = -s f' - (m z / s) f, on the oracle's L_lm and dL_lm/dz (each
    pinned to scipy and finite differences above)."""
    lmax = 40
    C = orc.spectrum([100.0, 100.0], lmax)
    J = orc.jblock_u(m, lmax, C, z1, z2)

    def funcs(z):
        L, dL = orc.legendre(m, lmax, math.acos(z))
        s = math.sqrt((1 - z) * (1 + z))
        return L, -s * dL - m * z / s * L

    L1, U1 = funcs(z1)
    L2, U2 = funcs(z2)
    Cm = C[m:]
    ref = np.array([[np.sum(Cm * L1 * L2), np.sum(Cm * L1 * U2)], [np.sum(Cm * U1 * L2), np.sum(Cm * U1 * U2)]])
    assert np.max(np.abs(J - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,kappa,lmax", [(16, 100.0, 15), (21, 900.0, 30), (12, 50.0, 14)])
def test_u_basis_factors_same_law(orc, n, kappa, lmax):
    """Factors in the basis (g, U g): covariance propagation reproduces the U-basis J at
    every ring of both walks (the mirror D = diag(1, -1) holds as in the z basis), and the
    field variance is the addition theorem's at every ring, as in the z basis."""
    C = orc.spectrum([kappa, kappa], lmax)
    n_phi = 2 * (lmax + 1)
    A, B = orc.setup(2, C, n, n_phi, basis="u")
    z = orc.grid(n)[1]
    s = orc.start_ring(n)
    even = n % 2 == 0
    D = np.diag([1.0, -1.0])
    worst = 0.0
    var = np.zeros(n)

    def cmp(S, K):
        d = np.sqrt(np.maximum(np.diag(K), 0))
        sc = np.outer(d, d)
        mask = sc > 1e-280
        return np.max(np.abs(S - K)[mask] / sc[mask]) if mask.any() else 0.0

    for m in range(A.shape[1]):
        w = 1.0 if m == 0 else 2.0
        S0 = B[0, m] @ B[0, m].T
        worst = max(worst, cmp(S0, orc.jblock_u(m, lmax, C, z[s], z[s])))
        var[s] += w * S0[0, 0]
        Sig, a = S0, s
        for j in range(2 if even else 1, A.shape[0]):
            b = s - j + 1 if even else s - j
            Sig = A[j, m] @ Sig @ A[j, m].T + B[j, m] @ B[j, m].T
            worst = max(worst, cmp(Sig, orc.jblock_u(m, lmax, C, z[b], z[b])))
            var[b] += w * Sig[0, 0]
        Sig, r, j0 = S0, s, 1
        if even:
            Sig = A[1, m] @ Sig @ A[1, m].T + B[1, m] @ B[1, m].T
            r, j0 = s + 1, 2
            worst = max(worst, cmp(Sig, orc.jblock_u(m, lmax, C, z[r], z[r])))
            var[r] += w * Sig[0, 0]
        for j in range(j0, A.shape[0]):
            Am, Bm = D @ A[j, m] @ D, D @ B[j, m] @ D
            Sig = Am @ Sig @ Am.T + Bm @ Bm.T
            r += 1
            worst = max(worst, cmp(Sig, orc.jblock_u(m, lmax, C, z[r], z[r])))
            var[r] += w * Sig[0, 0]
    assert worst < 1e-11
    ref = np.sum((2 * np.arange(lmax + 1) + 1) * C) / (4 * math.pi)
    np.testing.assert_allclose(var, ref, rtol=1e-11)


def _asym_grids():
    from paper_1709_10314_amd import workloads as w

    return {"random-14": w.random_asym_z(14, 5), "random-15": w.random_asym_z(15, 6),
            "shifted-16": w.shifted_z(16, 0.3), "shifted-13": w.shifted_z(13, 0.8)}


def _propagate_asym(orc, order, C, lmax, z, A, B, As, Bs):
    """Worst reproduction of J(b,b) and J(b,a) over both walks of a grid with its own
    southern sets (true coordinates, no mirror)."""
    n = len(z)
    s = orc.start_ring(n)
    even = n % 2 == 0
    worst = 0.0

    def cmp(S, K):
        d = np.sqrt(np.maximum(np.diag(K), 0))
        sc = np.outer(d, d)
        mask = sc > 1e-280
        return np.max(np.abs(S - K)[mask] / sc[mask]) if mask.any() else 0.0

    def jb(m, i1, i2):
        return orc.jblock_z(order, m, lmax, C, z[i1], z[i2])

    for m in range(A.shape[1]):
        S0 = B[0, m] @ B[0, m].T
        worst = max(worst, cmp(S0, jb(m, s, s)))
        Sig, a = S0, s
        for j in range(2 if even else 1, A.shape[0]):
            b = s - j + 1 if even else s - j
            cross = A[j, m] @ Sig
            Sig = A[j, m] @ Sig @ A[j, m].T + B[j, m] @ B[j, m].T
            worst = max(worst, cmp(Sig, jb(m, b, b)), cmp(cross, jb(m, b, a)))
            a = b
        Sig, a, j0 = S0, s, 1
        if even:
            cross = A[1, m] @ Sig
            Sig = A[1, m] @ Sig @ A[1, m].T + B[1, m] @ B[1, m].T
            worst = max(worst, cmp(Sig, jb(m, s + 1, s + 1)), cmp(cross, jb(m, s + 1, s)))
            a, j0 = s + 1, 2
        for j in range(j0, As.shape[0]):
            b = a + 1
            cross = As[j, m] @ Sig
            Sig = As[j, m] @ Sig @ As[j, m].T + Bs[j, m] @ Bs[j, m].T
            worst = max(worst, cmp(Sig, jb(m, b, b)), cmp(cross, jb(m, b, a)))
            a = b
    return worst


@pytest.mark.parametrize("n", [16, 17])
@pytest.mark.parametrize("order", [1, 2])
def test_southern_sets_of_a_symmetric_grid_are_the_mirror(orc, n, order):
    """On a symmetric grid the southern walk's own sets equal the mirrored northern ones
    (D A D, D B D, the remark after Alg. 1) and give the same samples, bit for bit: the
    Legendre values at -z are exactly the sign-flipped ones."""
    C = orc.spectrum([100.0] * order, 30)
    z = orc.grid(n)[1]
    A, B = orc.setup(order, C, n, 64, z=z)
    An, Bn, As, Bs = orc.setup_asym(order, C, n, 64, z)
    D = np.diag([(-1.0) ** p for p in range(order)])
    j0 = 2 if n % 2 == 0 else 1
    assert np.array_equal(An, A) and np.array_equal(Bn, B)
    assert np.array_equal(D @ A[j0:] @ D, As[j0:]) and np.array_equal(D @ B[j0:] @ D, Bs[j0:])
    T1, _ = orc.sample(order, n, 64, A, B, 5, 2)
    T2, _ = orc.sample(order, n, 64, An, Bn, 5, 2, south=(As, Bs))
    assert np.array_equal(T1, T2)


@pytest.mark.parametrize("grid", sorted(_asym_grids()))
@pytest.mark.parametrize("order,kappa,lmax", [(1, 64.0, 30), (2, 100.0, 25)])
def test_asymmetric_grid_factors_reproduce_ring_covariances(orc, grid, order, kappa, lmax):
    """A grid with no symmetry: the northern sets and the southern walk's own sets
    reproduce J at every ring of both walks by covariance propagation."""
    z = _asym_grids()[grid]
    C = orc.spectrum([kappa] * order, lmax)
    A, B, As, Bs = orc.setup_asym(order, C, len(z), 2 * (lmax + 1), z)
    assert _propagate_asym(orc, order, C, lmax, z, A, B, As, Bs) < 1e-11


@pytest.mark.parametrize("grid", sorted(_asym_grids()))
@pytest.mark.parametrize("order,kappa,lmax", [(1, 9.0, 24), (2, 50.0, 20)])
def test_asymmetric_grid_variance_closed_form(orc, grid, order, kappa, lmax):
    """The addition theorem at every ring of a grid with no symmetry: Var T(z_i, phi) =
    sum_l (2l+1) C_l / (4 pi), propagated through the northern and the southern sets."""
    z = _asym_grids()[grid]
    n = len(z)
    C = orc.spectrum([kappa] * order, lmax)
    A, B, As, Bs = orc.setup_asym(order, C, n, 2 * (lmax + 1), z)
    s = orc.start_ring(n)
    even = n % 2 == 0
    var = np.zeros(n)
    for m in range(A.shape[1]):
        w = 1.0 if m == 0 else 2.0
        S0 = B[0, m] @ B[0, m].T
        var[s] += w * S0[0, 0]
        Sig = S0
        for j in range(2 if even else 1, A.shape[0]):
            Sig = A[j, m] @ Sig @ A[j, m].T + B[j, m] @ B[j, m].T
            var[s - j + 1 if even else s - j] += w * Sig[0, 0]
        Sig, r, j0 = S0, s, 1
        if even:
            Sig = A[1, m] @ Sig @ A[1, m].T + B[1, m] @ B[1, m].T
            r, j0 = s + 1, 2
            var[r] += w * Sig[0, 0]
        for j in range(j0, As.shape[0]):
            Sig = As[j, m] @ Sig @ As[j, m].T + Bs[j, m] @ Bs[j, m].T
            r += 1
            var[r] += w * Sig[0, 0]
    ref = np.sum((2 * np.arange(lmax + 1) + 1) * C) / (4 * math.pi)
    np.testing.assert_allclose(var, ref, rtol=1e-11)


def test_explicit_grid_of_ring_centres_is_the_default(orc):
    """The ring-centre grid given as values gives the default factors (up to the rounding
    of sin(theta), taken from z instead of the complementary angle)."""
    for n, order in ((17, 1), (16, 2)):
        C = orc.spectrum([30.0] * order, 40)
        A, B = orc.setup(order, C, n, 82)
        A2, B2 = orc.setup(order, C, n, 82, z=orc.grid(n)[1])
        np.testing.assert_allclose(A2, A, rtol=0, atol=1e-12 * np.abs(A).max())
        np.testing.assert_allclose(B2, B, rtol=0, atol=1e-12 * np.abs(B).max())


def test_explicit_grid_rejects_bad_grids(orc):
    C = orc.spectrum([30.0], 10)
    z = orc.grid(8)[1]
    bad = [z[::-1].copy(), np.where(np.arange(8) == 7, -z[0] * 0.999, z), np.linspace(1.0, -1.0, 8),
           np.r_[z[:4], z[:4][::-1] * -1.0 + 1e-9]]
    for zb in bad:
        with pytest.raises(ValueError):
            orc.setup(1, C, 8, 16, z=zb)
    with pytest.raises(ValueError):
        orc.setup(1, C, 8, 16, z=z[:7])


def test_sample_reproducible_and_field_keyed(orc):
    """Field f of sample(seed, count) is keyed seed+f: sample(1, 3) = [sample(1+f, 1)]."""
    C = orc.spectrum([64.0], 15)
    A, B = orc.setup(1, C, 16, 32)
    T3, _ = orc.sample(1, 16, 32, A, B, 1, 3)
    for f in range(3):
        T1, _ = orc.sample(1, 16, 32, A, B, 1 + f, 1)
        assert np.array_equal(T3[f], T1[0])


@pytest.mark.slow
@pytest.mark.parametrize("order", [1, 3])
def test_empirical_covariance_matches_addition_theorem(orc, order):
    """Sec. 5's validation on a tiny grid: the covariance of N = 10^5 oracle samples
    against C_T(x,y) = sum_l (2l+1)/(4 pi) C_l P_l(<x,y>), within 5 standard errors
    (Isserlis: Var(x y) = C_xx C_yy + C_xy^2) plus the chain's deterministic Markov defect
    for pairs two or more rings apart (computed from the factors by propagation).  Order 3
    exercises the normals' counter map when a ring's three normals straddle two blocks."""
    kappa, n, lmax = 20.0, 8, 63
    n_phi = 2 * (lmax + 1)
    C = orc.spectrum([kappa] * order, lmax)
    A, B = orc.setup(order, C, n, n_phi)
    N = 100_000
    T, _ = orc.sample(order, n, n_phi, A, B, 12345, N)
    th, z = orc.grid(n)
    x = T[:, :, 0]                                      # reference column phi = 0
    jj = np.arange(0, n_phi, 8)
    phis = 2 * np.pi * jj / n_phi
    var = np.sum((2 * np.arange(lmax + 1) + 1) * C) / (4 * np.pi)
    defect = _markov_defect(orc, order, A, B, n, lmax, C)
    for a in range(n):
        y = T[:, :, jj]                                 # [N, n, len(jj)]
        emp = np.einsum("k,kbj->bj", x[:, a], y) / N
        cosg = (np.cos(th[a]) * np.cos(th)[:, None]
                + np.sin(th[a]) * np.sin(th)[:, None] * np.cos(phis)[None, :])
        ref = np.vectorize(lambda c: _addition_target(C, c))(cosg)
        se = np.sqrt((var * var + ref ** 2) / N)
        tol = 5 * se + defect[a][:, None]
        assert np.all(np.abs(emp - ref) <= tol), (a, np.max(np.abs(emp - ref) / tol))


def _chain_cov(order, A, B, n, m):
    """Joint covariance of the chain states of mode m over all rings, by exact
    propagation in generation order: x_new = P x_parent + Q w gives
    Cov(x_new, x_k) = P Cov(x_parent, x_k) and Var(x_new) = P Var(x_parent) P^T + Q Q^T."""
    s = n // 2 - 1 if n % 2 == 0 else (n - 1) // 2
    D = np.diag([(-1.0) ** p for p in range(order)])
    order_list = [(s, None, None, B[0, m])]
    even = n % 2 == 0
    for j in range(2 if even else 1, A.shape[0]):
        b = s - j + 1 if even else s - j
        order_list.append((b, b + 1, A[j, m], B[j, m]))
    prev, j0 = s, 1
    if even:
        order_list.append((s + 1, s, A[1, m], B[1, m]))
        prev, j0 = s + 1, 2
    for j in range(j0, A.shape[0]):
        order_list.append((prev + 1, prev, D @ A[j, m] @ D, D @ B[j, m] @ D))
        prev += 1
    cov = {}
    done = []
    for r, parent, P, Q in order_list:
        if parent is None:
            cov[(r, r)] = Q @ Q.T
        else:
            for k in done:
                cov[(r, k)] = P @ cov[(parent, k)]
                cov[(k, r)] = cov[(r, k)].T
            cov[(r, r)] = P @ cov[(parent, parent)] @ P.T + Q @ Q.T
        done.append(r)
    return cov


def _markov_defect(orc, order, A, B, n, lmax, C):
    """sum_m w_m |chain-implied Cov(g_m(z_a), g_m(z_b)) - J^m_00(a,b)|, an upper bound on
    the deterministic gap between the chain's field covariance and C_T for ring pair (a,b)."""
    th, _ = orc.grid(n)
    out = np.zeros((n, n))
    for m in range(A.shape[1]):
        w = 1.0 if m == 0 else 2.0
        cov = _chain_cov(order, A, B, n, m)
        for a in range(n):
            for b in range(n):
                Kab = orc.jblock_ring(order, m, lmax, C, n, a, b)[0, 0]
                out[a, b] += w * abs(cov[(a, b)][0, 0] - Kab)
    return out
