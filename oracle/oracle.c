/*
 * FP64 CPU oracle for the sampling method of Creasey & Lang, "Fast generation of
 * isotropic Gaussian random fields on the sphere" (arXiv:1709.10314).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path (the HIP
 * library) shares no code with it and never calls it.
 *
 * Everything here is plain, slow FP64 C, written so that each step can be checked
 * against the paper by eye:
 *   - grid and spectrum                         (Sec. 2, eq. (Cl); Sec. 4 grid)
 *   - fully normalised associated Legendre L_lm and dL_lm/dz by the forward
 *     recurrence in l, seeded with an extended-exponent sectoral value; second
 *     and third z-derivatives from the associated Legendre equation
 *                                               (Sec. 2, definition of L_lm)
 *   - cross-covariance blocks J^m_pq(z1,z2) as brute-force sums over l
 *                                               (Lemma 2.1, cross covariances)
 *   - transition A, innovation factor B, start factor B_eq
 *                                               (eqs. (trans_matrix),
 *                                                (innov_matrix), (state_initial);
 *                                                Alg. 1)
 *   - Philox4x32-10 words and Box-Muller normals (white-noise source; the paper
 *     leaves it open)
 *   - the state-space recursion outward from the equator, south half by mirror
 *                                               (eq. (state_space); Alg. 2; the
 *                                                symmetry remark after Alg. 1)
 *   - the inverse DFT along phi                 (Alg. 2, last step), also on rings
 *     with their own pixel counts and first-pixel longitudes (iso-latitude grids
 *     such as HEALPix, which Sec. 1 names)
 *
 * Readings where the paper is silent or garbled:
 *   grid      theta_i = pi (i + 1/2) / n_theta, z_i = cos(theta_i), ring 0 nearest z = +1;
 *             phi_j = 2 pi j / n_phi; z_i evaluated as sin(pi (n - 2i - 1) / (2n)).  For
 *             odd n_theta = 2k + 1 this is the symmetric example grid of Sec. 4 read as
 *             z_j = sin(pi j / (2k + 1)).  Alg. 1 also takes any grid symmetric about the
 *             equator (orc_setup_z), with sin(theta) = sqrt((1 - z)(1 + z)).
 *   modes     m = 0 .. m_top, m_top = min(ell_max, n_phi/2 - 1); the Nyquist mode is not used.
 *   DFT       unnormalised: T = g_0 + 2 sum_{m>=1} Re(g_m e^{i m phi}).
 *   A, B      A = J(b,a) J(a,a)^+ with J(b,a)_pq = E[x_b,p x_a,q];  S = J(b,b) - A J(a,b);
 *             both factorisations by an equilibrated, thresholded Cholesky (rules below).
 *   start     even n_theta: ring s = n_theta/2 - 1 from chol(J(s,s)), one crossing step
 *             to ring s+1 (= -z_s), then outward both ways; odd n_theta: start at the
 *             equator ring.  South steps use D A D, D B D with D = diag((-1)^p).
 *   noise     m = 0: one real chain (scale 1); m > 0: Re and Im chains with B scaled by
 *             1/sqrt(2) (complex standard normal with E|w|^2 = 1).
 *   RNG       key = (lo32, hi32) of (seed + field); counter = (floor(idx/4), m, part, 0) with
 *             idx = ring*M + q; word idx mod 4; u = (x + 0.5) 2^-32; Box-Muller on the word
 *             pairs (0,1) and (2,3).
 */
#include <complex.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXM 4            /* state dimension supported: value and z-derivatives up to the third */
#define ORC_TINY 1e-290       /* a block diagonal below this is treated as exactly zero */
#define ORC_TAU 1e-12         /* pivot / relative-variance threshold after equilibration */

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Threads of the parallel loops (timing only: the loops' results do not depend on it). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Threads an OpenMP region of the oracle will use. */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Grid (Sec. 4, with the ring-centre reading above).  z_i = cos(theta_i) and   */
/* sin(theta_i) are evaluated through the complementary angle                  */
/* pi/2 - theta_i = pi (n - 2i - 1) / (2n), whose numerator is an exact        */
/* integer: the equator ring of an odd grid gets z = 0 exactly and mirrored     */
/* rings get exactly opposite z, the symmetry z_{-i} = -z_i of Sec. 4.         */
/* ------------------------------------------------------------------------- */
void orc_ring_zs(int n_theta, int i, double* z, double* s)
{
    double q = (double)(n_theta - 2 * i - 1) / (2.0 * n_theta);
    *z = sin(M_PI * q);
    *s = cos(M_PI * q);
}

void orc_grid(int n_theta, double* theta, double* z)
{
    for (int i = 0; i < n_theta; ++i) {
        double zi, si;
        orc_ring_zs(n_theta, i, &zi, &si);
        if (theta) theta[i] = M_PI * (i + 0.5) / n_theta;
        if (z) z[i] = zi;
    }
}

/* ------------------------------------------------------------------------- */
/* Spectrum, eq. (Cl): C_l = prod_i (kappa_i + l(l+1))^-1 for l <= ell_max.     */
/* Returns 0, or -1 if some C_l is not finite and positive.                    */
/* ------------------------------------------------------------------------- */
int orc_spectrum(int n_kappa, const double* kappa, int ell_max, double* C)
{
    for (int l = 0; l <= ell_max; ++l) {
        double c = 1.0;
        for (int i = 0; i < n_kappa; ++i) c /= (kappa[i] + (double)l * (l + 1));
        if (!(c > 0.0) || !isfinite(c)) return -1;
        C[l] = c;
    }
    return 0;
}

/* The same product with complex kappa_i = kre[i] + i kim[i] (Sec. 3 allows complex   */
/* kappa_i, e.g. the pair +-i a of the spectrum (a^2 + l^2 (l+1)^2)^-1): the product   */
/* is formed in complex arithmetic and must come out real and positive (conjugate     */
/* pairs); returns -1 if some C_l is not (imaginary part above 1e-12 of its modulus).  */
int orc_spectrum_complex(int n_kappa, const double* kre, const double* kim, int ell_max, double* C)
{
    for (int l = 0; l <= ell_max; ++l) {
        double pr = 1.0, pi = 0.0;   /* running product of (kappa_i + l(l+1)) */
        for (int i = 0; i < n_kappa; ++i) {
            const double ar = kre[i] + (double)l * (l + 1), ai = kim[i];
            const double r = pr * ar - pi * ai, im = pr * ai + pi * ar;
            pr = r;
            pi = im;
        }
        if (!(pr > 0.0) || !isfinite(pr) || fabs(pi) > 1e-12 * fabs(pr)) return -1;
        C[l] = 1.0 / pr;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Fully normalised associated Legendre functions (Sec. 2):                    */
/*   L_lm(z) = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_lm(z),  z = cos(theta),     */
/* without the Condon-Shortley sign (it cancels in every product L_lm L_lm).   */
/* Fills L[l-m] and dL[l-m] = dL_lm/dz for l = m .. ell_max.                   */
/*                                                                             */
/* Sectoral start:  L_00 = 1/sqrt(4 pi),                                       */
/*                  L_kk = sqrt((2k+1)/(2k)) sin(theta) L_{k-1,k-1}.            */
/* First step:      L_{m+1,m} = sqrt(2m+3) z L_mm.                              */
/* Recurrence:      L_lm = a_lm (z L_{l-1,m} - L_{l-2,m} / a_{l-1,m}),          */
/*                  a_lm = sqrt((4l^2 - 1)/(l^2 - m^2)).                        */
/* Derivative:      (1 - z^2) dL_lm/dz = -l z L_lm                              */
/*                        + sqrt((2l+1)(l^2 - m^2)/(2l-1)) L_{l-1,m}.           */
/* The running pair carries a binary exponent e (value = p * 2^e) so that the   */
/* sin^m(theta) seed cannot underflow; values are returned as plain doubles     */
/* (ldexp), i.e. anything below the FP64 range comes back as zero/subnormal.    */
/* ------------------------------------------------------------------------- */
void orc_legendre_zs(int m, int ell_max, double z, double s, double* L, double* dL)
{
    const double s2 = s * s;
    const double big = ldexp(1.0, 480), small = ldexp(1.0, -480);
    int e = 0;
    double p = 1.0 / sqrt(4.0 * M_PI);
    for (int k = 1; k <= m; ++k) {
        p *= sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
        if (fabs(p) < small) { p *= big; e -= 480; }
    }
    if (ell_max < m) return;
    /* l = m */
    L[0] = ldexp(p, e);
    if (dL) dL[0] = ldexp(-(double)m * z * p / s2, e);
    if (ell_max == m) return;
    /* l = m + 1 */
    double p0 = p;
    double p1 = sqrt(2.0 * m + 3.0) * z * p;
    L[1] = ldexp(p1, e);
    if (dL) {
        double l = m + 1.0;
        double c = sqrt((2.0 * l + 1.0) * (l * l - (double)m * m) / (2.0 * l - 1.0));
        dL[1] = ldexp((-l * z * p1 + c * p0) / s2, e);
    }
    for (int li = m + 2; li <= ell_max; ++li) {
        double l = li, lm1 = li - 1;
        double a = sqrt((4.0 * l * l - 1.0) / (l * l - (double)m * m));
        double a_prev = sqrt((4.0 * lm1 * lm1 - 1.0) / (lm1 * lm1 - (double)m * m));
        double p2 = a * (z * p1 - p0 / a_prev);
        p0 = p1;
        p1 = p2;
        if (e < 0 && (fabs(p1) > big || fabs(p0) > big)) {
            p0 *= small;
            p1 *= small;
            e += 480;
        }
        L[li - m] = ldexp(p1, e);
        if (dL) {
            double c = sqrt((2.0 * l + 1.0) * (l * l - (double)m * m) / (2.0 * l - 1.0));
            dL[li - m] = ldexp((-l * z * p1 + c * p0) / s2, e);
        }
    }
}

/* The same at z = cos(theta), s = sin(theta). */
void orc_legendre(int m, int ell_max, double theta, double* L, double* dL)
{
    orc_legendre_zs(m, ell_max, cos(theta), sin(theta), L, dL);
}

/* ------------------------------------------------------------------------- */
/* Higher z-derivatives from the associated Legendre equation, which L_lm       */
/* solves for every l (primes are z-derivatives):                              */
/*   (1 - z^2) L2 = 2 z L1 - (l(l+1) - m^2/(1 - z^2)) L0,                      */
/* and its derivative                                                          */
/*   (1 - z^2) L3 = 4 z L2 + 2 L1 - (l(l+1) - m^2/(1 - z^2)) L1                */
/*                  + 2 m^2 z / (1 - z^2)^2 L0,                                */
/* with Lk = d^k L_lm / dz^k.  F[k][l-m] = Lk for k < nd (nd <= 4),            */
/* l = m .. ell_max; each F[k] holds ell_max - m + 1 values.                   */
/* ------------------------------------------------------------------------- */
void orc_legendre_derivs(int m, int ell_max, double z, double s, int nd, double* const* F)
{
    const int n = ell_max - m + 1;
    if (n <= 0 || nd <= 0) return;
    orc_legendre_zs(m, ell_max, z, s, F[0], nd > 1 ? F[1] : NULL);
    const double s2 = s * s;
    const double mm = (double)m * m;
    for (int k = 0; k < n && nd > 2; ++k) {
        const double l = m + k;
        const double c = l * (l + 1.0) - mm / s2;
        F[2][k] = (2.0 * z * F[1][k] - c * F[0][k]) / s2;
        if (nd > 3)
            F[3][k] = (4.0 * z * F[2][k] + 2.0 * F[1][k] - c * F[1][k] + 2.0 * mm * z / (s2 * s2) * F[0][k]) / s2;
    }
}

/* ------------------------------------------------------------------------- */
/* Cross-covariance block (Lemma 2.1 and the cross covariances of Sec. 2):     */
/*   J_pq = sum_{l=m}^{ell_max} C_l  d^p L_lm(z1)  d^q L_lm(z2),  p,q < M,     */
/* with z1 = cos(theta1), z2 = cos(theta2).  J[p*M + q].                       */
/* ------------------------------------------------------------------------- */
void orc_jblock_zs(int order, int m, int ell_max, const double* C, double z1, double s1, double z2,
                   double s2, double* J)
{
    int n = ell_max - m + 1;
    for (int i = 0; i < order * order; ++i) J[i] = 0.0;
    if (n <= 0) return;
    double* buf = (double*)malloc(sizeof(double) * 2 * ORC_MAXM * n);
    double* F1[ORC_MAXM];
    double* F2[ORC_MAXM];
    for (int k = 0; k < ORC_MAXM; ++k) {
        F1[k] = buf + (size_t)k * n;
        F2[k] = buf + (size_t)(ORC_MAXM + k) * n;
    }
    int nd = order < 2 ? 2 : order;
    orc_legendre_derivs(m, ell_max, z1, s1, nd, F1);
    orc_legendre_derivs(m, ell_max, z2, s2, nd, F2);
    for (int p = 0; p < order; ++p)
        for (int q = 0; q < order; ++q) {
            const double* f1 = F1[p];
            const double* f2 = F2[q];
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += C[m + k] * f1[k] * f2[k];
            J[p * order + q] = acc;
        }
    free(buf);
}

/* ------------------------------------------------------------------------- */
/* Order 2 in the basis (g, U g) of Sec. 3 (eq. (Jmatrix_more_efficient)).      */
/* U_m f = -(1 - z^2)^{(m+1)/2} d/dz[(1 - z^2)^{-m/2} f] maps P^m to P^{m+1}     */
/* (Sec. 3); for the normalised functions here (no Condon-Shortley sign) that   */
/* reads U_m L_lm = -sqrt((l+m+1)(l-m)) L_{l,m+1}, which is what is summed       */
/* (exactly zero at l = m, no cancellation near the poles).  The value          */
/* component is unchanged, so the field's law is the same; the realisations     */
/* differ from those of the z-derivative basis.                                */
/* ------------------------------------------------------------------------- */
void orc_jblock_zs_u(int m, int ell_max, const double* C, double z1, double s1, double z2, double s2, double* J)
{
    int n = ell_max - m + 1;
    for (int i = 0; i < 4; ++i) J[i] = 0.0;
    if (n <= 0) return;
    double* L1 = (double*)calloc(4 * (size_t)n, sizeof(double));
    double* U1 = L1 + n;
    double* L2 = L1 + 2 * n;
    double* U2 = L1 + 3 * n;
    orc_legendre_zs(m, ell_max, z1, s1, L1, NULL);
    orc_legendre_zs(m, ell_max, z2, s2, L2, NULL);
    if (n > 1) {
        /* L_{l,m+1} for l = m+1 .. ell_max into slots 1 .. n-1 */
        orc_legendre_zs(m + 1, ell_max, z1, s1, U1 + 1, NULL);
        orc_legendre_zs(m + 1, ell_max, z2, s2, U2 + 1, NULL);
        for (int k = 1; k < n; ++k) {
            const double l = m + k;
            const double f = -sqrt((l + m + 1.0) * (l - m));
            U1[k] *= f;
            U2[k] *= f;
        }
    }
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) {
            const double* f1 = p ? U1 : L1;
            const double* f2 = q ? U2 : L2;
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += C[m + k] * f1[k] * f2[k];
            J[p * 2 + q] = acc;
        }
    free(L1);
}

/* ------------------------------------------------------------------------- */
/* Sec. 3: the cross covariance of one mode from the Green's function, order 1, */
/* C_l = 1/(kappa + l(l+1)) for every l >= 0 (no band limit; one kappa, so the   */
/* partial fractions of eq. (C_ell_efficient) are the spectrum itself, b = 1).   */
/* With kappa = -lambda(lambda+1), eq. (Jmatrix_efficient) reads                */
/*   J^m(z1, z2) = Gamma(1+lambda-m) Gamma(-lambda-m)/(4 pi) P^m(-z1) P^m(z2),   */
/* z1 <= z2, with P^m = P^m_lambda of eq. (Legendre_hypergeometric):            */
/*   P^m(x) = (-lambda)_m (1+lambda)_m / m! ((1-x)/(1+x))^{m/2} G_m(x),          */
/*   G_m(x) = 2F1(-lambda, lambda+1; 1+m; (1-x)/2).                              */
/* Written out with Pi_m = (-lambda)_m (1+lambda)_m = prod_{k=1}^m (k^2-k+kappa) */
/* and Gamma(1+lambda) Gamma(-lambda) = pi / |sin(pi lambda)| (reflection):      */
/*   J^m(z1, z2) = 1/(4 |sin pi lambda|) (Pi_m / m!^2) w^m G_m(-z1) G_m(z2),      */
/*   w = sqrt((1+z1)(1-z2) / ((1-z1)(1+z2))) <= 1.                               */
/* lambda = -1/2 + i tau (tau = sqrt(kappa - 1/4)) for kappa > 1/4, where        */
/* |sin pi lambda| = cosh(pi tau); for 0 < kappa <= 1/4 lambda is real,          */
/* (-1 + sqrt(1 - 4 kappa))/2, and |sin pi lambda| = -sin(pi lambda).            */
/* The series of G_m has positive terms ((n-lambda)(n+lambda+1) = n^2+n+kappa):  */
/*   x >= 0 (argument t <= 1/2): the series itself;                              */
/*   x < 0: G_0 and G_1 from the series, or near x = -1 from the continuation of  */
/*   2F1 about t = 1 for c - a - b a non-negative integer (Abramowitz & Stegun    */
/*   15.3.11; DLMF 15.8.10), with its logarithm and digamma terms, then G_m by    */
/*   the three-term recurrence in                                                */
/*   the order of the Ferrers functions (DLMF 14.10.1) rewritten for G_m:        */
/*     G_{m+2} = (m+1)(m+2)/q_{m+1} (1+x)/(1-x) [G_m - 2x/(1+x) G_{m+1}],         */
/*     q_k = k^2 + k + kappa,                                                    */
/*   whose terms are both positive for x < 0 (no cancellation).                  */
/* Arguments come as (z, s = sin theta) pairs, and 1 -+ z as s^2/(1 +- z) on the  */
/* side where that is the accurate form.                                         */
/* ------------------------------------------------------------------------- */
static double complex green_lambda(double kappa)
{
    if (kappa > 0.25) return -0.5 + I * sqrt(kappa - 0.25);
    return (-1.0 + sqrt(1.0 - 4.0 * kappa)) / 2.0;
}

static double green_abs_sin(double kappa)
{
    if (kappa > 0.25) return cosh(M_PI * sqrt(kappa - 0.25));
    return -sin(M_PI * creal(green_lambda(kappa)));
}

/* digamma for Re z > 0: shift to Re z >= 20 by psi(z) = psi(z+1) - 1/z, then the  */
/* asymptotic series ln z - 1/(2z) - sum_k B_2k / (2k z^2k) to z^-10.              */
static double complex cdigamma(double complex z)
{
    double complex acc = 0.0;
    while (creal(z) < 20.0) {
        acc -= 1.0 / z;
        z += 1.0;
    }
    const double complex r = 1.0 / (z * z);
    const double complex ser =
        r * (1.0 / 12 - r * (1.0 / 120 - r * (1.0 / 252 - r * (1.0 / 240 - r * (1.0 / 132)))));
    return acc + clog(z) - 0.5 / z - ser;
}

/* psi(-lambda + k) + psi(lambda + 1 + k) (real for both kinds of lambda) */
static double green_psi_pair(double kappa, double k)
{
    const double complex lam = green_lambda(kappa);
    return creal(cdigamma(-lam + k) + cdigamma(lam + 1.0 + k));
}

/* G_m at argument t = (1 - x)/2 by its series (used for t <= 1/2). */
static double green_G_series(int m, double kappa, double t)
{
    double sum = 1.0, term = 1.0;
    for (int n = 0; n < 200000; ++n) {
        const double ratio = ((double)n * n + n + kappa) / ((n + 1.0) * (n + 1.0 + m)) * t;
        term *= ratio;
        sum += term;
        if (ratio < 1.0 && term < 1e-18 * sum) break;
    }
    return sum;
}

/* G_0 and G_1 at t = (1 - x)/2 >= 1/2 from the continuation about t = 1, u = 1 - t:  */
/*   G_0 = -g sum_k c_k u^k [ln u - 2 psi(k+1) + psi(a+k) + psi(b+k)],                */
/*   G_1 = g/kappa + g u sum_k d_k u^k [ln u - psi(k+1) - psi(k+2) + psi(a+k+1)       */
/*                                       + psi(b+k+1)],                               */
/* a = -lambda, b = lambda + 1, g = 1/(Gamma(a) Gamma(b)) = |sin pi lambda| / pi,      */
/* c_k = (a)_k (b)_k / k!^2, d_k = (a+1)_k (b+1)_k / (k! (k+1)!).                      */
static void green_G01_far(double kappa, double u, double* G0, double* G1)
{
    const double g = green_abs_sin(kappa) / M_PI;
    const double L = log(u);
    const double euler = 0.57721566490153286061;
    double c = 1.0, d = 1.0, uk = 1.0, s0 = 0.0, s1 = 0.0;
    double psi_k1 = -euler;              /* psi(k+1) */
    for (int k = 0; k < 100000; ++k) {
        const double psi_k2 = psi_k1 + 1.0 / (k + 1.0);   /* psi(k+2) */
        const double t0 = c * uk * (L - 2.0 * psi_k1 + green_psi_pair(kappa, k));
        const double t1 = d * uk * (L - psi_k1 - psi_k2 + green_psi_pair(kappa, k + 1.0));
        s0 += t0;
        s1 += t1;
        const double dk = k;
        c *= (dk * dk + dk + kappa) / ((dk + 1.0) * (dk + 1.0));
        d *= ((dk + 1.0) * (dk + 1.0) + (dk + 1.0) + kappa) / ((dk + 1.0) * (dk + 2.0));
        uk *= u;
        psi_k1 = psi_k2;
        if (k > 4 && fabs(t0) < 1e-18 * fabs(s0) && fabs(t1) < 1e-18 * fabs(s1) &&
            (dk * dk + dk + kappa) / ((dk + 1.0) * (dk + 1.0)) * u < 0.9)
            break;
    }
    *G0 = -g * s0;
    *G1 = g / kappa + g * u * s1;
}

/* G_0 .. G_{m_top} at the ring value x (with s = sin theta) into G.  For x < 0 the    */
/* continuation about t = 1 is used where u = 1 - t is small against 1/(kappa + 1):     */
/* further out its terms cancel (the sum is G_0 / g, and g = |sin pi lambda| / pi grows  */
/* like e^{pi tau}), and there the series in t converges in about 37 / u terms instead.  */
static void green_G_all(int m_top, double kappa, double x, double s, double* G)
{
    if (x >= 0.0) {
        const double t = s * s / (2.0 * (1.0 + x));         /* (1 - x)/2 */
        for (int m = 0; m <= m_top; ++m) G[m] = green_G_series(m, kappa, t);
        return;
    }
    const double u = s * s / (2.0 * (1.0 - x));             /* (1 + x)/2 = 1 - t */
    double g0, g1;
    if (u * (kappa + 1.0) <= 0.5) {
        green_G01_far(kappa, u, &g0, &g1);
    } else {
        g0 = green_G_series(0, kappa, 1.0 - u);
        g1 = green_G_series(1, kappa, 1.0 - u);
    }
    G[0] = g0;
    if (m_top >= 1) G[1] = g1;
    const double opx = 2.0 * u, omx = 1.0 - x;              /* 1 + x, 1 - x */
    for (int k = 0; k + 2 <= m_top; ++k) {                  /* G_{k+2} from G_k, G_{k+1} */
        const double q = (k + 1.0) * (k + 1.0) + (k + 1.0) + kappa;
        G[k + 2] = (k + 1.0) * (k + 2.0) / q * (opx / omx) * (G[k] - 2.0 * x / opx * G[k + 1]);
    }
}

double orc_green_G(int m, double kappa, double x, double s)
{
    double* G = (double*)malloc(sizeof(double) * (m + 1));
    green_G_all(m, kappa, x, s, G);
    const double v = G[m];
    free(G);
    return v;
}

/* P^m_lambda(x) of eq. (Legendre_hypergeometric); returned as a plain double (it     */
/* overflows for large m away from x = 1; the covariance below never forms it).     */
double orc_green_P(int m, double kappa, double x, double s)
{
    double pre = 1.0;
    for (int k = 1; k <= m; ++k) pre *= ((double)k * k - k + kappa) / k;
    const double omx = x >= 0.0 ? s * s / (1.0 + x) : 1.0 - x;
    const double opx = x >= 0.0 ? 1.0 + x : s * s / (1.0 - x);
    return pre * pow(omx / opx, 0.5 * m) * orc_green_G(m, kappa, x, s);
}

/* The factor of J^m(z1, z2) that does not hold G: (Pi_m / m!^2) w^m / (4 |sin pi lambda|), */
/* z1 <= z2.                                                                            */
static double green_J_scale(int m, double kappa, double z1, double s1, double z2, double s2)
{
    double ratio = 1.0;                                      /* Pi_m / m!^2 */
    for (int k = 1; k <= m; ++k) ratio *= ((double)k * k - k + kappa) / ((double)k * k);
    double wm = 1.0;
    if (z1 != z2 && m > 0) {
        /* ln w = (ln(1+z1) + ln(1-z2) - ln(1-z1) - ln(1+z2)) / 2 */
        const double l1p = z1 >= 0.0 ? log1p(z1) : log(s1 * s1 / (1.0 - z1));
        const double l1m = z1 >= 0.0 ? log(s1 * s1 / (1.0 + z1)) : log1p(-z1);
        const double l2p = z2 >= 0.0 ? log1p(z2) : log(s2 * s2 / (1.0 - z2));
        const double l2m = z2 >= 0.0 ? log(s2 * s2 / (1.0 + z2)) : log1p(-z2);
        wm = exp(0.5 * m * (l1p + l2m - l1m - l2p));
    }
    return ratio * wm / (4.0 * green_abs_sin(kappa));
}

/* J^m(z1, z2) of eq. (Jmatrix_efficient), order 1 (1 x 1 block). */
void orc_jblock_green(int m, double kappa, double z1, double s1, double z2, double s2, double* J)
{
    if (z1 > z2) {
        double t = z1; z1 = z2; z2 = t;
        t = s1; s1 = s2; s2 = t;
    }
    J[0] = green_J_scale(m, kappa, z1, s1, z2, s2) * orc_green_G(m, kappa, -z1, s1) * orc_green_G(m, kappa, z2, s2);
}

/* Order 2 (two distinct real kappa_1, kappa_2 > 0) in the basis (g, U g) of Sec. 3:       */
/* the partial fractions of eq. (C_ell_efficient), C_l = b_1/(l(l+1) + kappa_1)              */
/* + b_2/(l(l+1) + kappa_2) with b_1 = 1/(kappa_2 - kappa_1) = -b_2, and eq. (Jmatrix_efficient) */
/* with P^{m+p} for p, q < 2.  Written out as for order 1, for z1 <= z2:                    */
/*   J_pq = sum_i b_i (Pi^i_m / m!^2) w^m / (4 |sin pi lambda_i|) (-1)^p                      */
/*          (a_i r1)^p G^i_{m+p}(-z1) (a_i r2)^q G^i_{m+q}(z2),                              */
/*   a_i = (m^2 + m + kappa_i) / (m + 1)  (= Pi^i_{m+1} / (Pi^i_m (m+1))),                   */
/*   r1 = sqrt((1 + z1)/(1 - z1)), r2 = sqrt((1 - z2)/(1 + z2)),                             */
/* and J(z1, z2) = J(z2, z1)^T for z1 > z2.  J[p*2 + q].                                     */
static void green2_block(int m, const double* kap, double z1, double s1, double z2, double s2, const double* Gn1_0,
                         const double* Gn1_1, const double* Gp2_0, const double* Gp2_1, double* J)
{
    /* Gn1_i[0..1] = G^i_m(-z1), G^i_{m+1}(-z1); Gp2_i[0..1] = G^i_m(z2), G^i_{m+1}(z2) */
    const double b1 = 1.0 / (kap[1] - kap[0]);
    const double b[2] = {b1, -b1};
    const double* Gn[2] = {Gn1_0, Gn1_1};
    const double* Gp[2] = {Gp2_0, Gp2_1};
    /* r1 = sqrt((1+z1)/(1-z1)), r2 = sqrt((1-z2)/(1+z2)), 1 -+ z through sin^2 on the small side */
    const double opz1 = z1 >= 0.0 ? 1.0 + z1 : s1 * s1 / (1.0 - z1), omz1 = z1 >= 0.0 ? s1 * s1 / (1.0 + z1) : 1.0 - z1;
    const double opz2 = z2 >= 0.0 ? 1.0 + z2 : s2 * s2 / (1.0 - z2), omz2 = z2 >= 0.0 ? s2 * s2 / (1.0 + z2) : 1.0 - z2;
    const double r1 = sqrt(opz1 / omz1), r2 = sqrt(omz2 / opz2);
    for (int i = 0; i < 4; ++i) J[i] = 0.0;
    for (int i = 0; i < 2; ++i) {
        const double sc = b[i] * green_J_scale(m, kap[i], z1, s1, z2, s2);
        const double a = ((double)m * m + m + kap[i]) / (m + 1.0);
        const double u[2] = {Gn[i][0], -a * r1 * Gn[i][1]};   /* (-1)^p (a r1)^p G_{m+p}(-z1) */
        const double v[2] = {Gp[i][0], a * r2 * Gp[i][1]};    /* (a r2)^q G_{m+q}(z2) */
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) J[p * 2 + q] += sc * u[p] * v[q];
    }
}

/* J^m(z1, z2) of order 2 from the Green's functions (2 x 2 block, see green2_block). */
void orc_jblock_green2(int m, const double* kap, double z1, double s1, double z2, double s2, double* J)
{
    const int swap = z1 > z2;
    if (swap) {
        double t = z1; z1 = z2; z2 = t;
        t = s1; s1 = s2; s2 = t;
    }
    double gn[2][2], gp[2][2];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k) {
            gn[i][k] = orc_green_G(m + k, kap[i], -z1, s1);
            gp[i][k] = orc_green_G(m + k, kap[i], z2, s2);
        }
    double K[4];
    green2_block(m, kap, z1, s1, z2, s2, gn[0], gn[1], gp[0], gp[1], K);
    if (swap) {
        J[0] = K[0]; J[1] = K[2]; J[2] = K[1]; J[3] = K[3];
    } else {
        for (int i = 0; i < 4; ++i) J[i] = K[i];
    }
}

/* ------------------------------------------------------------------------- */
/* Sec. 3 with a complex-conjugate pair kappa_{1,2} = alpha +- i beta (beta > 0), the form of */
/* the Sec. 5 spectrum C_l = 1/((l(l+1))^2 + 10) = 1/((l(l+1) + i sqrt10)(l(l+1) - i sqrt10)).  */
/* Every step of the real case holds with complex arithmetic: lambda = -1/2 + sqrt(1/4 -       */
/* kappa) (either root: G_m and sin(pi lambda) are symmetric under lambda -> -1 - lambda),     */
/* the series and continuation of G_m with complex terms, and Gamma(1+lambda) Gamma(-lambda)   */
/* = -pi / sin(pi lambda), so that                                                           */
/*   J^m_kappa(z1, z2) = (Pi_m / m!^2) w^m G_m(-z1) G_m(z2) / (-4 sin pi lambda),  z1 <= z2.    */
/* For the real cases -sin(pi lambda) = |sin(pi lambda)|, the form above.  The partial fractions */
/* have b_1 = 1/(kappa_2 - kappa_1) = i / (2 beta) = -b_2, and the kappa_2 term is the complex  */
/* conjugate of the kappa_1 term, so the order-2 block in the basis (g, U g) is                 */
/*   J_pq = 2 Re[ b_1 (Pi_m / m!^2) w^m / (-4 sin pi lambda_1) (-1)^p (a_1 r1)^p              */
/*                G_{m+p}(-z1) (a_1 r2)^q G_{m+q}(z2) ],  a_1 = (m^2 + m + kappa_1) / (m + 1).   */
/* ------------------------------------------------------------------------- */
static double complex greenc_lambda(double complex kappa) { return -0.5 + csqrt(0.25 - kappa); }

static double complex greenc_G_series(int m, double complex kappa, double t)
{
    double complex sum = 1.0, term = 1.0;
    for (int n = 0; n < 200000; ++n) {
        const double complex ratio = ((double)n * n + n + kappa) / ((n + 1.0) * (n + 1.0 + m)) * t;
        term *= ratio;
        sum += term;
        if (cabs(ratio) < 1.0 && cabs(term) < 1e-18 * cabs(sum)) break;
    }
    return sum;
}

/* the continuation about t = 1 (as green_G01_far), g = 1/(Gamma(a) Gamma(b)) = -sin(pi lambda)/pi */
static void greenc_G01_far(double complex kappa, double u, double complex* G0, double complex* G1)
{
    const double complex lam = greenc_lambda(kappa);
    const double complex g = -csin(M_PI * lam) / M_PI;
    const double L = log(u);
    const double euler = 0.57721566490153286061;
    double complex c = 1.0, d = 1.0, s0 = 0.0, s1 = 0.0;
    double uk = 1.0, psi_k1 = -euler;
    for (int k = 0; k < 100000; ++k) {
        const double psi_k2 = psi_k1 + 1.0 / (k + 1.0);
        const double complex pp0 = cdigamma(-lam + k) + cdigamma(lam + 1.0 + k);
        const double complex pp1 = cdigamma(-lam + k + 1.0) + cdigamma(lam + 2.0 + k);
        const double complex t0 = c * uk * (L - 2.0 * psi_k1 + pp0);
        const double complex t1 = d * uk * (L - psi_k1 - psi_k2 + pp1);
        s0 += t0;
        s1 += t1;
        const double dk = k;
        const double complex rc = (dk * dk + dk + kappa) / ((dk + 1.0) * (dk + 1.0));
        c *= rc;
        d *= ((dk + 1.0) * (dk + 1.0) + (dk + 1.0) + kappa) / ((dk + 1.0) * (dk + 2.0));
        uk *= u;
        psi_k1 = psi_k2;
        if (k > 4 && cabs(t0) < 1e-18 * cabs(s0) && cabs(t1) < 1e-18 * cabs(s1) && cabs(rc) * u < 0.9) break;
    }
    *G0 = -g * s0;
    *G1 = g / kappa + g * u * s1;
}

/* G_0 .. G_{m_top} at x (s = sin theta), as green_G_all with |kappa| in the switch rule */
static void greenc_G_all(int m_top, double complex kappa, double x, double s, double complex* G)
{
    if (x >= 0.0) {
        const double t = s * s / (2.0 * (1.0 + x));
        for (int m = 0; m <= m_top; ++m) G[m] = greenc_G_series(m, kappa, t);
        return;
    }
    const double u = s * s / (2.0 * (1.0 - x));
    double complex g0, g1;
    if (u * (cabs(kappa) + 1.0) <= 0.5) {
        greenc_G01_far(kappa, u, &g0, &g1);
    } else {
        g0 = greenc_G_series(0, kappa, 1.0 - u);
        g1 = greenc_G_series(1, kappa, 1.0 - u);
    }
    G[0] = g0;
    if (m_top >= 1) G[1] = g1;
    const double opx = 2.0 * u, omx = 1.0 - x;
    for (int k = 0; k + 2 <= m_top; ++k) {
        const double complex q = (k + 1.0) * (k + 1.0) + (k + 1.0) + kappa;
        G[k + 2] = (k + 1.0) * (k + 2.0) / q * (opx / omx) * (G[k] - 2.0 * x / opx * G[k + 1]);
    }
}

/* G_m and G_{m+1} at x: the series alone for x >= 0, else the recurrence from G_0, G_1 */
static void greenc_G_pair(int m, double complex kappa, double x, double s, double complex* out)
{
    if (x >= 0.0) {
        const double t = s * s / (2.0 * (1.0 + x));
        out[0] = greenc_G_series(m, kappa, t);
        out[1] = greenc_G_series(m + 1, kappa, t);
        return;
    }
    double complex* G = (double complex*)malloc(sizeof(double complex) * (m + 2));
    greenc_G_all(m + 1, kappa, x, s, G);
    out[0] = G[m];
    out[1] = G[m + 1];
    free(G);
}

/* G_m at x for complex kappa = kre + i kim: out[0] = Re, out[1] = Im. */
void orc_greenc_G(int m, double kre, double kim, double x, double s, double* out)
{
    double complex* G = (double complex*)malloc(sizeof(double complex) * (m + 1));
    greenc_G_all(m, kre + I * kim, x, s, G);
    out[0] = creal(G[m]);
    out[1] = cimag(G[m]);
    free(G);
}

/* J^m(z1, z2) of order 2 for the pair alpha +- i beta in the basis (g, U g); kap = {alpha, beta}. */
void orc_jblock_green2c(int m, const double* kap, double z1, double s1, double z2, double s2, double* J)
{
    const int swap = z1 > z2;
    if (swap) {
        double t = z1; z1 = z2; z2 = t;
        t = s1; s1 = s2; s2 = t;
    }
    const double complex kappa = kap[0] + I * kap[1];
    double complex gn[2], gp[2];
    greenc_G_pair(m, kappa, -z1, s1, gn);
    greenc_G_pair(m, kappa, z2, s2, gp);
    /* (Pi_m / m!^2) w^m / (-4 sin pi lambda), w as in green_J_scale */
    double complex ratio = 1.0;
    for (int k = 1; k <= m; ++k) ratio *= ((double)k * k - k + kappa) / ((double)k * k);
    double wm = 1.0;
    const double l1p = z1 >= 0.0 ? log1p(z1) : log(s1 * s1 / (1.0 - z1));
    const double l1m = z1 >= 0.0 ? log(s1 * s1 / (1.0 + z1)) : log1p(-z1);
    const double l2p = z2 >= 0.0 ? log1p(z2) : log(s2 * s2 / (1.0 - z2));
    const double l2m = z2 >= 0.0 ? log(s2 * s2 / (1.0 + z2)) : log1p(-z2);
    if (z1 != z2 && m > 0) wm = exp(0.5 * m * (l1p + l2m - l1m - l2p));
    const double complex lam = greenc_lambda(kappa);
    const double complex b1 = I / (2.0 * kap[1]);
    const double complex sc = b1 * ratio * wm / (-4.0 * csin(M_PI * lam));
    const double r1 = exp(0.5 * (l1p - l1m)), r2 = exp(0.5 * (l2m - l2p));
    const double complex a = ((double)m * m + m + kappa) / (m + 1.0);
    const double complex u[2] = {gn[0], -a * r1 * gn[1]};
    const double complex v[2] = {gp[0], a * r2 * gp[1]};
    double K[4];
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) K[p * 2 + q] = 2.0 * creal(sc * u[p] * v[q]);
    if (swap) {
        J[0] = K[0]; J[1] = K[2]; J[2] = K[1]; J[3] = K[3];
    } else {
        for (int i = 0; i < 4; ++i) J[i] = K[i];
    }
}

/* The same with z1 = cos(theta1), z2 = cos(theta2). */
void orc_jblock(int order, int m, int ell_max, const double* C, double theta1, double theta2,
                double* J)
{
    orc_jblock_zs(order, m, ell_max, C, cos(theta1), sin(theta1), cos(theta2), sin(theta2), J);
}

/* ------------------------------------------------------------------------- */
/* Thresholded Cholesky of an equilibrated symmetric M x M matrix X:           */
/* X ~= G G^T with G lower triangular, positive kept pivots.  A pivot that is   */
/* not above ORC_TAU is dropped: its column of G is zero and kept[j] = 0.       */
/* ------------------------------------------------------------------------- */
static void thr_chol(int M, const double* X, double* G, int* kept)
{
    for (int i = 0; i < M * M; ++i) G[i] = 0.0;
    for (int j = 0; j < M; ++j) {
        double d = X[j * M + j];
        for (int k = 0; k < j; ++k) d -= G[j * M + k] * G[j * M + k];
        if (!(d > ORC_TAU)) { kept[j] = 0; continue; }
        kept[j] = 1;
        double gjj = sqrt(d);
        G[j * M + j] = gjj;
        for (int i = j + 1; i < M; ++i) {
            double v = X[i * M + j];
            for (int k = 0; k < j; ++k) v -= G[i * M + k] * G[j * M + k];
            G[i * M + j] = v / gjj;
        }
    }
}

/* Start factor, eq. (state_initial): B_eq B_eq^T = J(s,s). */
void orc_start_factor(int M, const double* Kss, double* Beq)
{
    double d[ORC_MAXM], R[ORC_MAXM * ORC_MAXM], G[ORC_MAXM * ORC_MAXM];
    int kept[ORC_MAXM];
    for (int p = 0; p < M; ++p) d[p] = Kss[p * M + p] > ORC_TINY ? 1.0 / sqrt(Kss[p * M + p]) : 0.0;
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q) R[p * M + q] = d[p] * Kss[p * M + q] * d[q];
    thr_chol(M, R, G, kept);
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q)
            Beq[p * M + q] = d[p] > 0.0 ? sqrt(Kss[p * M + p]) * G[p * M + q] : 0.0;
}

/* One conditional step a -> b, eqs. (trans_matrix) and (innov_matrix):        */
/*   A = J(b,a) J(a,a)^+,   S = J(b,b) - A J(a,b),   B B^T = S,                 */
/* where Kba[p*M+q] = E[x_b,p x_a,q].  Both sides are first equilibrated by     */
/* the block diagonals, so the algebra runs on correlations.                   */
void orc_step_factors(int M, const double* Kaa, const double* Kbb, const double* Kba,
                      double* A, double* B)
{
    double da[ORC_MAXM], db[ORC_MAXM];
    double Raa[ORC_MAXM * ORC_MAXM], Rbb[ORC_MAXM * ORC_MAXM], Rba[ORC_MAXM * ORC_MAXM];
    double G[ORC_MAXM * ORC_MAXM], At[ORC_MAXM * ORC_MAXM], St[ORC_MAXM * ORC_MAXM];
    double Q[ORC_MAXM * ORC_MAXM], H[ORC_MAXM * ORC_MAXM], e[ORC_MAXM];
    int kept[ORC_MAXM], kept2[ORC_MAXM];

    for (int p = 0; p < M; ++p) {
        da[p] = Kaa[p * M + p] > ORC_TINY ? 1.0 / sqrt(Kaa[p * M + p]) : 0.0;
        db[p] = Kbb[p * M + p] > ORC_TINY ? 1.0 / sqrt(Kbb[p * M + p]) : 0.0;
    }
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q) {
            Raa[p * M + q] = da[p] * Kaa[p * M + q] * da[q];
            Rbb[p * M + q] = db[p] * Kbb[p * M + q] * db[q];
            Rba[p * M + q] = db[p] * Kba[p * M + q] * da[q];
        }
    thr_chol(M, Raa, G, kept);

    /* With Raa = G G^T on the kept pivots, eq. (innov_matrix) reads
       St = Rbb - (Rba G^-T)(Rba G^-T)^T and eq. (trans_matrix) At = (Rba G^-T) G^-1:
       Y = Rba G^-T by forward substitution (row i of Y solves G y = Rba[i,:]^T), then
       At = Y G^-1 by back substitution; this keeps rounding at eps/sqrt(pivot) instead
       of the eps/pivot of an explicit inverse. */
    double Y[ORC_MAXM * ORC_MAXM];
    for (int i = 0; i < M; ++i) {
        double u[ORC_MAXM];
        for (int j = 0; j < M; ++j) {               /* forward: G y = v */
            if (!kept[j]) { Y[i * M + j] = 0.0; continue; }
            double v = Rba[i * M + j];
            for (int k = 0; k < j; ++k) if (kept[k]) v -= G[j * M + k] * Y[i * M + k];
            Y[i * M + j] = v / G[j * M + j];
        }
        for (int j = M - 1; j >= 0; --j) {          /* backward: G^T u = y */
            if (!kept[j]) { u[j] = 0.0; continue; }
            double v = Y[i * M + j];
            for (int k = j + 1; k < M; ++k) if (kept[k]) v -= G[k * M + j] * u[k];
            u[j] = v / G[j * M + j];
        }
        for (int j = 0; j < M; ++j) At[i * M + j] = u[j];
    }
    /* St = Rbb - Y Y^T (symmetric by construction) */
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q) {
            double v = Rbb[p * M + q];
            for (int k = 0; k < M; ++k) v -= Y[p * M + k] * Y[q * M + k];
            St[p * M + q] = v;
        }
    /* B~ = chol(St) with its own equilibration; a relative conditional variance
       not above ORC_TAU is treated as zero */
    for (int p = 0; p < M; ++p) e[p] = St[p * M + p] > ORC_TAU ? 1.0 / sqrt(St[p * M + p]) : 0.0;
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q) Q[p * M + q] = e[p] * St[p * M + q] * e[q];
    thr_chol(M, Q, H, kept2);
    /* undo the equilibration */
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q) {
            double sb = db[p] > 0.0 ? sqrt(Kbb[p * M + p]) : 0.0;
            A[p * M + q] = sb * At[p * M + q] * da[q];
            B[p * M + q] = e[p] > 0.0 ? sb * H[p * M + q] / e[p] : 0.0;
        }
}

/* ------------------------------------------------------------------------- */
/* Factor-set bookkeeping.  Factor set j of mode m:                            */
/*   even n_theta (s = n/2 - 1):  j = 0 start at ring s; j = 1 crossing s -> s+1; */
/*                                j >= 2 north step (s-j+2) -> (s-j+1).        */
/*   odd n_theta  (s = (n-1)/2):  j = 0 start at the equator ring s;           */
/*                                j >= 1 north step (s-j+1) -> (s-j).          */
/* The south half reuses set j conjugated by D (mirror z -> -z).               */
/* ------------------------------------------------------------------------- */
int orc_n_sets(int n_theta) { return (n_theta % 2 == 0) ? n_theta / 2 + 1 : (n_theta + 1) / 2; }
int orc_start_ring(int n_theta) { return (n_theta % 2 == 0) ? n_theta / 2 - 1 : (n_theta - 1) / 2; }
int orc_m_top(int ell_max, int n_phi)
{
    int m = n_phi / 2 - 1;
    return ell_max < m ? ell_max : m;
}

/* Ring pair (a, b) of factor set j in the north chain (b = s+1 for the crossing). */
static void set_rings(int n_theta, int j, int* a, int* b)
{
    int s = orc_start_ring(n_theta);
    if (j == 0) { *a = *b = s; return; }
    if (n_theta % 2 == 0) {
        if (j == 1) { *a = s; *b = s + 1; return; }
        *a = s - j + 2; *b = s - j + 1;
    } else {
        *a = s - j + 1; *b = s - j;
    }
}

/* ------------------------------------------------------------------------- */
/* Alg. 1 for the modes listed in `modes` (each <= m_top) and factor sets       */
/* j = 0..n_sets-1.  A and B are [n_sets][n_modes][M][M] (row-major, B lower    */
/* triangular); for j = 0, A = 0 and B = B_eq.  n_sets may be smaller than      */
/* orc_n_sets(n_theta) to cover only the rings nearest the start.              */
/* zgrid: the ring values z_0 > z_1 > ... > z_{n-1} of Alg. 1's grid argument,  */
/* with sin(theta) = sqrt((1 - z)(1 + z)); NULL selects the ring centres.       */
/* south = 0: the northern sets (start, crossing for even n_theta, then the     */
/* steps towards ring 0); south = 1: the same sets for the southern walk in     */
/* its own (true) coordinates: start, crossing, then the steps (s+j-1) -> (s+j) */
/* towards ring n-1.                                                           */
/* ------------------------------------------------------------------------- */
static int grid_ok(const double* zgrid, int n_theta, int symmetric)
{
    for (int i = 0; i < n_theta; ++i) {
        if (!(zgrid[i] > -1.0 && zgrid[i] < 1.0)) return 0;
        if (i > 0 && !(zgrid[i] < zgrid[i - 1])) return 0;
        if (symmetric && zgrid[n_theta - 1 - i] != -zgrid[i]) return 0;
    }
    return 1;
}

/* basis 0: value and z-derivatives; 1: (g, U g) of Sec. 3 (order 2); 2: the Green's   */
/* function of Sec. 3 at order 1, C then holding the single kappa (no band limit);     */
/* 3: the Green's functions at order 2 in the basis (g, U g), C holding two distinct   */
/* kappa; 4: the same for the complex-conjugate pair C[0] +- i C[1] (C[1] > 0).        */
static void jblock_basis(int order, int basis, int m, int ell_max, const double* C, double z1, double s1, double z2,
                         double s2, double* J)
{
    if (basis == 2)
        orc_jblock_green(m, C[0], z1, s1, z2, s2, J);
    else if (basis == 3)
        orc_jblock_green2(m, C, z1, s1, z2, s2, J);
    else if (basis == 4)
        orc_jblock_green2c(m, C, z1, s1, z2, s2, J);
    else if (basis == 1)
        orc_jblock_zs_u(m, ell_max, C, z1, s1, z2, s2, J);
    else
        orc_jblock_zs(order, m, ell_max, C, z1, s1, z2, s2, J);
}

static void ring_value(int n_theta, const double* zgrid, int i, double* z, double* s)
{
    if (zgrid) {
        *z = zgrid[i];
        *s = sqrt((1.0 - *z) * (1.0 + *z));
    } else {
        orc_ring_zs(n_theta, i, z, s);
    }
}

static void setup_sets(int order, int ell_max, const double* C, int n_theta, const double* zgrid, int n_sets,
                       const int* modes, int n_modes, int south, int basis, double* A, double* B)
{
    int MM = order * order;
    const int s = orc_start_ring(n_theta);
    const int j0 = (n_theta % 2 == 0) ? 2 : 1;
    /* basis 2: G_m(z_i) and G_m(-z_i) of every ring, tabulated once ([ring][m]) */
    double *Gp = NULL, *Gn = NULL;
    int mt = 0;
    if (basis == 2) {
        for (int i = 0; i < n_modes; ++i) mt = modes[i] > mt ? modes[i] : mt;
        Gp = (double*)malloc(sizeof(double) * (size_t)n_theta * (mt + 1));
        Gn = (double*)malloc(sizeof(double) * (size_t)n_theta * (mt + 1));
#pragma omp parallel for schedule(dynamic, 1)
        for (int i = 0; i < n_theta; ++i) {
            double zi, si;
            ring_value(n_theta, zgrid, i, &zi, &si);
            green_G_all(mt, C[0], zi, si, Gp + (size_t)i * (mt + 1));
            green_G_all(mt, C[0], -zi, si, Gn + (size_t)i * (mt + 1));
        }
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_modes; ++i) {
        int m = modes[i];
        double Kaa[ORC_MAXM * ORC_MAXM], Kbb[ORC_MAXM * ORC_MAXM], Kba[ORC_MAXM * ORC_MAXM];
        for (int j = 0; j < n_sets; ++j) {
            int a, b;
            if (south && j >= j0) {
                a = s + j - 1;
                b = s + j;
            } else {
                set_rings(n_theta, j, &a, &b);
            }
            double za, sa, zb, sb;
            ring_value(n_theta, zgrid, a, &za, &sa);
            ring_value(n_theta, zgrid, b, &zb, &sb);
            double* Aj = A + ((size_t)j * n_modes + i) * MM;
            double* Bj = B + ((size_t)j * n_modes + i) * MM;
            if (basis == 2) {
                /* J(x, y) = scale(x <= y) G_m(-x) G_m(y) for the lower ring value x */
                const size_t w = (size_t)mt + 1;
                Kaa[0] = green_J_scale(m, C[0], za, sa, za, sa) * Gn[a * w + m] * Gp[a * w + m];
                if (j == 0) {
                    Aj[0] = 0.0;
                    orc_start_factor(1, Kaa, Bj);
                    continue;
                }
                Kbb[0] = green_J_scale(m, C[0], zb, sb, zb, sb) * Gn[b * w + m] * Gp[b * w + m];
                if (za <= zb)
                    Kba[0] = green_J_scale(m, C[0], za, sa, zb, sb) * Gn[a * w + m] * Gp[b * w + m];
                else
                    Kba[0] = green_J_scale(m, C[0], zb, sb, za, sa) * Gn[b * w + m] * Gp[a * w + m];
                orc_step_factors(1, Kaa, Kbb, Kba, Aj, Bj);
                continue;
            }
            if (j == 0) {
                jblock_basis(order, basis, m, ell_max, C, za, sa, za, sa, Kaa);
                for (int k = 0; k < MM; ++k) Aj[k] = 0.0;
                orc_start_factor(order, Kaa, Bj);
                continue;
            }
            jblock_basis(order, basis, m, ell_max, C, za, sa, za, sa, Kaa);
            jblock_basis(order, basis, m, ell_max, C, zb, sb, zb, sb, Kbb);
            jblock_basis(order, basis, m, ell_max, C, zb, sb, za, sa, Kba);
            orc_step_factors(order, Kaa, Kbb, Kba, Aj, Bj);
        }
    }
    free(Gp);
    free(Gn);
}

/* Symmetric grids (the south is the mirror of the north, the remark after Alg. 1). */
int orc_setup_modes_z(int order, int ell_max, const double* C, int n_theta, const double* zgrid,
                      int n_sets, const int* modes, int n_modes, double* A, double* B)
{
    if (order < 1 || order > ORC_MAXM || n_theta < 2 || ell_max < 0) return -1;
    if (zgrid && !grid_ok(zgrid, n_theta, 1)) return -1;
    int total = orc_n_sets(n_theta);
    if (n_sets > total) n_sets = total;
    setup_sets(order, ell_max, C, n_theta, zgrid, n_sets, modes, n_modes, 0, 0, A, B);
    return 0;
}

/* The same in the basis (g, U g) of Sec. 3 (order 2; basis 1), or the z-derivative one
   (basis 0). */
/* The Green's-function setups (bases 2-4) evaluate G_m and sin(pi lambda), which grow like
 * exp(pi sqrt|kappa|), and their products, in FP64: |kappa| is held to ORC_GREEN_MAX_KAPPA (G and
 * |sin pi lambda| then stay below about 1e137; near |kappa| = 1e5 the products leave the FP64 range). */
#define ORC_GREEN_MAX_KAPPA 1e4
/* below 1e-5 the continuation about t = 1 loses digits as lambda -> 0 (5e-11 at kappa = 1e-7) */
#define ORC_GREEN_MIN_KAPPA 1e-5
static int green_kappa_ok(int order, int basis, const double* C)
{
    /* the pair alpha +- i beta: the series' terms n^2 + n + kappa turn sign (alpha < 0) or rotate
     * (beta large) and cancel; alpha >= -50 and beta <= 1000 keep G_m within about 1e-11 */
    if (basis == 4)
        return hypot(C[0], C[1]) <= ORC_GREEN_MAX_KAPPA && hypot(C[0], C[1]) >= ORC_GREEN_MIN_KAPPA && C[0] >= -50.0 &&
               C[1] <= 1000.0;
    for (int i = 0; i < order; ++i)
        if (!(C[i] <= ORC_GREEN_MAX_KAPPA) || !(C[i] >= ORC_GREEN_MIN_KAPPA)) return 0;
    /* two real roots: the weights +-1/(kappa_2 - kappa_1) cancel about log10(kappa / |kappa_2 -
     * kappa_1|) digits, so the roots keep a relative distance of 1e-3 (a field then moves by 5e-11
     * when kappa moves by one unit in the last place) */
    if (basis == 3 && !(fabs(C[1] - C[0]) >= 1e-3 * fmax(C[0], C[1]))) return 0;
    return 1;
}

int orc_setup_modes_zb(int order, int basis, int ell_max, const double* C, int n_theta, const double* zgrid,
                       int n_sets, const int* modes, int n_modes, double* A, double* B)
{
    if (order < 1 || order > ORC_MAXM || n_theta < 2 || ell_max < 0) return -1;
    if (basis != 0 && !(basis == 1 && order == 2) && !(basis == 2 && order == 1 && C[0] > 0.0) &&
        !(basis == 3 && order == 2 && C[0] > 0.0 && C[1] > 0.0 && C[0] != C[1]) &&
        !(basis == 4 && order == 2 && C[1] > 0.0 && isfinite(C[0]) && isfinite(C[1])))
        return -1;
    if (basis >= 2 && !green_kappa_ok(order, basis, C)) return -1;
    if (zgrid && !grid_ok(zgrid, n_theta, 1)) return -1;
    int total = orc_n_sets(n_theta);
    if (n_sets > total) n_sets = total;
    setup_sets(order, ell_max, C, n_theta, zgrid, n_sets, modes, n_modes, 0, basis, A, B);
    return 0;
}

/* Any strictly decreasing grid in (-1, 1): the northern sets (A, B) and the sets of */
/* the southern walk in true coordinates (As, Bs), same shapes; basis as in         */
/* orc_setup_modes_zb.                                                           */
int orc_setup_modes_asym_b(int order, int basis, int ell_max, const double* C, int n_theta, const double* zgrid,
                           int n_sets, const int* modes, int n_modes, double* A, double* B, double* As, double* Bs)
{
    if (order < 1 || order > ORC_MAXM || n_theta < 2 || ell_max < 0 || !zgrid) return -1;
    if (basis != 0 && !(basis == 1 && order == 2)) return -1;
    if (!grid_ok(zgrid, n_theta, 0)) return -1;
    int total = orc_n_sets(n_theta);
    if (n_sets > total) n_sets = total;
    setup_sets(order, ell_max, C, n_theta, zgrid, n_sets, modes, n_modes, 0, basis, A, B);
    setup_sets(order, ell_max, C, n_theta, zgrid, n_sets, modes, n_modes, 1, basis, As, Bs);
    return 0;
}

int orc_setup_modes_asym(int order, int ell_max, const double* C, int n_theta, const double* zgrid, int n_sets,
                         const int* modes, int n_modes, double* A, double* B, double* As, double* Bs)
{
    return orc_setup_modes_asym_b(order, 0, ell_max, C, n_theta, zgrid, n_sets, modes, n_modes, A, B, As, Bs);
}

/* The same on the ring-centre grid. */
int orc_setup_modes(int order, int ell_max, const double* C, int n_theta, int n_sets,
                    const int* modes, int n_modes, double* A, double* B)
{
    return orc_setup_modes_z(order, ell_max, C, n_theta, NULL, n_sets, modes, n_modes, A, B);
}

/* Alg. 1 for every mode m = 0..m_top (zgrid as in orc_setup_modes_z). */
int orc_setup_z(int order, int ell_max, const double* C, int n_theta, const double* zgrid, int n_phi,
                int n_sets, double* A, double* B)
{
    int m_top = orc_m_top(ell_max, n_phi);
    int* modes = (int*)malloc(sizeof(int) * (m_top + 1));
    if (!modes) return -1;
    for (int m = 0; m <= m_top; ++m) modes[m] = m;
    int rc = orc_setup_modes_z(order, ell_max, C, n_theta, zgrid, n_sets, modes, m_top + 1, A, B);
    free(modes);
    return rc;
}

int orc_setup(int order, int ell_max, const double* C, int n_theta, int n_phi, int n_sets,
              double* A, double* B)
{
    return orc_setup_z(order, ell_max, C, n_theta, NULL, n_phi, n_sets, A, B);
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of            */
/*   (c0,c1,c2,c3) -> (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0)) */
/* with A = 0xD2511F53, B = 0xCD9E8D57, and the key bumped by the Weyl          */
/* constants (0x9E3779B9, 0xBB67AE85) between rounds.                          */
/* ------------------------------------------------------------------------- */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t pa = (uint64_t)0xD2511F53u * c0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Normal xi_q feeding ring `ring` of chain (m, part) of the field with key
   `key`; Box-Muller in FP64 on the words of one Philox block. */
double orc_normal(uint64_t key, int m, int part, int ring, int order, int q)
{
    int idx = ring * order + q;
    uint32_t ctr[4] = {(uint32_t)(idx / 4), (uint32_t)m, (uint32_t)part, 0u};
    uint32_t k[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
    uint32_t w[4];
    orc_philox(ctr, k, w);
    int word = idx % 4;
    int pair = word / 2;
    double u0 = ((double)w[2 * pair] + 0.5) * ldexp(1.0, -32);
    double u1 = ((double)w[2 * pair + 1] + 0.5) * ldexp(1.0, -32);
    double r = sqrt(-2.0 * log(u0));
    return (word % 2 == 0) ? r * cos(2.0 * M_PI * u1) : r * sin(2.0 * M_PI * u1);
}

/* ------------------------------------------------------------------------- */
/* Alg. 2, chain part: for every field f (key seed+f), mode m and part, draw    */
/* the start state at ring s (eq. (state_initial)) and run eq. (state_space)    */
/* outward in both hemispheres, for the modes listed in `modes` with factors     */
/* [n_sets][n_modes][M][M] as orc_setup_modes writes them.                      */
/* g is [count][n_theta][n_modes][2] (Re, Im).  Only factor sets j < n_sets are  */
/* used; rings they do not reach stay NaN.                                      */
/* ------------------------------------------------------------------------- */
int orc_sample_modes_list_south(int order, int n_theta, const int* modes, int n_modes, int n_sets,
                                const double* A, const double* B, const double* As, const double* Bs,
                                uint64_t seed, int count, double* g)
{
    const int M = order, MM = order * order;
    const int s = orc_start_ring(n_theta);
    const int even = (n_theta % 2 == 0);
    const size_t row = (size_t)n_modes * 2;
    for (size_t i = 0; i < (size_t)count * n_theta * row; ++i) g[i] = NAN;
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int f = 0; f < count; ++f)
        for (int i = 0; i < n_modes; ++i) {
            const int m = modes[i];
            uint64_t key = seed + (uint64_t)f;
            double* gf = g + (size_t)f * n_theta * row;
            for (int part = 0; part < 2; ++part) {
                if (m == 0 && part == 1) {                 /* g_0 is real */
                    for (int r = 0; r < n_theta; ++r) gf[r * row + 2 * i + 1] = 0.0;
                    continue;
                }
                const double sc = (m == 0) ? 1.0 : 1.0 / sqrt(2.0);
                double xs[ORC_MAXM], x[ORC_MAXM], xn[ORC_MAXM], w[ORC_MAXM];
                /* start ring s */
                const double* B0 = B + (size_t)i * MM;
                for (int q = 0; q < M; ++q) w[q] = orc_normal(key, m, part, s, M, q);
                for (int p = 0; p < M; ++p) {
                    xs[p] = 0.0;
                    for (int q = 0; q < M; ++q) xs[p] += sc * B0[p * M + q] * w[q];
                }
                gf[(size_t)s * row + 2 * i + part] = xs[0];
                /* north: rings s-1 .. 0 */
                for (int p = 0; p < M; ++p) x[p] = xs[p];
                for (int j = even ? 2 : 1; j < n_sets; ++j) {
                    int r = even ? s - j + 1 : s - j;
                    const double* Aj = A + ((size_t)j * n_modes + i) * MM;
                    const double* Bj = B + ((size_t)j * n_modes + i) * MM;
                    for (int q = 0; q < M; ++q) w[q] = orc_normal(key, m, part, r, M, q);
                    for (int p = 0; p < M; ++p) {
                        xn[p] = 0.0;
                        for (int q = 0; q < M; ++q) xn[p] += Aj[p * M + q] * x[q] + sc * Bj[p * M + q] * w[q];
                    }
                    for (int p = 0; p < M; ++p) x[p] = xn[p];
                    gf[(size_t)r * row + 2 * i + part] = x[0];
                }
                /* south: crossing (even n) then the steps towards ring n-1: the northern
                   sets mirrored with D A D, D B D, or the southern sets As, Bs as given */
                for (int p = 0; p < M; ++p) x[p] = xs[p];
                int r = s;
                int j0 = 1;
                if (even) {
                    if (n_sets < 2) continue;
                    const double* Aj = A + ((size_t)1 * n_modes + i) * MM;
                    const double* Bj = B + ((size_t)1 * n_modes + i) * MM;
                    r = s + 1;
                    for (int q = 0; q < M; ++q) w[q] = orc_normal(key, m, part, r, M, q);
                    for (int p = 0; p < M; ++p) {
                        xn[p] = 0.0;
                        for (int q = 0; q < M; ++q) xn[p] += Aj[p * M + q] * x[q] + sc * Bj[p * M + q] * w[q];
                    }
                    for (int p = 0; p < M; ++p) x[p] = xn[p];
                    gf[(size_t)r * row + 2 * i + part] = x[0];
                    j0 = 2;
                }
                for (int j = j0; j < n_sets; ++j) {
                    r += 1;
                    const double* Aj = (As ? As : A) + ((size_t)j * n_modes + i) * MM;
                    const double* Bj = (Bs ? Bs : B) + ((size_t)j * n_modes + i) * MM;
                    for (int q = 0; q < M; ++q) w[q] = orc_normal(key, m, part, r, M, q);
                    for (int p = 0; p < M; ++p) {
                        xn[p] = 0.0;
                        for (int q = 0; q < M; ++q) {
                            /* mirrored: D X D of the northern set; own sets: as they are */
                            double sgn = (As || (p + q) % 2 == 0) ? 1.0 : -1.0;
                            xn[p] += sgn * (Aj[p * M + q] * x[q] + sc * Bj[p * M + q] * w[q]);
                        }
                    }
                    for (int p = 0; p < M; ++p) x[p] = xn[p];
                    gf[(size_t)r * row + 2 * i + part] = x[0];
                }
            }
        }
    return 0;
}

/* Symmetric grids: the south mirrors the northern sets. */
int orc_sample_modes_list(int order, int n_theta, const int* modes, int n_modes, int n_sets,
                          const double* A, const double* B, uint64_t seed, int count, double* g)
{
    return orc_sample_modes_list_south(order, n_theta, modes, n_modes, n_sets, A, B, NULL, NULL, seed, count, g);
}

/* Chains for every mode m = 0..m_top: g is [count][n_theta][m_top+1][2]. */
int orc_sample_modes(int order, int n_theta, int m_top, int n_sets, const double* A,
                     const double* B, uint64_t seed, int count, double* g)
{
    int* modes = (int*)malloc(sizeof(int) * (m_top + 1));
    if (!modes) return -1;
    for (int m = 0; m <= m_top; ++m) modes[m] = m;
    int rc = orc_sample_modes_list(order, n_theta, modes, m_top + 1, n_sets, A, B, seed, count, g);
    free(modes);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Alg. 2, last step: inverse DFT along phi for rings [r0, r1) of each field:   */
/*   T(z_i, phi_j) = g_0 + 2 sum_{m=1}^{m_top} (Re g_m cos(m phi_j)             */
/*                                              - Im g_m sin(m phi_j)),         */
/* phi_j = 2 pi j / n_phi, twiddles indexed exactly by (m j) mod n_phi.         */
/* g is [count][n_theta][m_top+1][2]; T is [count][r1-r0][n_phi].               */
/* ------------------------------------------------------------------------- */
int orc_dft(int n_theta, int n_phi, int m_top, int count, int r0, int r1, const double* g, double* T)
{
    double* cs = (double*)malloc(sizeof(double) * 2 * n_phi);
    if (!cs) return -1;
    for (int k = 0; k < n_phi; ++k) {
        cs[2 * k] = cos(2.0 * M_PI * k / n_phi);
        cs[2 * k + 1] = sin(2.0 * M_PI * k / n_phi);
    }
    const size_t row = (size_t)(m_top + 1) * 2;
    const int nr = r1 - r0;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int f = 0; f < count; ++f)
        for (int i = r0; i < r1; ++i) {
            const double* gr = g + ((size_t)f * n_theta + i) * row;
            double* Tr = T + ((size_t)f * nr + (i - r0)) * n_phi;
            for (int j = 0; j < n_phi; ++j) {
                double acc = 0.0;
                for (int m = 1; m <= m_top; ++m) {
                    size_t k = ((size_t)m * j) % (size_t)n_phi;
                    acc += gr[2 * m] * cs[2 * k] - gr[2 * m + 1] * cs[2 * k + 1];
                }
                Tr[j] = gr[0] + 2.0 * acc;
            }
        }
    free(cs);
    return 0;
}

/* Full plain method for convenience: setup + chains + DFT on all rings. */
int orc_sample(int order, int n_theta, int n_phi, int m_top, const double* A, const double* B,
               uint64_t seed, int count, double* g_work, double* T)
{
    int ns = orc_n_sets(n_theta);
    orc_sample_modes(order, n_theta, m_top, ns, A, B, seed, count, g_work);
    return orc_dft(n_theta, n_phi, m_top, count, 0, n_theta, g_work, T);
}

/* ------------------------------------------------------------------------- */
/* Alg. 2's last step on rings that each have their own pixel count n_i and   */
/* first-pixel longitude phi0_i (iso-latitude grids such as HEALPix, Sec. 1): */
/*   T(z_i, phi_ij) = g_0 + 2 sum_{m=1}^{m_top} Re(g_m e^{i m phi_ij}),          */
/*   phi_ij = phi0_i + 2 pi j / n_i,  j < n_i,                                  */
/* the same sum as orc_dft evaluated at each pixel; every mode is kept, also   */
/* those above n_i / 2.  e^{i m phi_ij} = e^{i m phi0_i} e^{2 pi i k / n_i}     */
/* with k = (m j) mod n_i.  g is [count][n_theta][m_top+1][2]; ring i of field  */
/* f goes to T[f * off[n_theta] + off[i] + j], off[] the prefix sums of n_i.    */
/* ------------------------------------------------------------------------- */
int orc_dft_rings(int n_theta, int m_top, int count, const int* n_ring, const double* phi0,
                  const int64_t* off, const double* g, double* T)
{
    const size_t row = (size_t)(m_top + 1) * 2;
    const int64_t total = off[n_theta];
    int bad = 0;
#pragma omp parallel for collapse(2) schedule(dynamic, 1) reduction(| : bad)
    for (int f = 0; f < count; ++f)
        for (int i = 0; i < n_theta; ++i) {
            const int n = n_ring[i];
            const double* gr = g + ((size_t)f * n_theta + i) * row;
            double* Tr = T + (size_t)f * total + off[i];
            double* cs = (double*)malloc(sizeof(double) * 2 * (n + m_top + 1));
            if (!cs) { bad = 1; continue; }
            double* ph = cs + 2 * n;   /* e^{i m phi0}, m <= m_top */
            for (int k = 0; k < n; ++k) {
                cs[2 * k] = cos(2.0 * M_PI * k / n);
                cs[2 * k + 1] = sin(2.0 * M_PI * k / n);
            }
            for (int m = 0; m <= m_top; ++m) {
                ph[2 * m] = cos(m * phi0[i]);
                ph[2 * m + 1] = sin(m * phi0[i]);
            }
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int m = 1; m <= m_top; ++m) {
                    size_t k = ((size_t)m * j) % (size_t)n;
                    double c = ph[2 * m] * cs[2 * k] - ph[2 * m + 1] * cs[2 * k + 1];
                    double s = ph[2 * m + 1] * cs[2 * k] + ph[2 * m] * cs[2 * k + 1];
                    acc += gr[2 * m] * c - gr[2 * m + 1] * s;
                }
                Tr[j] = gr[0] + 2.0 * acc;
            }
            free(cs);
        }
    return bad ? -1 : 0;
}
