// FP64 setup on the GPU: spectrum, cross-covariance blocks by Legendre sums, and the
// transition / innovation / start factors of every (mode, ring step)
// (Creasey & Lang, Alg. 1; Lemma 2.1; eqs. (trans_matrix), (innov_matrix), (state_initial)).
#include "green_pair.h"
#include "smf_internal.h"

namespace smf {
namespace {

// ---------------------------------------------------------------- spectrum, eq. (Cl)
__global__ void spectrum_kernel(const double* __restrict__ kappa, int n_kappa,
                                const double* __restrict__ c_explicit, int ell_max,
                                double* __restrict__ C, int* __restrict__ bad)
{
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > ell_max) return;
    double c;
    if (c_explicit) {
        c = c_explicit[l];
    } else {
        double ll = (double)l * (double)(l + 1);
        double den = 1.0;
        for (int i = 0; i < n_kappa; ++i) den *= (kappa[i] + ll);
        c = 1.0 / den;
    }
    // finite and strictly positive, NaN rejected
    if (!(c > 0.0) || !(c <= 1.7976931348623157e308)) atomicOr(bad, 1);
    C[l] = c;
}

// ---------------------------------------------------------------- twiddles
__global__ void twiddle_kernel(int n, double* __restrict__ tw64, float* __restrict__ tw32)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double sn, cs;
    sincospi(2.0 * (double)t / (double)n, &sn, &cs);   // e^{+2 pi i t / n}
    tw64[2 * t] = cs;
    tw64[2 * t + 1] = sn;
    tw32[2 * t] = (float)cs;
    tw32[2 * t + 1] = (float)sn;
}

// ---------------------------------------------------------------- Legendre stream
// Fully normalised L_lm(z) (no Condon-Shortley sign) and dL_lm/dz along l for one ring,
// carried as mantissa pair (p0 = L_{l-1}, p1 = L_l) times 2^e so the sin^m seed cannot
// underflow.  value()/deriv() return plain doubles (0 or subnormal below FP64 range).
struct LegendreStream {
    double z, inv_s2, p0, p1;
    int e;
    __device__ double value() const { return ldexp(p1, e); }
};

constexpr double kUp = 0x1p400;      // rescale unit 2^400
constexpr double kDown = 0x1p-400;

// ---------------------------------------------------------------- factorisations
// Equilibration weight 1/sqrt(d) of a diagonal entry, zero if it is not above kTiny.
__device__ inline double eq_weight(double d) { return d > kTiny ? 1.0 / sqrt(d) : 0.0; }

// Order 1: scalar blocks.  Writes A (transition) and B (innovation sd).
__device__ inline void factors_m1(double kaa, double kbb, double kba, double& A, double& B)
{
    const double da = eq_weight(kaa), db = eq_weight(kbb);
    const double raa = da * kaa * da, rbb = db * kbb * db, rba = db * kba * da;
    // R_aa = g^2; y = R_ba / g; At = y / g; St = R_bb - y^2 (eq. (innov_matrix) via the
    // Cholesky factor of R_aa rather than its inverse)
    const double gaa = (raa > kTau) ? sqrt(raa) : 0.0;
    const double y = gaa > 0.0 ? rba / gaa : 0.0;
    const double at = gaa > 0.0 ? y / gaa : 0.0;
    const double st = rbb - y * y;
    const double e = st > kTau ? 1.0 / sqrt(st) : 0.0;
    const double q = e * st * e;
    const double bt = (e > 0.0 && q > kTau) ? sqrt(q) / e : 0.0;
    const double sb = db > 0.0 ? sqrt(kbb) : 0.0;
    A = sb * at * da;
    B = sb * bt;
}

// Order 1 start: B_eq = sqrt(J(s,s)).
__device__ inline double start_m1(double kss)
{
    const double d = eq_weight(kss);
    const double r = d * kss * d;
    return (d > 0.0 && r > kTau) ? sqrt(kss) * sqrt(r) : 0.0;
}

// Thresholded Cholesky of a symmetric 2x2 (x00, x01, x11) that is already equilibrated.
// Lower factor (g00, g10, g11); a dropped pivot leaves its column zero.
__device__ inline void chol2(double x00, double x01, double x11, double& g00, double& g10,
                             double& g11, bool& k0, bool& k1)
{
    k0 = x00 > kTau;
    g00 = k0 ? sqrt(x00) : 0.0;
    g10 = k0 ? x01 / g00 : 0.0;
    const double piv = x11 - g10 * g10;
    k1 = piv > kTau;
    g11 = k1 ? sqrt(piv) : 0.0;
}

// Order 2 step a -> b.  kaa, kbb symmetric (00, 01, 11); kba full with
// kba[p][q] = E[x_b,p x_a,q].  A row-major 2x2, B lower (b00, b10, b11).
__device__ void factors_m2(const double kaa[3], const double kbb[3], const double kba[4],
                           double A[4], double B[3])
{
    const double da0 = eq_weight(kaa[0]), da1 = eq_weight(kaa[2]);
    const double db0 = eq_weight(kbb[0]), db1 = eq_weight(kbb[2]);
    // equilibrated blocks
    const double r00 = da0 * kaa[0] * da0, r01 = da0 * kaa[1] * da1, r11 = da1 * kaa[2] * da1;
    const double s00 = db0 * kbb[0] * db0, s01 = db0 * kbb[1] * db1, s11 = db1 * kbb[2] * db1;
    const double c00 = db0 * kba[0] * da0, c01 = db0 * kba[1] * da1;
    const double c10 = db1 * kba[2] * da0, c11 = db1 * kba[3] * da1;
    double g00, g10, g11;
    bool k0, k1;
    chol2(r00, r01, r11, g00, g10, g11, k0, k1);
    // With R = G G^T on the kept pivots: Y = C G^-T (row i solves G y = c_i), then
    // At = Y G^-1 and St = S - Y Y^T (eqs. (trans_matrix), (innov_matrix)); rounding
    // grows as eps / g11 rather than the eps / g11^2 of an explicit inverse.  A dropped
    // pivot leaves its column of Y and At zero.
    const double y00 = k0 ? c00 / g00 : 0.0;
    const double y10 = k0 ? c10 / g00 : 0.0;
    const double y01 = k1 ? (c01 - g10 * y00) / g11 : 0.0;
    const double y11 = k1 ? (c11 - g10 * y10) / g11 : 0.0;
    const double t01 = k1 ? y01 / g11 : 0.0;
    const double t11 = k1 ? y11 / g11 : 0.0;
    const double t00 = k0 ? (y00 - t01 * g10) / g00 : 0.0;
    const double t10 = k0 ? (y10 - t11 * g10) / g00 : 0.0;
    const double q00 = s00 - (y00 * y00 + y01 * y01);
    const double q11 = s11 - (y10 * y10 + y11 * y11);
    const double q01 = s01 - (y00 * y10 + y01 * y11);
    // its own equilibration, then the thresholded Cholesky
    const double e0 = q00 > kTau ? 1.0 / sqrt(q00) : 0.0;
    const double e1 = q11 > kTau ? 1.0 / sqrt(q11) : 0.0;
    double h00, h10, h11;
    bool j0, j1;
    chol2(e0 * q00 * e0, e0 * q01 * e1, e1 * q11 * e1, h00, h10, h11, j0, j1);
    // undo both equilibrations
    const double sb0 = db0 > 0.0 ? sqrt(kbb[0]) : 0.0;
    const double sb1 = db1 > 0.0 ? sqrt(kbb[2]) : 0.0;
    A[0] = sb0 * t00 * da0;
    A[1] = sb0 * t01 * da1;
    A[2] = sb1 * t10 * da0;
    A[3] = sb1 * t11 * da1;
    B[0] = e0 > 0.0 ? sb0 * h00 / e0 : 0.0;
    B[1] = e1 > 0.0 ? sb1 * h10 / e1 : 0.0;
    B[2] = e1 > 0.0 ? sb1 * h11 / e1 : 0.0;
}

// Order 2 start: B_eq = chol(J(s,s)) through the equilibrated thresholded Cholesky.
__device__ void start_m2(const double k[3], double B[3])
{
    const double d0 = eq_weight(k[0]), d1 = eq_weight(k[2]);
    double g00, g10, g11;
    bool k0, k1;
    chol2(d0 * k[0] * d0, d0 * k[1] * d1, d1 * k[2] * d1, g00, g10, g11, k0, k1);
    const double s0 = d0 > 0.0 ? sqrt(k[0]) : 0.0;
    const double s1 = d1 > 0.0 ? sqrt(k[2]) : 0.0;
    B[0] = s0 * g00;
    B[1] = s1 * g10;
    B[2] = s1 * g11;
}

// ---------------------------------------------------------------- orders 3 and 4
// Thresholded lower Cholesky of an equilibrated symmetric M x M matrix (row-major): a pivot
// not above kTau is dropped, its column of G stays zero.
template <int M>
__device__ inline void chol_gen(const double (&X)[M * M], double (&G)[M * M], bool (&kept)[M])
{
#pragma unroll
    for (int i = 0; i < M * M; ++i) G[i] = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double d = X[j * M + j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= G[j * M + k] * G[j * M + k];
        kept[j] = d > kTau;
        const double gjj = kept[j] ? sqrt(d) : 0.0;
        G[j * M + j] = gjj;
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            double v = X[i * M + j];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= G[i * M + k] * G[j * M + k];
            G[i * M + j] = kept[j] ? v / gjj : 0.0;
        }
    }
}

// One step a -> b for M >= 3, the same algebra as factors_m2 on M x M blocks: equilibrate,
// J(a,a) = G G^T on the kept pivots, Y = J(b,a) G^-T (forward substitution per row),
// A = Y G^-1 (back substitution), S = J(b,b) - Y Y^T, B = chol(S) after S's own
// equilibration, both equilibrations undone.  Kaa, Kbb, Kba full row-major.
template <int M>
__device__ void factors_gen(const double (&Kaa)[M * M], const double (&Kbb)[M * M], const double (&Kba)[M * M],
                            double (&A)[M * M], double (&B)[M * M])
{
    double da[M], db[M];
#pragma unroll
    for (int p = 0; p < M; ++p) {
        da[p] = eq_weight(Kaa[p * M + p]);
        db[p] = eq_weight(Kbb[p * M + p]);
    }
    double R[M * M], S[M * M], Cba[M * M];
#pragma unroll
    for (int p = 0; p < M; ++p)
#pragma unroll
        for (int q = 0; q < M; ++q) {
            R[p * M + q] = da[p] * Kaa[p * M + q] * da[q];
            S[p * M + q] = db[p] * Kbb[p * M + q] * db[q];
            Cba[p * M + q] = db[p] * Kba[p * M + q] * da[q];
        }
    double G[M * M];
    bool kept[M];
    chol_gen<M>(R, G, kept);
    double Y[M * M], At[M * M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
            double v = Cba[i * M + j];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= G[j * M + k] * Y[i * M + k];
            Y[i * M + j] = kept[j] ? v / G[j * M + j] : 0.0;
        }
#pragma unroll
        for (int j = M - 1; j >= 0; --j) {
            double v = Y[i * M + j];
#pragma unroll
            for (int k = j + 1; k < M; ++k) v -= G[k * M + j] * At[i * M + k];
            At[i * M + j] = kept[j] ? v / G[j * M + j] : 0.0;
        }
    }
#pragma unroll
    for (int p = 0; p < M; ++p)
#pragma unroll
        for (int q = 0; q < M; ++q) {
            double v = S[p * M + q];
#pragma unroll
            for (int k = 0; k < M; ++k) v -= Y[p * M + k] * Y[q * M + k];
            S[p * M + q] = v;
        }
    double e[M];
#pragma unroll
    for (int p = 0; p < M; ++p) e[p] = S[p * M + p] > kTau ? 1.0 / sqrt(S[p * M + p]) : 0.0;
    double Q[M * M], H[M * M];
#pragma unroll
    for (int p = 0; p < M; ++p)
#pragma unroll
        for (int q = 0; q < M; ++q) Q[p * M + q] = e[p] * S[p * M + q] * e[q];
    bool kept2[M];
    chol_gen<M>(Q, H, kept2);
#pragma unroll
    for (int p = 0; p < M; ++p) {
        const double sb = db[p] > 0.0 ? sqrt(Kbb[p * M + p]) : 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) {
            A[p * M + q] = sb * At[p * M + q] * da[q];
            B[p * M + q] = e[p] > 0.0 ? sb * H[p * M + q] / e[p] : 0.0;
        }
    }
}

// Start factor for M >= 3: B_eq = chol(J(s,s)) through the equilibrated thresholded Cholesky.
template <int M>
__device__ void start_gen(const double (&K)[M * M], double (&B)[M * M])
{
    double d[M], R[M * M], G[M * M];
    bool kept[M];
#pragma unroll
    for (int p = 0; p < M; ++p) d[p] = eq_weight(K[p * M + p]);
#pragma unroll
    for (int p = 0; p < M; ++p)
#pragma unroll
        for (int q = 0; q < M; ++q) R[p * M + q] = d[p] * K[p * M + q] * d[q];
    chol_gen<M>(R, G, kept);
#pragma unroll
    for (int p = 0; p < M; ++p)
#pragma unroll
        for (int q = 0; q < M; ++q) B[p * M + q] = d[p] > 0.0 ? sqrt(K[p * M + p]) * G[p * M + q] : 0.0;
}

// ---------------------------------------------------------------- factor kernel
// One thread per (set j, mode m); a 64-lane block holds consecutive sets of one mode, so
// the l loop and its coefficients are uniform across the wave.  Each thread runs the
// Legendre recurrence at its two rings a, b (Sec. 2 definition of L_lm), accumulates
// J(a,a), J(b,b), J(b,a) (Lemma 2.1 and the cross covariances), and factorises.
// zgrid: the ring values of an explicit grid (Alg. 1's grid argument), or null for the
// ring centres.  south: the southern walk's own sets of a grid with no symmetry: set
// j >= j0 is the step (s+j-1) -> (s+j), stored mirrored (D A D, D B D with
// D = diag((-1)^p)) so that the walk applies it to y = D x as it applies the mirrored
// northern sets; sets below j0 (start, crossing) as in the northern table.
// UB (order 2): the state basis (g, U g) of Sec. 3 in place of (g, dg/dz), with
// U_m L_lm = -sqrt((l+m+1)(l-m)) L_{l,m+1} (U maps P^m to P^{m+1}) summed from a second
// Legendre stream of order m+1.
template <int M, bool UB = false>
__global__ __launch_bounds__(64) void factor_kernel(Geometry g, const double* __restrict__ C,
                                                    const double* __restrict__ zgrid, int south,
                                                    double* __restrict__ f64,
                                                    float* __restrict__ f32)
{
    const int j = blockIdx.x * 64 + threadIdx.x;
    const int m = blockIdx.y;
    if (j >= g.n_sets) return;
    const bool mirror = south && j >= (g.even ? 2 : 1);
    int a, b;
    if (mirror) {
        a = g.s + j - 1; b = g.s + j;
    } else if (j == 0) {
        a = b = g.s;
    } else if (g.even) {
        if (j == 1) { a = g.s; b = g.s + 1; }
        else { a = g.s - j + 2; b = g.s - j + 1; }
    } else {
        a = g.s - j + 1; b = g.s - j;
    }
    // z = cos(theta) and sin(theta) through the complementary angle
    // pi/2 - theta = pi (n - 2i - 1) / (2n): the equator ring of an odd grid gets z = 0
    // exactly and mirrored rings get exactly opposite z
    LegendreStream ra, rb;
    double sa, sb;
    if (zgrid) {
        ra.z = zgrid[a];
        rb.z = zgrid[b];
        sa = sqrt((1.0 - ra.z) * (1.0 + ra.z));
        sb = sqrt((1.0 - rb.z) * (1.0 + rb.z));
    } else {
        sincospi((double)(g.n_theta - 2 * a - 1) / (2.0 * g.n_theta), &ra.z, &sa);
        sincospi((double)(g.n_theta - 2 * b - 1) / (2.0 * g.n_theta), &rb.z, &sb);
    }
    ra.inv_s2 = 1.0 / (sa * sa);
    rb.inv_s2 = 1.0 / (sb * sb);
    // sectoral seed L_mm = sqrt((2m+1)/(4pi) prod_k (2k-1)/(2k)) sin^m, built as
    // L_kk = sqrt((2k+1)/(2k)) sin L_{k-1,k-1} from L_00 = 1/sqrt(4 pi)
    double pa = 0.28209479177387814347, pb = pa;   // 1/sqrt(4 pi)
    int ea = 0, eb = 0;
    for (int k = 1; k <= m; ++k) {
        const double f = sqrt((2.0 * k + 1.0) / (2.0 * k));
        pa *= f * sa;
        pb *= f * sb;
        if (fabs(pa) < kDown) { pa *= kUp; ea -= 400; }
        if (fabs(pb) < kDown) { pb *= kUp; eb -= 400; }
    }
    ra.p0 = 0.0; ra.p1 = pa; ra.e = ea;
    rb.p0 = 0.0; rb.p1 = pb; rb.e = eb;
    // (UB) the order-(m+1) stream: sectoral seed L_{m+1,m+1} one factor on from L_mm
    LegendreStream qa = ra, qb = rb;
    double inv_q_prev = 0.0;
    if constexpr (UB) {
        const double f = sqrt((2.0 * m + 3.0) / (2.0 * m + 2.0));
        qa.p1 = pa * f * sa;
        qb.p1 = pb * f * sb;
        if (fabs(qa.p1) < kDown) { qa.p1 *= kUp; qa.e -= 400; }
        if (fabs(qb.p1) < kDown) { qb.p1 *= kUp; qb.e -= 400; }
    }

    double Kaa[3] = {0, 0, 0}, Kbb[3] = {0, 0, 0}, Kba[4] = {0, 0, 0, 0};
    // M >= 3: full blocks (only the upper triangles of J(a,a), J(b,b) are accumulated)
    double KaaG[M * M] = {}, KbbG[M * M] = {}, KbaG[M * M] = {};
    const double dm = (double)m;
    double inv_a_prev = 0.0;   // 1 / a_{l-1,m}
    for (int l = m; l <= g.ell_max; ++l) {
        const double dl = (double)l;
        double c_der;          // sqrt((2l+1)(l^2-m^2)/(2l-1)) = (2l+1)/a_lm
        if (l == m) {
            c_der = 0.0;
        } else if (l == m + 1) {
            const double a1 = sqrt(2.0 * dm + 3.0);
            ra.p0 = ra.p1; ra.p1 = a1 * ra.z * ra.p0;
            rb.p0 = rb.p1; rb.p1 = a1 * rb.z * rb.p0;
            inv_a_prev = 1.0 / a1;
            c_der = a1;
        } else {
            const double q = (4.0 * dl * dl - 1.0) / ((dl - dm) * (dl + dm));
            const double al = sqrt(q);
            double t = al * (ra.z * ra.p1 - inv_a_prev * ra.p0);
            ra.p0 = ra.p1; ra.p1 = t;
            t = al * (rb.z * rb.p1 - inv_a_prev * rb.p0);
            rb.p0 = rb.p1; rb.p1 = t;
            inv_a_prev = 1.0 / al;
            c_der = (2.0 * dl + 1.0) * inv_a_prev;
        }
        if (ra.e < 0 && fabs(ra.p1) > kUp) { ra.p0 *= kDown; ra.p1 *= kDown; ra.e += 400; }
        if (rb.e < 0 && fabs(rb.p1) > kUp) { rb.p0 *= kDown; rb.p1 *= kDown; rb.e += 400; }
        const double cl = C[l];
        const double va = ra.value(), vb = rb.value();
        if constexpr (M == 1) {
            Kaa[0] = fma(cl * va, va, Kaa[0]);
            Kbb[0] = fma(cl * vb, vb, Kbb[0]);
            Kba[0] = fma(cl * vb, va, Kba[0]);
        } else if constexpr (M >= 3) {
            // value and z-derivatives up to M-1: the first as for M = 2, the higher ones
            // from the associated Legendre equation,
            //   (1 - z^2) L2 = 2 z L1 - c L0,
            //   (1 - z^2) L3 = 4 z L2 + 2 L1 - c L1 + 2 m^2 z / (1 - z^2)^2 L0,
            // c = l(l+1) - m^2 / (1 - z^2), Lk = d^k L_lm / dz^k
            double Fa[M], Fb[M];
            Fa[0] = va;
            Fb[0] = vb;
            Fa[1] = ldexp((c_der * ra.p0 - dl * ra.z * ra.p1) * ra.inv_s2, ra.e);
            Fb[1] = ldexp((c_der * rb.p0 - dl * rb.z * rb.p1) * rb.inv_s2, rb.e);
            const double ll = dl * (dl + 1.0), mm = dm * dm;
            const double ca = ll - mm * ra.inv_s2, cb = ll - mm * rb.inv_s2;
            Fa[2] = (2.0 * ra.z * Fa[1] - ca * Fa[0]) * ra.inv_s2;
            Fb[2] = (2.0 * rb.z * Fb[1] - cb * Fb[0]) * rb.inv_s2;
            if constexpr (M >= 4) {
                Fa[3] = (4.0 * ra.z * Fa[2] + 2.0 * Fa[1] - ca * Fa[1] + 2.0 * mm * ra.z * ra.inv_s2 * ra.inv_s2 * Fa[0]) *
                        ra.inv_s2;
                Fb[3] = (4.0 * rb.z * Fb[2] + 2.0 * Fb[1] - cb * Fb[1] + 2.0 * mm * rb.z * rb.inv_s2 * rb.inv_s2 * Fb[0]) *
                        rb.inv_s2;
            }
#pragma unroll
            for (int p = 0; p < M; ++p) {
                const double cfa = cl * Fa[p], cfb = cl * Fb[p];
#pragma unroll
                for (int q = p; q < M; ++q) {
                    KaaG[p * M + q] = fma(cfa, Fa[q], KaaG[p * M + q]);
                    KbbG[p * M + q] = fma(cfb, Fb[q], KbbG[p * M + q]);
                }
#pragma unroll
                for (int q = 0; q < M; ++q) KbaG[p * M + q] = fma(cfb, Fa[q], KbaG[p * M + q]);
            }
        } else {
            double da, db;
            if constexpr (UB) {
                // L_{l,m+1} for l >= m+1 by the same recurrence in order m+1; U_m L_lm from it
                const double dm1 = dm + 1.0;
                da = db = 0.0;
                if (l == m + 2) {
                    const double a1 = sqrt(2.0 * dm1 + 3.0);
                    qa.p0 = qa.p1; qa.p1 = a1 * qa.z * qa.p0;
                    qb.p0 = qb.p1; qb.p1 = a1 * qb.z * qb.p0;
                    inv_q_prev = 1.0 / a1;
                } else if (l > m + 2) {
                    const double q = (4.0 * dl * dl - 1.0) / ((dl - dm1) * (dl + dm1));
                    const double al = sqrt(q);
                    double t = al * (qa.z * qa.p1 - inv_q_prev * qa.p0);
                    qa.p0 = qa.p1; qa.p1 = t;
                    t = al * (qb.z * qb.p1 - inv_q_prev * qb.p0);
                    qb.p0 = qb.p1; qb.p1 = t;
                    inv_q_prev = 1.0 / al;
                }
                if (qa.e < 0 && fabs(qa.p1) > kUp) { qa.p0 *= kDown; qa.p1 *= kDown; qa.e += 400; }
                if (qb.e < 0 && fabs(qb.p1) > kUp) { qb.p0 *= kDown; qb.p1 *= kDown; qb.e += 400; }
                if (l > m) {
                    const double f = -sqrt((dl + dm + 1.0) * (dl - dm));
                    da = f * qa.value();
                    db = f * qb.value();
                }
            } else {
                // (1 - z^2) dL_l/dz = -l z L_l + c_der L_{l-1}
                da = ldexp((c_der * ra.p0 - dl * ra.z * ra.p1) * ra.inv_s2, ra.e);
                db = ldexp((c_der * rb.p0 - dl * rb.z * rb.p1) * rb.inv_s2, rb.e);
            }
            const double cva = cl * va, cda = cl * da, cvb = cl * vb, cdb = cl * db;
            Kaa[0] = fma(cva, va, Kaa[0]);
            Kaa[1] = fma(cva, da, Kaa[1]);
            Kaa[2] = fma(cda, da, Kaa[2]);
            Kbb[0] = fma(cvb, vb, Kbb[0]);
            Kbb[1] = fma(cvb, db, Kbb[1]);
            Kbb[2] = fma(cdb, db, Kbb[2]);
            Kba[0] = fma(cvb, va, Kba[0]);
            Kba[1] = fma(cvb, da, Kba[1]);
            Kba[2] = fma(cdb, va, Kba[2]);
            Kba[3] = fma(cdb, da, Kba[3]);
        }
    }

    const size_t base = ((size_t)j * g.m_rows + m) * factor_stride(M);
    if constexpr (M >= 3) {
#pragma unroll
        for (int p = 0; p < M; ++p)
#pragma unroll
            for (int q = 0; q < p; ++q) {
                KaaG[p * M + q] = KaaG[q * M + p];
                KbbG[p * M + q] = KbbG[q * M + p];
            }
        double A[M * M] = {}, B[M * M];
        if (j == 0) start_gen<M>(KaaG, B);
        else factors_gen<M>(KaaG, KbbG, KbaG, A, B);
        if (mirror) {
#pragma unroll
            for (int i = 0; i < M * M; ++i)
                if (((i / M) + (i % M)) & 1) { A[i] = -A[i]; B[i] = -B[i]; }
        }
        constexpr int E = factor_stride(M);
        double v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = 0.0;
#pragma unroll
        for (int i = 0; i < M * M; ++i) v[i] = A[i];
#pragma unroll
        for (int p = 0; p < M; ++p)
#pragma unroll
            for (int q = 0; q <= p; ++q) v[b_index<M>(p, q)] = B[p * M + q];
#pragma unroll
        for (int i = 0; i < E; ++i) f64[base + i] = v[i];
        if (f32) {
#pragma unroll
            for (int i = 0; i < E; ++i) f32[base + i] = (float)v[i];
        }
    } else if constexpr (M == 1) {
        double A, B;
        if (j == 0) { A = 0.0; B = start_m1(Kaa[0]); }
        else factors_m1(Kaa[0], Kbb[0], Kba[0], A, B);
        f64[base] = A;
        f64[base + 1] = B;
        if (f32) { f32[base] = (float)A; f32[base + 1] = (float)B; }
    } else {
        double A[4] = {0, 0, 0, 0}, B[3];
        if (j == 0) start_m2(Kaa, B);
        else factors_m2(Kaa, Kbb, Kba, A, B);
        if (mirror) {   // D A D, D B D: the off-diagonal entries change sign
            A[1] = -A[1];
            A[2] = -A[2];
            B[1] = -B[1];
        }
        const double v[8] = {A[0], A[1], A[2], A[3], B[0], B[1], B[2], 0.0};
#pragma unroll
        for (int i = 0; i < 8; ++i) f64[base + i] = v[i];
        if (f32) {
#pragma unroll
            for (int i = 0; i < 8; ++i) f32[base + i] = (float)v[i];
        }
    }
}

// Block transitions for the affine scan across rings: for fine block b of the main-walk
// sets [J_b, J_{b+1}), J_b = j0 + floor(walk b / blocks), the product
// Phi_b = A_{J_{b+1}-1} ... A_{J_b} of the step matrices of eq. (state_space), i.e. the map
// the block applies to its start state when its noise is zero.  One thread per (m, b).
template <int M>
__global__ __launch_bounds__(64) void phi_kernel(Geometry g, const double* __restrict__ f64, int blocks,
                                                 double* __restrict__ phi64, float* __restrict__ phi32)
{
    const int m = blockIdx.x * 64 + threadIdx.x;
    const int b = blockIdx.y;
    if (m > g.m_top) return;
    const int j0 = g.even ? 2 : 1;
    const long walk = g.n_sets - j0;
    const int jb = j0 + (int)(walk * b / blocks), je = j0 + (int)(walk * (b + 1) / blocks);
    constexpr int E = factor_stride(M);
    double p[M * M];
#pragma unroll
    for (int i = 0; i < M * M; ++i) p[i] = (i % (M + 1) == 0) ? 1.0 : 0.0;
    for (int j = jb; j < je; ++j) {
        const double* r = f64 + ((size_t)j * g.m_rows + m) * E;
        if constexpr (M == 1) {
            p[0] = r[0] * p[0];
        } else if constexpr (M == 2) {
            const double q00 = r[0] * p[0] + r[1] * p[2], q01 = r[0] * p[1] + r[1] * p[3];
            const double q10 = r[2] * p[0] + r[3] * p[2], q11 = r[2] * p[1] + r[3] * p[3];
            p[0] = q00; p[1] = q01; p[2] = q10; p[3] = q11;
        } else {
            // A row-major in the record's first M*M values
            double q[M * M];
#pragma unroll
            for (int a = 0; a < M; ++a)
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    double acc = 0.0;
#pragma unroll
                    for (int k = 0; k < M; ++k) acc += r[a * M + k] * p[k * M + c];
                    q[a * M + c] = acc;
                }
#pragma unroll
            for (int i = 0; i < M * M; ++i) p[i] = q[i];
        }
    }
    const size_t o = ((size_t)b * g.m_rows + m) * (M * M);
#pragma unroll
    for (int i = 0; i < M * M; ++i) {
        phi64[o + i] = p[i];
        if (phi32) phi32[o + i] = (float)p[i];
    }
}

// ---------------------------------------------------------------- Sec. 3, order 1
// Cross covariances without a band limit from the Green's function of the mode's
// operator: C_l = 1/(kappa + l(l+1)) for every l, kappa = -lambda(lambda+1), and
// eq. (Jmatrix_efficient) with P^m_lambda of eq. (Legendre_hypergeometric) gives, for
// z1 <= z2,
//   J^m(z1, z2) = R_m w^m H_m(-z1) H_m(z2) / (4 |sin pi lambda|),
//   R_m = prod_{k<=m} (k^2 - k + kappa) / k^2   (the Pochhammer products over m!^2),
//   w^2 = (1 + z1)(1 - z2) / ((1 - z1)(1 + z2)),
//   H_m(x) = 2F1(-lambda, lambda+1; 1+m; (1-x)/2),
// using Gamma(1+lambda-m) Gamma(-lambda-m) = pi / (|sin pi lambda| R_m m!^2).  H_m has a
// series of positive terms, term ratio (n^2 + n + kappa) / ((n+1)(n+1+m)) t.  It is
// summed directly for x >= 0 (t <= 1/2) and, for x < 0, H_0 and H_1 come from the
// series or, close to x = -1, from the logarithmic continuation of 2F1 about t = 1
// (c - a - b = 0 and 1; Abramowitz & Stegun 15.3.11), and H_m from the three-term
// recurrence in the order of the Ferrers functions rewritten for H_m,
//   H_{m+2} = (m+1)(m+2) / q_{m+1} * (1+x)/(1-x) * (H_m - 2x/(1+x) H_{m+1}),
// whose two terms are positive for x < 0.  The values of H per ring are tabulated by
// two kernels (one thread per (ring, m) for the series side, one per ring for the
// recurrence side), and the factor kernel reads the table.
struct GreenConst {
    double kappa;
    double inv4s;        // 1 / (4 |sin pi lambda|)
    double g;            // |sin pi lambda| / pi = 1 / (Gamma(-lambda) Gamma(lambda+1))
    double lam_re, tau;  // lambda = lam_re + i tau (tau = 0: real lambda)
};

// (z, sin theta) of ring i: explicit grid or ring centres (as the Legendre-sum setup)
__device__ inline void green_ring(const Geometry& g, const double* __restrict__ zgrid, int i, double& z,
                                  double& sn)
{
    if (zgrid) {
        z = zgrid[i];
        sn = sqrt((1.0 - z) * (1.0 + z));
    } else {
        sincospi((double)(g.n_theta - 2 * i - 1) / (2.0 * g.n_theta), &z, &sn);
    }
}

__device__ double green_series(int m, double kappa, double t)
{
    double acc = 1.0, term = 1.0;
    for (int n = 0; n < 1000000; ++n) {
        const double dn = (double)n;
        const double r = (dn * dn + dn + kappa) / ((dn + 1.0) * (dn + 1.0 + (double)m)) * t;
        term *= r;
        acc += term;
        if (r < 1.0 && term < 1e-18 * acc) break;
    }
    return acc;
}

// Re of the digamma at p + i q (p > 0): shifted up to p >= 20, then the asymptotic series
// log w - 1/(2w) - 1/(12 w^2) + 1/(120 w^4) - 1/(252 w^6) + 1/(240 w^8) - 1/(132 w^10).
__device__ double re_digamma(double p, double q)
{
    double shift = 0.0;
    while (p < 20.0) {
        shift += p / (p * p + q * q);   // Re 1/(p + i q)
        p += 1.0;
    }
    const double r2 = p * p + q * q;
    // powers of 1/w = (p - i q)/r2, real parts only where needed
    const double wr = p / r2, wi = -q / r2;          // 1/w
    const double w2r = wr * wr - wi * wi, w2i = 2.0 * wr * wi;
    const double w4r = w2r * w2r - w2i * w2i, w4i = 2.0 * w2r * w2i;
    const double w6r = w4r * w2r - w4i * w2i, w6i = w4r * w2i + w4i * w2r;
    const double w8r = w4r * w4r - w4i * w4i, w8i = 2.0 * w4r * w4i;
    const double w10r = w8r * w2r - w8i * w2i;
    (void)w6i;
    const double logw = 0.5 * log(r2);
    return logw - 0.5 * wr - w2r / 12.0 + w4r / 120.0 - w6r / 252.0 + w8r / 240.0 - w10r / 132.0 - shift;
}

// psi(a + k) + psi(b + k), a = -lambda, b = lambda + 1
__device__ inline double psi_sum(const GreenConst& c, double k)
{
    if (c.tau != 0.0) return 2.0 * re_digamma(0.5 + k, c.tau);
    return re_digamma(-c.lam_re + k, 0.0) + re_digamma(c.lam_re + 1.0 + k, 0.0);
}

// H_0 and H_1 at t = 1 - u from the continuation about t = 1:
//   H_0 = -g sum_k c_k u^k [log u - 2 psi(k+1) + psi(a+k) + psi(b+k)],
//   H_1 = g/kappa + g u sum_k d_k u^k [log u - psi(k+1) - psi(k+2) + psi(a+k+1) + psi(b+k+1)],
// c_k = (a)_k (b)_k / k!^2, d_k = (a+1)_k (b+1)_k / (k! (k+1)!).
__device__ void green_h01_far(const GreenConst& c, double u, double& h0, double& h1)
{
    const double lu = log(u);
    double ck = 1.0, dk = 1.0, uk = 1.0, s0 = 0.0, s1 = 0.0;
    double psi1 = -0.57721566490153286061;    // psi(1)
    for (int k = 0; k < 100000; ++k) {
        const double dkk = (double)k;
        const double psi2 = psi1 + 1.0 / (dkk + 1.0);
        const double e0 = ck * uk * (lu - 2.0 * psi1 + psi_sum(c, dkk));
        const double e1 = dk * uk * (lu - psi1 - psi2 + psi_sum(c, dkk + 1.0));
        s0 += e0;
        s1 += e1;
        const double rc = (dkk * dkk + dkk + c.kappa) / ((dkk + 1.0) * (dkk + 1.0));
        ck *= rc;
        dk *= ((dkk + 1.0) * (dkk + 2.0) + c.kappa) / ((dkk + 1.0) * (dkk + 2.0));
        uk *= u;
        psi1 = psi2;
        if (k > 4 && rc * u < 0.9 && fabs(e0) < 1e-18 * fabs(s0) && fabs(e1) < 1e-18 * fabs(s1)) break;
    }
    h0 = -c.g * s0;
    h1 = c.g / c.kappa + c.g * u * s1;
}

// Series side of the table: thread (ring i, mode m) fills H_m(+-z_i) for the sign that
// makes the argument non-negative (both at z_i = 0).
// Tables hold H_m for m = 0..m_hi (m_top at order 1, m_top + 1 at order 2), `w` values per ring.
__global__ __launch_bounds__(64) void green_series_kernel(Geometry g, const double* __restrict__ zgrid, GreenConst c,
                                                          int m_hi, int w, double* __restrict__ hp,
                                                          double* __restrict__ hn)
{
    const int m = blockIdx.x * 64 + threadIdx.x;
    const int i = blockIdx.y;
    if (m > m_hi) return;
    double z, sn;
    green_ring(g, zgrid, i, z, sn);
    const size_t o = (size_t)i * w + m;
    // t = (1 - x)/2 with 1 - x = sin^2 / (1 + x) for x >= 0
    if (z >= 0.0) hp[o] = green_series(m, c.kappa, sn * sn / (2.0 * (1.0 + z)));
    if (z <= 0.0) hn[o] = green_series(m, c.kappa, sn * sn / (2.0 * (1.0 - z)));
}

// Recurrence side: one thread per ring fills H_m(x) for x = -|z_i| < 0, m = 0..m_hi.
__global__ __launch_bounds__(64) void green_recur_kernel(Geometry g, const double* __restrict__ zgrid, GreenConst c,
                                                         int m_hi, int w, double* __restrict__ hp,
                                                         double* __restrict__ hn)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= g.n_theta) return;
    double z, sn;
    green_ring(g, zgrid, i, z, sn);
    if (z == 0.0) return;
    const double x = -fabs(z);
    double* __restrict__ h = (z > 0.0 ? hn : hp) + (size_t)i * w;
    const double u = sn * sn / (2.0 * (1.0 - x));       // (1 + x)/2
    double h0, h1;
    if (u * (c.kappa + 1.0) <= 0.5) {
        green_h01_far(c, u, h0, h1);
    } else {
        h0 = green_series(0, c.kappa, 1.0 - u);
        h1 = green_series(1, c.kappa, 1.0 - u);
    }
    h[0] = h0;
    if (m_hi >= 1) h[1] = h1;
    const double opx = 2.0 * u, omx = 1.0 - x;
    const double ratio = opx / omx, cross = -2.0 * x / opx;
    for (int k = 0; k + 2 <= m_hi; ++k) {
        const double dk = (double)k;
        const double q = (dk + 1.0) * (dk + 2.0) + c.kappa;
        const double h2 = (dk + 1.0) * (dk + 2.0) / q * ratio * fma(cross, h1, h0);
        h[k + 2] = h2;
        h0 = h1;
        h1 = h2;
    }
}

// log(1 + z) and log(1 - z), each through sin^2 theta where that side is the small one
__device__ inline void green_logs(double z, double sn, double& lp, double& lm)
{
    if (z >= 0.0) {
        lp = log1p(z);
        lm = log(sn * sn / (1.0 + z));
    } else {
        lp = log(sn * sn / (1.0 - z));
        lm = log1p(-z);
    }
}

// J^m between rings x (lower value) and y, from the tables
__device__ inline double green_j(const GreenConst& c, double rm, int m, double zx, double sx, double zy, double sy,
                                 double hx_neg, double hy_pos)
{
    double wm = 1.0;
    if (zx != zy && m > 0) {
        double lpx, lmx, lpy, lmy;
        green_logs(zx, sx, lpx, lmx);
        green_logs(zy, sy, lpy, lmy);
        wm = exp(0.5 * (double)m * ((lpx - lmx) + (lmy - lpy)));
    }
    return rm * wm * hx_neg * hy_pos * c.inv4s;
}

GreenConst green_const(double kappa)
{
    GreenConst c;
    c.kappa = kappa;
    double abs_sin;
    if (kappa > 0.25) {
        c.lam_re = -0.5;
        c.tau = sqrt(kappa - 0.25);
        abs_sin = cosh(M_PI * c.tau);
    } else {
        c.lam_re = (-1.0 + sqrt(1.0 - 4.0 * kappa)) / 2.0;
        c.tau = 0.0;
        abs_sin = -sin(M_PI * c.lam_re);
    }
    c.inv4s = 1.0 / (4.0 * abs_sin);
    c.g = abs_sin / M_PI;
    return c;
}

// One thread per (set j, mode m), sets as in factor_kernel (south: the southern walk's own
// steps, stored mirrored; at order 1 the mirror leaves the record unchanged).
__global__ __launch_bounds__(64) void green_factor_kernel(Geometry g, const double* __restrict__ zgrid, GreenConst c,
                                                          int south, int w, const double* __restrict__ hp,
                                                          const double* __restrict__ hn, double* __restrict__ f64,
                                                          float* __restrict__ f32)
{
    const int j = blockIdx.x * 64 + threadIdx.x;
    const int m = blockIdx.y;
    if (j >= g.n_sets) return;
    int a, b;
    if (south && j >= (g.even ? 2 : 1)) {
        a = g.s + j - 1; b = g.s + j;
    } else if (j == 0) {
        a = b = g.s;
    } else if (g.even) {
        if (j == 1) { a = g.s; b = g.s + 1; }
        else { a = g.s - j + 2; b = g.s - j + 1; }
    } else {
        a = g.s - j + 1; b = g.s - j;
    }
    double rm = 1.0;
    for (int k = 1; k <= m; ++k) {
        const double dk = (double)k;
        rm *= (dk * dk - dk + c.kappa) / (dk * dk);
    }
    double za, sa, zb, sb;
    green_ring(g, zgrid, a, za, sa);
    green_ring(g, zgrid, b, zb, sb);
    const size_t oa = (size_t)a * w + m, ob = (size_t)b * w + m;
    const double kaa = green_j(c, rm, m, za, sa, za, sa, hn[oa], hp[oa]);
    const size_t base = ((size_t)j * g.m_rows + m) * factor_stride(1);
    double A, B;
    if (j == 0) {
        A = 0.0;
        B = start_m1(kaa);
    } else {
        const double kbb = green_j(c, rm, m, zb, sb, zb, sb, hn[ob], hp[ob]);
        const double kba = za <= zb ? green_j(c, rm, m, za, sa, zb, sb, hn[oa], hp[ob])
                                    : green_j(c, rm, m, zb, sb, za, sa, hn[ob], hp[oa]);
        factors_m1(kaa, kbb, kba, A, B);
    }
    f64[base] = A;
    f64[base + 1] = B;
    if (f32) { f32[base] = (float)A; f32[base + 1] = (float)B; }
}

// Order 2 (two distinct kappa, the basis (g, U g) of Sec. 3): with the partial fractions
// C_l = b_0/(l(l+1) + kappa_0) + b_1/(l(l+1) + kappa_1), b_0 = 1/(kappa_1 - kappa_0) = -b_1
// (eq. (C_ell_efficient)), eq. (Jmatrix_efficient) takes P^{m+p}(-z1) P^{m+q}(z2) for
// p, q < 2 (z1 <= z2), and P^{m+1} / P^m adds the factor a (1 -+ z)/(1 +- z) ^(1/2) with
// a = (m^2 + m + kappa)/(m + 1):
//   J_pq = sum_i b_i R^i_m w^m / (4 |sin pi lambda_i|) (-1)^p (a_i r1)^p H^i_{m+p}(-z1)
//          (a_i r2)^q H^i_{m+q}(z2),  r1 = sqrt((1+z1)/(1-z1)), r2 = sqrt((1-z2)/(1+z2)).
// hn1[i][k] = H^i_{m+k}(-z1), hp2[i][k] = H^i_{m+k}(z2); J[p*2 + q].
__device__ void green2_pair(const GreenConst* c, const double* rm, int m, double z1, double s1, double z2, double s2,
                            const double (&hn1)[2][2], const double (&hp2)[2][2], double (&J)[4])
{
    double wm = 1.0, lp1, lm1, lp2, lm2;
    green_logs(z1, s1, lp1, lm1);
    green_logs(z2, s2, lp2, lm2);
    if (z1 != z2 && m > 0) wm = exp(0.5 * (double)m * ((lp1 - lm1) + (lm2 - lp2)));
    const double r1 = exp(0.5 * (lp1 - lm1)), r2 = exp(0.5 * (lm2 - lp2));
    const double b0 = 1.0 / (c[1].kappa - c[0].kappa);
#pragma unroll
    for (int k = 0; k < 4; ++k) J[k] = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double sc = (i == 0 ? b0 : -b0) * rm[i] * wm * c[i].inv4s;
        const double a = ((double)m * m + m + c[i].kappa) / (m + 1.0);
        const double u0 = hn1[i][0], u1 = -a * r1 * hn1[i][1];
        const double v0 = hp2[i][0], v1 = a * r2 * hp2[i][1];
        J[0] = fma(sc * u0, v0, J[0]);
        J[1] = fma(sc * u0, v1, J[1]);
        J[2] = fma(sc * u1, v0, J[2]);
        J[3] = fma(sc * u1, v1, J[3]);
    }
}

// One thread per (set j, mode m) at order 2, sets and mirror as in factor_kernel.
__global__ __launch_bounds__(64) void green2_factor_kernel(Geometry g, const double* __restrict__ zgrid, GreenConst c0,
                                                           GreenConst c1, int south, int w,
                                                           const double* __restrict__ hp,
                                                           const double* __restrict__ hn, double* __restrict__ f64,
                                                           float* __restrict__ f32)
{
    const int j = blockIdx.x * 64 + threadIdx.x;
    const int m = blockIdx.y;
    if (j >= g.n_sets) return;
    const bool mirror = south && j >= (g.even ? 2 : 1);
    int a, b;
    if (mirror) {
        a = g.s + j - 1; b = g.s + j;
    } else if (j == 0) {
        a = b = g.s;
    } else if (g.even) {
        if (j == 1) { a = g.s; b = g.s + 1; }
        else { a = g.s - j + 2; b = g.s - j + 1; }
    } else {
        a = g.s - j + 1; b = g.s - j;
    }
    const GreenConst c[2] = {c0, c1};
    double rm[2] = {1.0, 1.0};
    for (int k = 1; k <= m; ++k) {
        const double dk = (double)k;
        rm[0] *= (dk * dk - dk + c0.kappa) / (dk * dk);
        rm[1] *= (dk * dk - dk + c1.kappa) / (dk * dk);
    }
    double za, sa, zb, sb;
    green_ring(g, zgrid, a, za, sa);
    green_ring(g, zgrid, b, zb, sb);
    // table i (kappa_i) starts at i * n_theta * w
    const size_t tstride = (size_t)g.n_theta * w;
    double hna[2][2], hpa[2][2], hnb[2][2], hpb[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            hna[i][k] = hn[i * tstride + (size_t)a * w + m + k];
            hpa[i][k] = hp[i * tstride + (size_t)a * w + m + k];
            hnb[i][k] = hn[i * tstride + (size_t)b * w + m + k];
            hpb[i][k] = hp[i * tstride + (size_t)b * w + m + k];
        }
    double Ja[4], Jb[4], Jx[4];
    green2_pair(c, rm, m, za, sa, za, sa, hna, hpa, Ja);
    const double kaa[3] = {Ja[0], 0.5 * (Ja[1] + Ja[2]), Ja[3]};
    double A[4] = {0, 0, 0, 0}, B[3];
    if (j == 0) {
        start_m2(kaa, B);
    } else {
        green2_pair(c, rm, m, zb, sb, zb, sb, hnb, hpb, Jb);
        const double kbb[3] = {Jb[0], 0.5 * (Jb[1] + Jb[2]), Jb[3]};
        double kba[4];
        if (zb <= za) {                       // J(z_b, z_a) directly: E[x_b,p x_a,q]
            green2_pair(c, rm, m, zb, sb, za, sa, hnb, hpa, Jx);
            kba[0] = Jx[0]; kba[1] = Jx[1]; kba[2] = Jx[2]; kba[3] = Jx[3];
        } else {                              // J(z_a, z_b) transposed
            green2_pair(c, rm, m, za, sa, zb, sb, hna, hpb, Jx);
            kba[0] = Jx[0]; kba[1] = Jx[2]; kba[2] = Jx[1]; kba[3] = Jx[3];
        }
        factors_m2(kaa, kbb, kba, A, B);
    }
    if (mirror) {   // D A D, D B D: the off-diagonal entries change sign
        A[1] = -A[1];
        A[2] = -A[2];
        B[1] = -B[1];
    }
    const size_t base = ((size_t)j * g.m_rows + m) * factor_stride(2);
    const double v[8] = {A[0], A[1], A[2], A[3], B[0], B[1], B[2], 0.0};
#pragma unroll
    for (int i = 0; i < 8; ++i) f64[base + i] = v[i];
    if (f32) {
#pragma unroll
        for (int i = 0; i < 8; ++i) f32[base + i] = (float)v[i];
    }
}

// ---- Sec. 3 for a complex-conjugate pair kappa = alpha +- i beta (order 2, basis (g, U g)) ----
// The order-1 formulas hold with complex arithmetic: lambda = -1/2 + sqrt(1/4 - kappa),
// G_m by its series (x >= 0) or by the continuation about t = 1 and the m-recurrence (x < 0),
// J^m_kappa = (Pi_m / m!^2) w^m G_m(-z1) G_m(z2) / (-4 sin pi lambda).  The kappa_2 term of the
// partial fractions is the complex conjugate of the kappa_1 term, b_1 = i / (2 beta), so
// J_pq = 2 Re[b_1 (...)_1]: only kappa_1's tables are built.
struct Zd {
    double re, im;
};
__device__ __host__ inline Zd zadd(Zd a, Zd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __host__ inline Zd zsub(Zd a, Zd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __host__ inline Zd zmul(Zd a, Zd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __host__ inline Zd zscale(Zd a, double s) { return {a.re * s, a.im * s}; }
__device__ __host__ inline Zd zdiv(Zd a, Zd b)
{
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __host__ inline double zabs(Zd a) { return hypot(a.re, a.im); }

struct GreenConstC {
    Zd kappa;
    Zd lam;      // -1/2 + sqrt(1/4 - kappa)
    Zd g;        // -sin(pi lambda) / pi = 1 / (Gamma(-lambda) Gamma(lambda + 1))
    Zd sc;       // 1 / (-4 sin pi lambda)
    double beta;
};

GreenConstC greenc_const(double alpha, double beta)
{
    GreenConstC c;
    c.kappa = {alpha, beta};
    // principal square root of 1/4 - kappa
    const double xr = 0.25 - alpha, xi = -beta;
    const double r = hypot(xr, xi);
    double sr = sqrt(0.5 * (r + xr)), si = sqrt(0.5 * (r - xr));
    if (xi < 0.0) si = -si;
    c.lam = {-0.5 + sr, si};
    // sin(pi (a + i b)) = sin(pi a) cosh(pi b) + i cos(pi a) sinh(pi b)
    const Zd sn = {sin(M_PI * c.lam.re) * cosh(M_PI * c.lam.im), cos(M_PI * c.lam.re) * sinh(M_PI * c.lam.im)};
    c.g = zscale(sn, -1.0 / M_PI);
    c.sc = zdiv({1.0, 0.0}, zscale(sn, -4.0));
    c.beta = beta;
    return c;
}

__device__ Zd greenc_series(int m, Zd kappa, double t)
{
    Zd acc = {1.0, 0.0}, term = {1.0, 0.0};
    for (int n = 0; n < 1000000; ++n) {
        const double dn = (double)n;
        const double den = t / ((dn + 1.0) * (dn + 1.0 + (double)m));
        const Zd r = {(dn * dn + dn + kappa.re) * den, kappa.im * den};
        term = zmul(term, r);
        acc = zadd(acc, term);
        if (zabs(r) < 1.0 && zabs(term) < 1e-18 * zabs(acc)) break;
    }
    return acc;
}

// digamma at z (not a pole): shifted up to Re z >= 20 by psi(z) = psi(z + 1) - 1/z, then the
// asymptotic series log z - 1/(2z) - 1/(12 z^2) + 1/(120 z^4) - 1/(252 z^6) + 1/(240 z^8) - 1/(132 z^10)
__device__ Zd zdigamma(Zd z)
{
    Zd shift = {0.0, 0.0};
    while (z.re < 20.0) {
        shift = zadd(shift, zdiv({1.0, 0.0}, z));
        z.re += 1.0;
    }
    const Zd w = zdiv({1.0, 0.0}, z);
    const Zd w2 = zmul(w, w), w4 = zmul(w2, w2), w6 = zmul(w4, w2), w8 = zmul(w4, w4), w10 = zmul(w8, w2);
    Zd v = {log(zabs(z)), atan2(z.im, z.re)};
    v = zsub(v, zscale(w, 0.5));
    v = zsub(v, zscale(w2, 1.0 / 12.0));
    v = zadd(v, zscale(w4, 1.0 / 120.0));
    v = zsub(v, zscale(w6, 1.0 / 252.0));
    v = zadd(v, zscale(w8, 1.0 / 240.0));
    v = zsub(v, zscale(w10, 1.0 / 132.0));
    return zsub(v, shift);
}

// H_0 and H_1 at t = 1 - u from the continuation about t = 1 (as green_h01_far, complex)
__device__ void greenc_h01_far(const GreenConstC& c, double u, Zd& h0, Zd& h1)
{
    const double lu = log(u);
    const Zd mlam = {-c.lam.re, -c.lam.im}, lam1 = {c.lam.re + 1.0, c.lam.im};
    Zd ck = {1.0, 0.0}, dk = {1.0, 0.0}, s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
    double uk = 1.0, psi1 = -0.57721566490153286061;    // psi(1)
    for (int k = 0; k < 100000; ++k) {
        const double dkk = (double)k;
        const double psi2 = psi1 + 1.0 / (dkk + 1.0);
        const Zd pp0 = zadd(zdigamma({mlam.re + dkk, mlam.im}), zdigamma({lam1.re + dkk, lam1.im}));
        const Zd pp1 = zadd(zdigamma({mlam.re + dkk + 1.0, mlam.im}), zdigamma({lam1.re + dkk + 1.0, lam1.im}));
        const Zd e0 = zscale(zmul(ck, {lu - 2.0 * psi1 + pp0.re, pp0.im}), uk);
        const Zd e1 = zscale(zmul(dk, {lu - psi1 - psi2 + pp1.re, pp1.im}), uk);
        s0 = zadd(s0, e0);
        s1 = zadd(s1, e1);
        const Zd rc = zscale({dkk * dkk + dkk + c.kappa.re, c.kappa.im}, 1.0 / ((dkk + 1.0) * (dkk + 1.0)));
        ck = zmul(ck, rc);
        dk = zmul(dk, zscale({(dkk + 1.0) * (dkk + 2.0) + c.kappa.re, c.kappa.im}, 1.0 / ((dkk + 1.0) * (dkk + 2.0))));
        uk *= u;
        psi1 = psi2;
        if (k > 4 && zabs(rc) * u < 0.9 && zabs(e0) < 1e-18 * zabs(s0) && zabs(e1) < 1e-18 * zabs(s1)) break;
    }
    h0 = zscale(zmul(c.g, s0), -1.0);
    h1 = zadd(zdiv(c.g, c.kappa), zscale(zmul(c.g, s1), u));
}

// The tables of kappa_1, complex values interleaved (re, im): as green_series_kernel and
// green_recur_kernel.
__global__ __launch_bounds__(64) void greenc_series_kernel(Geometry g, const double* __restrict__ zgrid, GreenConstC c,
                                                           int m_hi, int w, double* __restrict__ hp,
                                                           double* __restrict__ hn)
{
    const int m = blockIdx.x * 64 + threadIdx.x;
    const int i = blockIdx.y;
    if (m > m_hi) return;
    double z, sn;
    green_ring(g, zgrid, i, z, sn);
    const size_t o = 2 * ((size_t)i * w + m);
    if (z >= 0.0) {
        const Zd v = greenc_series(m, c.kappa, sn * sn / (2.0 * (1.0 + z)));
        hp[o] = v.re;
        hp[o + 1] = v.im;
    }
    if (z <= 0.0) {
        const Zd v = greenc_series(m, c.kappa, sn * sn / (2.0 * (1.0 - z)));
        hn[o] = v.re;
        hn[o + 1] = v.im;
    }
}

__global__ __launch_bounds__(64) void greenc_recur_kernel(Geometry g, const double* __restrict__ zgrid, GreenConstC c,
                                                          int m_hi, int w, double* __restrict__ hp,
                                                          double* __restrict__ hn)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= g.n_theta) return;
    double z, sn;
    green_ring(g, zgrid, i, z, sn);
    if (z == 0.0) return;
    const double x = -fabs(z);
    double* __restrict__ h = (z > 0.0 ? hn : hp) + 2 * (size_t)i * w;
    const double u = sn * sn / (2.0 * (1.0 - x));
    Zd h0, h1;
    if (u * (zabs(c.kappa) + 1.0) <= 0.5) {
        greenc_h01_far(c, u, h0, h1);
    } else {
        h0 = greenc_series(0, c.kappa, 1.0 - u);
        h1 = greenc_series(1, c.kappa, 1.0 - u);
    }
    h[0] = h0.re;
    h[1] = h0.im;
    if (m_hi >= 1) {
        h[2] = h1.re;
        h[3] = h1.im;
    }
    const double opx = 2.0 * u, omx = 1.0 - x;
    const double ratio = opx / omx, cross = -2.0 * x / opx;
    for (int k = 0; k + 2 <= m_hi; ++k) {
        const double dk = (double)k;
        const Zd q = {(dk + 1.0) * (dk + 2.0) + c.kappa.re, c.kappa.im};
        const Zd f = zdiv({(dk + 1.0) * (dk + 2.0) * ratio, 0.0}, q);
        const Zd h2 = zmul(f, zadd(h0, zscale(h1, cross)));
        h[2 * (k + 2)] = h2.re;
        h[2 * (k + 2) + 1] = h2.im;
        h0 = h1;
        h1 = h2;
    }
}

// J_pq between rings 1 (lower value) and 2 from kappa_1's tables: hn1[k] = G_{m+k}(-z1),
// hp2[k] = G_{m+k}(z2), rm = Pi_m / m!^2 of kappa_1
__device__ void greenc2_pair(const GreenConstC& c, Zd rm, int m, double z1, double s1, double z2, double s2,
                             const Zd (&hn1)[2], const Zd (&hp2)[2], double (&J)[4])
{
    double wm = 1.0, lp1, lm1, lp2, lm2;
    green_logs(z1, s1, lp1, lm1);
    green_logs(z2, s2, lp2, lm2);
    if (z1 != z2 && m > 0) wm = exp(0.5 * (double)m * ((lp1 - lm1) + (lm2 - lp2)));
    const double r1 = exp(0.5 * (lp1 - lm1)), r2 = exp(0.5 * (lm2 - lp2));
    // 2 b_1 = i / beta
    const Zd sc = zmul({0.0, 1.0 / c.beta}, zscale(zmul(rm, c.sc), wm));
    const Zd a = zscale({(double)m * m + m + c.kappa.re, c.kappa.im}, 1.0 / (m + 1.0));
    const Zd u[2] = {hn1[0], zscale(zmul(a, hn1[1]), -r1)};
    const Zd v[2] = {hp2[0], zscale(zmul(a, hp2[1]), r2)};
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) J[p * 2 + q] = zmul(sc, zmul(u[p], v[q])).re;
}

// One thread per (set j, mode m) for the conjugate pair, sets and mirror as in factor_kernel.
__global__ __launch_bounds__(64) void greenc2_factor_kernel(Geometry g, const double* __restrict__ zgrid, GreenConstC c,
                                                            int south, int w, const double* __restrict__ hp,
                                                            const double* __restrict__ hn, double* __restrict__ f64,
                                                            float* __restrict__ f32)
{
    const int j = blockIdx.x * 64 + threadIdx.x;
    const int m = blockIdx.y;
    if (j >= g.n_sets) return;
    const bool mirror = south && j >= (g.even ? 2 : 1);
    int a, b;
    if (mirror) {
        a = g.s + j - 1; b = g.s + j;
    } else if (j == 0) {
        a = b = g.s;
    } else if (g.even) {
        if (j == 1) { a = g.s; b = g.s + 1; }
        else { a = g.s - j + 2; b = g.s - j + 1; }
    } else {
        a = g.s - j + 1; b = g.s - j;
    }
    Zd rm = {1.0, 0.0};
    for (int k = 1; k <= m; ++k) {
        const double dk = (double)k;
        rm = zmul(rm, zscale({dk * dk - dk + c.kappa.re, c.kappa.im}, 1.0 / (dk * dk)));
    }
    double za, sa, zb, sb;
    green_ring(g, zgrid, a, za, sa);
    green_ring(g, zgrid, b, zb, sb);
    Zd hna[2], hpa[2], hnb[2], hpb[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const size_t oa = 2 * ((size_t)a * w + m + k), ob = 2 * ((size_t)b * w + m + k);
        hna[k] = {hn[oa], hn[oa + 1]};
        hpa[k] = {hp[oa], hp[oa + 1]};
        hnb[k] = {hn[ob], hn[ob + 1]};
        hpb[k] = {hp[ob], hp[ob + 1]};
    }
    double Ja[4], Jb[4], Jx[4];
    greenc2_pair(c, rm, m, za, sa, za, sa, hna, hpa, Ja);
    const double kaa[3] = {Ja[0], 0.5 * (Ja[1] + Ja[2]), Ja[3]};
    double A[4] = {0, 0, 0, 0}, B[3];
    if (j == 0) {
        start_m2(kaa, B);
    } else {
        greenc2_pair(c, rm, m, zb, sb, zb, sb, hnb, hpb, Jb);
        const double kbb[3] = {Jb[0], 0.5 * (Jb[1] + Jb[2]), Jb[3]};
        double kba[4];
        if (zb <= za) {
            greenc2_pair(c, rm, m, zb, sb, za, sa, hnb, hpa, Jx);
            kba[0] = Jx[0]; kba[1] = Jx[1]; kba[2] = Jx[2]; kba[3] = Jx[3];
        } else {
            greenc2_pair(c, rm, m, za, sa, zb, sb, hna, hpb, Jx);
            kba[0] = Jx[0]; kba[1] = Jx[2]; kba[2] = Jx[1]; kba[3] = Jx[3];
        }
        factors_m2(kaa, kbb, kba, A, B);
    }
    if (mirror) {
        A[1] = -A[1];
        A[2] = -A[2];
        B[1] = -B[1];
    }
    const size_t base = ((size_t)j * g.m_rows + m) * factor_stride(2);
    const double v[8] = {A[0], A[1], A[2], A[3], B[0], B[1], B[2], 0.0};
#pragma unroll
    for (int i = 0; i < 8; ++i) f64[base + i] = v[i];
    if (f32) {
#pragma unroll
        for (int i = 0; i < 8; ++i) f32[base + i] = (float)v[i];
    }
}

}  // namespace

hipError_t launch_phi(const Geometry& g, const double* f64, int blocks, double* phi64, float* phi32,
                      hipStream_t st)
{
    dim3 grid((g.m_top + 64) / 64, blocks);
    switch (g.order) {
        case 1: hipLaunchKernelGGL(phi_kernel<1>, grid, dim3(64), 0, st, g, f64, blocks, phi64, phi32); break;
        case 2: hipLaunchKernelGGL(phi_kernel<2>, grid, dim3(64), 0, st, g, f64, blocks, phi64, phi32); break;
        case 3: hipLaunchKernelGGL(phi_kernel<3>, grid, dim3(64), 0, st, g, f64, blocks, phi64, phi32); break;
        case 4: hipLaunchKernelGGL(phi_kernel<4>, grid, dim3(64), 0, st, g, f64, blocks, phi64, phi32); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_spectrum(const double* kappa_dev, int n_kappa, const double* c_explicit_dev,
                           int ell_max, double* C_dev, int* bad_dev, hipStream_t st)
{
    const int n = ell_max + 1;
    hipLaunchKernelGGL(spectrum_kernel, dim3((n + 255) / 256), dim3(256), 0, st, kappa_dev,
                       n_kappa, c_explicit_dev, ell_max, C_dev, bad_dev);
    return hipGetLastError();
}

hipError_t launch_factors(const Geometry& g, const double* C_dev, const double* z_dev, int south, int ubasis,
                          double* f64, float* f32, hipStream_t st)
{
    dim3 grid((g.n_sets + 63) / 64, g.m_top + 1);
    if (ubasis) {
        if (g.order != 2) return hipErrorInvalidValue;
        hipLaunchKernelGGL((factor_kernel<2, true>), grid, dim3(64), 0, st, g, C_dev, z_dev, south, f64, f32);
        return hipGetLastError();
    }
    switch (g.order) {
        case 1: hipLaunchKernelGGL(factor_kernel<1>, grid, dim3(64), 0, st, g, C_dev, z_dev, south, f64, f32); break;
        case 2: hipLaunchKernelGGL(factor_kernel<2>, grid, dim3(64), 0, st, g, C_dev, z_dev, south, f64, f32); break;
        case 3: hipLaunchKernelGGL(factor_kernel<3>, grid, dim3(64), 0, st, g, C_dev, z_dev, south, f64, f32); break;
        case 4: hipLaunchKernelGGL(factor_kernel<4>, grid, dim3(64), 0, st, g, C_dev, z_dev, south, f64, f32); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_green_tables(const Geometry& g, int n_kappa, const double* kappa, const double* z_dev, double* hp,
                               double* hn, hipStream_t st)
{
    const int m_hi = g.m_top + (g.order - 1), w = g.m_rows + 1;
    const size_t tstride = (size_t)g.n_theta * w;
    for (int i = 0; i < n_kappa; ++i) {
        GreenConst c = green_const(kappa[i]);
        hipLaunchKernelGGL(green_series_kernel, dim3((m_hi + 64) / 64, g.n_theta), dim3(64), 0, st, g, z_dev, c, m_hi,
                           w, hp + i * tstride, hn + i * tstride);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(green_recur_kernel, dim3((g.n_theta + 63) / 64), dim3(64), 0, st, g, z_dev, c, m_hi, w,
                           hp + i * tstride, hn + i * tstride);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_factors_green(const Geometry& g, const double* kappa, const double* z_dev, int south,
                                const double* hp, const double* hn, double* f64, float* f32, hipStream_t st)
{
    const int w = g.m_rows + 1;
    const dim3 grid((g.n_sets + 63) / 64, g.m_top + 1);
    if (g.order == 1) {
        hipLaunchKernelGGL(green_factor_kernel, grid, dim3(64), 0, st, g, z_dev, green_const(kappa[0]), south, w, hp,
                           hn, f64, f32);
    } else if (g.order == 2) {
        hipLaunchKernelGGL(green2_factor_kernel, grid, dim3(64), 0, st, g, z_dev, green_const(kappa[0]),
                           green_const(kappa[1]), south, w, hp, hn, f64, f32);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_twiddles(int n_phi, double* tw64, float* tw32, hipStream_t st)
{
    hipLaunchKernelGGL(twiddle_kernel, dim3((n_phi + 255) / 256), dim3(256), 0, st, n_phi, tw64,
                       tw32);
    return hipGetLastError();
}

hipError_t launch_green_pair(const Geometry& g, double alpha, double beta, const double* z_dev, int south,
                              double* hp, double* hn, double* f64, float* f32, hipStream_t st)
{
    if (g.order != 2 || !(beta > 0.0)) return hipErrorInvalidValue;
    const GreenConstC c = greenc_const(alpha, beta);
    const int m_hi = g.m_top + 1, w = g.m_rows + 1;
    hipLaunchKernelGGL(greenc_series_kernel, dim3((m_hi + 64) / 64, g.n_theta), dim3(64), 0, st, g, z_dev, c, m_hi, w,
                       hp, hn);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(greenc_recur_kernel, dim3((g.n_theta + 63) / 64), dim3(64), 0, st, g, z_dev, c, m_hi, w, hp,
                       hn);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((g.n_sets + 63) / 64, g.m_top + 1);
    hipLaunchKernelGGL(greenc2_factor_kernel, grid, dim3(64), 0, st, g, z_dev, c, south, w, hp, hn, f64, f32);
    return hipGetLastError();
}

}  // namespace smf
