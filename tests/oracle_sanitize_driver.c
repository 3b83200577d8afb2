/* Test infrastructure: a driver that calls the oracle's entry points on small inputs, built
 * together with oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitizers.py, so that any out-of-bounds access, leak or undefined
 * operation in the oracle is reported.  Exit status: 0 when every call returned its success
 * code, 1 otherwise (the sanitizers abort on their own findings). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_n_sets(int n_theta);
int orc_m_top(int ell_max, int n_phi);
void orc_grid(int n_theta, double* theta, double* z);
int orc_spectrum(int n_kappa, const double* kappa, int ell_max, double* C);
int orc_spectrum_complex(int n_kappa, const double* kre, const double* kim, int ell_max, double* C);
void orc_legendre(int m, int ell_max, double theta, double* L, double* dL);
void orc_jblock(int order, int m, int ell_max, const double* C, double theta1, double theta2, double* J);
void orc_jblock_green(int m, double kappa, double z1, double s1, double z2, double s2, double* J);
void orc_jblock_green2(int m, const double* kap, double z1, double s1, double z2, double s2, double* J);
void orc_jblock_green2c(int m, const double* kap, double z1, double s1, double z2, double s2, double* J);
void orc_greenc_G(int m, double kre, double kim, double x, double s, double* out);
double orc_green_G(int m, double kappa, double x, double s);
double orc_green_P(int m, double kappa, double x, double s);
int orc_setup_modes_zb(int order, int basis, int ell_max, const double* C, int n_theta, const double* zgrid,
                       int n_sets, const int* modes, int n_modes, double* A, double* B);
int orc_setup_modes_asym_b(int order, int basis, int ell_max, const double* C, int n_theta, const double* zgrid,
                           int n_sets, const int* modes, int n_modes, double* A, double* B, double* As, double* Bs);
int orc_sample_modes_list_south(int order, int n_theta, const int* modes, int n_modes, int n_sets,
                                const double* A, const double* B, const double* As, const double* Bs,
                                uint64_t seed, int count, double* g);
int orc_dft(int n_theta, int n_phi, int m_top, int count, int r0, int r1, const double* g, double* T);
int orc_dft_rings(int n_theta, int m_top, int count, const int* n_ring, const double* phi0,
                  const int64_t* off, const double* g, double* T);
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
double orc_normal(uint64_t key, int m, int part, int ring, int order, int q);

static int failures = 0;

static void check(int ok, const char* what)
{
    if (!ok) {
        fprintf(stderr, "oracle call failed: %s\n", what);
        ++failures;
    }
}

static double* zeros(size_t n)
{
    double* p = (double*)calloc(n ? n : 1, sizeof(double));
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* Alg. 1 then Alg. 2 (chains, then the DFT) for one grid and basis; zgrid NULL for ring
 * centres, asym != 0 for the southern walk's own factor sets. */
static void setup_and_sample(int order, int basis, int ell_max, const double* C, int n_theta, int n_phi,
                             const double* zgrid, int asym, const char* what)
{
    const int ns = orc_n_sets(n_theta);
    const int m_top = orc_m_top(ell_max, n_phi);
    const int nm = m_top + 1;
    const int count = 2;
    int* modes = (int*)malloc(sizeof(int) * (size_t)nm);
    if (!modes) exit(2);
    for (int m = 0; m < nm; ++m) modes[m] = m;
    const size_t nf = (size_t)ns * nm * order * order;
    double *A = zeros(nf), *B = zeros(nf), *As = asym ? zeros(nf) : NULL, *Bs = asym ? zeros(nf) : NULL;
    int rc = asym ? orc_setup_modes_asym_b(order, basis, ell_max, C, n_theta, zgrid, ns, modes, nm, A, B, As, Bs)
                  : orc_setup_modes_zb(order, basis, ell_max, C, n_theta, zgrid, ns, modes, nm, A, B);
    check(rc == 0, what);
    double* g = zeros((size_t)count * n_theta * nm * 2);
    double* T = zeros((size_t)count * n_theta * n_phi);
    rc = orc_sample_modes_list_south(order, n_theta, modes, nm, ns, A, B, As, Bs, 12345u, count, g);
    check(rc == 0, what);
    rc = orc_dft(n_theta, n_phi, m_top, count, 0, n_theta, g, T);
    check(rc == 0, what);
    for (size_t i = 0; i < (size_t)count * n_theta * n_phi; ++i) check(isfinite(T[i]), what);
    free(modes);
    free(A);
    free(B);
    free(As);
    free(Bs);
    free(g);
    free(T);
}

int main(void)
{
    const double kappa[4] = {9.0, 16.0, 25.0, 36.0};
    const int ell_max = 12, n_phi = 32;
    double* C = zeros(ell_max + 1);

    /* orders 1 to 4, even and odd grids, ring centres */
    for (int order = 1; order <= 4; ++order) {
        check(orc_spectrum(order, kappa, ell_max, C) == 0, "spectrum");
        setup_and_sample(order, 0, ell_max, C, 8, n_phi, NULL, 0, "setup, even grid");
        setup_and_sample(order, 0, ell_max, C, 7, n_phi, NULL, 0, "setup, odd grid");
        setup_and_sample(order, 0, ell_max, C, 2, n_phi, NULL, 0, "setup, two rings");
    }
    /* an explicit grid with no symmetry, and the U basis at order 2 */
    check(orc_spectrum(2, kappa, ell_max, C) == 0, "spectrum");
    double z[9];
    for (int i = 0; i < 9; ++i) z[i] = 0.9 - 0.21 * i - 0.003 * i * i;
    setup_and_sample(2, 0, ell_max, C, 9, n_phi, z, 1, "asymmetric grid");
    setup_and_sample(2, 1, ell_max, C, 8, n_phi, NULL, 0, "U basis");
    /* the Green's-function setups of Sec. 3 (no band limit: every mode below n_phi / 2) */
    const double kg1[1] = {40.0}, kg2[2] = {16.0, 400.0};
    setup_and_sample(1, 2, 0, kg1, 8, n_phi, NULL, 0, "Green order 1");
    setup_and_sample(2, 3, 0, kg2, 7, n_phi, NULL, 0, "Green order 2");
    const double kpair[2] = {0.0, sqrt(10.0)};
    setup_and_sample(2, 4, 0, kpair, 8, n_phi, NULL, 0, "Green order 2, conjugate pair");
    /* the paper's complex pair kappa = +-i sqrt(10) */
    const double kre[2] = {0.0, 0.0}, kim[2] = {sqrt(10.0), -sqrt(10.0)};
    check(orc_spectrum_complex(2, kre, kim, ell_max, C) == 0, "complex spectrum");

    /* pieces on their own */
    double L[13], dL[13], J[16], th[8], zz[8];
    orc_grid(8, th, zz);
    orc_legendre(3, ell_max, 0.7, L, dL);
    orc_jblock(3, 2, ell_max, C, 0.4, 1.1, J);
    orc_jblock_green(5, 40.0, -0.3, sqrt(1 - 0.09), 0.6, 0.8, J);
    orc_jblock_green2(5, kg2, -0.3, sqrt(1 - 0.09), 0.6, 0.8, J);
    orc_jblock_green2c(5, kpair, -0.3, sqrt(1 - 0.09), 0.6, 0.8, J);
    double gc[2];
    orc_greenc_G(7, 2.0, 5.0, -0.95, sqrt(1 - 0.95 * 0.95), gc);
    check(isfinite(gc[0]) && isfinite(gc[1]), "Green G, complex degree");
    check(isfinite(orc_green_G(7, 0.2, -0.95, sqrt(1 - 0.95 * 0.95))), "Green G, real degree");
    check(isfinite(orc_green_P(7, 40.0, 0.5, sqrt(0.75))), "Green P");
    const uint32_t ctr[4] = {1u, 2u, 3u, 4u}, key[2] = {5u, 6u};
    uint32_t out[4];
    orc_philox(ctr, key, out);
    check(isfinite(orc_normal(7u, 3, 1, 2, 2, 1)), "normal");

    /* rings with their own pixel counts, modes aliasing on the short ones */
    const int nr = 5;
    const int n_ring[5] = {2, 6, 10, 14, 32};
    const double phi0[5] = {0.0, 0.3, 1.0, 2.0, 0.05};
    int64_t off[6] = {0};
    for (int i = 0; i < nr; ++i) off[i + 1] = off[i] + n_ring[i];
    const int mt = 20, count = 2;
    double* g = zeros((size_t)count * nr * (mt + 1) * 2);
    for (size_t i = 0; i < (size_t)count * nr * (mt + 1) * 2; ++i) g[i] = sin(0.37 * (double)i);
    double* T = zeros((size_t)count * off[nr]);
    check(orc_dft_rings(nr, mt, count, n_ring, phi0, off, g, T) == 0, "dft_rings");
    free(g);
    free(T);
    free(C);
    if (failures) fprintf(stderr, "%d oracle calls failed\n", failures);
    else printf("oracle sanitizer driver: every call succeeded\n");
    return failures ? 1 : 0;
}
