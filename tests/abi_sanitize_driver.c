/* Test infrastructure: a driver of the C ABI's host logic (argument checks, error paths,
 * error strings) for a build of the library whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer, run by tests/test_oracle_sanitizers.py on a machine with or
 * without a GPU: every call below either rejects its arguments before any device work or
 * reports a missing device.  Exit status 0 when every call returned an expected code. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "smf.h"

static int failures = 0;

static void expect(int rc, int want, int or_want, const char* what)
{
    if (rc != want && rc != or_want) {
        fprintf(stderr, "%s: returned %d (%s)\n", what, rc, smf_error_string(rc));
        ++failures;
    }
}

int main(void)
{
    const double kappa[2] = {9.0, 16.0};
    double c_ell[17];
    for (int l = 0; l <= 16; ++l) c_ell[l] = 1.0 / (1.0 + l * (l + 1.0));
    smf_spectrum ok = {2, 2, kappa, NULL, 16};
    smf_plan* plan = (smf_plan*)0x1;

    expect(smf_set_log_level(-1), SMF_EINVAL, SMF_EINVAL, "log level -1");
    if (smf_set_log_level(1) < 0) ++failures;   /* the rejections below are also explained on stderr */
    for (int code = -6; code <= 1; ++code)
        if (!smf_error_string(code) || !strlen(smf_error_string(code))) ++failures;

    /* smf_setup: every invalid argument, then a valid one (no device: SMF_EHIP) */
    expect(smf_setup(NULL, 8, 32, SMF_FP64, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "setup NULL spec");
    expect(smf_setup(&ok, 8, 32, SMF_FP64, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "setup NULL out");
    smf_spectrum bad = ok;
    bad.order = 5;
    expect(smf_setup(&bad, 8, 32, SMF_FP64, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "setup order 5");
    bad = ok;
    bad.ell_max = -1;
    expect(smf_setup(&bad, 8, 32, SMF_FP64, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "setup ell_max -1");
    bad = ok;
    bad.kappa = NULL;
    expect(smf_setup(&bad, 8, 32, SMF_FP64, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "setup kappa NULL");
    expect(smf_setup(&ok, 1, 32, SMF_FP64, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "setup one ring");
    expect(smf_setup(&ok, 8, 48, SMF_FP64, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "setup n_phi 48");
    expect(smf_setup(&ok, 8, 32, 3, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "setup flags 3");
    expect(smf_setup(&ok, 8, 32, SMF_FP64 | SMF_FUSED, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "setup fused");
    smf_spectrum one = {1, 1, kappa, NULL, 16};
    expect(smf_setup(&one, 8, 32, SMF_FP64 | SMF_UBASIS, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "U basis order 1");
    smf_spectrum same = {2, 2, (const double[]){4.0, 4.0}, NULL, 16};
    expect(smf_setup(&same, 8, 32, SMF_FP64 | SMF_GREEN, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "Green repeated kappa");
    smf_spectrum pair0 = {2, 2, (const double[]){0.0, 0.0}, NULL, 0};
    expect(smf_setup(&pair0, 8, 32, SMF_FP64 | SMF_GREEN | SMF_KAPPA_PAIR, NULL, &plan), SMF_EINVAL, SMF_EINVAL,
           "pair beta 0");
    smf_spectrum big1 = {1, 1, (const double[]){2e4}, NULL, 0};
    expect(smf_setup(&big1, 8, 32, SMF_FP64 | SMF_GREEN, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "Green kappa 2e4");
    smf_spectrum pair1 = {2, 2, (const double[]){0.0, 3.0}, NULL, 0};
    expect(smf_setup(&pair1, 8, 32, SMF_FP64 | SMF_KAPPA_PAIR, NULL, &plan), SMF_EINVAL, SMF_EINVAL,
           "pair without Green");
    plan = NULL;
    expect(smf_setup(&pair1, 8, 32, SMF_FP64 | SMF_GREEN | SMF_KAPPA_PAIR, NULL, &plan), SMF_EHIP, SMF_OK,
           "pair valid");
    if (plan) smf_destroy(plan);
    smf_spectrum explicit_c = {1, 0, NULL, c_ell, 16};
    expect(smf_setup(&explicit_c, 8, 32, SMF_FP32, NULL, &plan), SMF_EHIP, SMF_OK, "setup explicit C_l");
    expect(smf_setup(&ok, 8, 32, SMF_FP64, NULL, &plan), SMF_EHIP, SMF_OK, "setup valid");
    if (plan && plan != (smf_plan*)0x1) smf_destroy(plan);

    /* explicit grids */
    const double z_bad[4] = {0.5, 0.6, -0.1, -0.5};
    expect(smf_setup_grid(&ok, 4, z_bad, 32, SMF_FP64, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "grid not decreasing");
    const double z_ok[4] = {0.7, 0.2, -0.2, -0.7};
    plan = NULL;
    expect(smf_setup_grid(&ok, 4, z_ok, 32, SMF_FP64, NULL, &plan), SMF_EHIP, SMF_OK, "grid valid");
    if (plan) smf_destroy(plan);

    /* rings */
    const int n_ring[4] = {4, 8, 8, 4};
    const int n_odd[4] = {4, 7, 8, 4};
    const double phi0[4] = {0.1, 0.0, 0.0, 0.1};
    expect(smf_setup_rings(&ok, 4, NULL, n_odd, phi0, SMF_FP32, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "odd ring");
    expect(smf_setup_rings(&ok, 4, NULL, NULL, phi0, SMF_FP32, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "rings NULL");
    /* the FP64 ring limit (4096 pixels) holds with the Green's-function flags too */
    const int n_big[4] = {4, 8192, 8, 4};
    smf_spectrum green1 = {1, 1, kappa, NULL, 16};
    expect(smf_setup_rings(&green1, 4, NULL, n_big, phi0, SMF_FP64 | SMF_GREEN, NULL, &plan), SMF_EINVAL, SMF_EINVAL,
           "FP64 Green ring of 8192 pixels");
    plan = NULL;
    expect(smf_setup_rings(&ok, 4, NULL, n_ring, phi0, SMF_FP32, NULL, &plan), SMF_EHIP, SMF_OK, "rings valid");
    if (plan) smf_destroy(plan);

    /* batch */
    const int nt[2] = {8, 16}, np[2] = {32, 8192};
    smf_spectrum specs[2] = {ok, ok};
    expect(smf_setup_batch(2, specs, nt, np, SMF_FP32, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "batch n_phi 8192");
    expect(smf_setup_batch(0, specs, nt, np, SMF_FP32, NULL, &plan), SMF_EINVAL, SMF_EINVAL, "batch empty");

    /* calls on no plan */
    expect(smf_sample(NULL, 1, 1, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "sample NULL");
    expect(smf_sample_modes(NULL, 1, 1, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "sample_modes NULL");
    expect(smf_transform(NULL, 1, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "transform NULL");
    expect(smf_sample_rings(NULL, 1, 1, NULL, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "sample_rings NULL");
    expect(smf_sample_rings_noalloc(NULL, 1, 1, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "noalloc NULL");
    expect(smf_synthesize_rings(NULL, 1, NULL, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "synthesize NULL");
    expect(smf_sample_batch(NULL, NULL, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "batch sample NULL");
    expect(smf_measure_normals(1, 0, 1, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "measure normals bad");
    expect(smf_measure_fma(0, 1, NULL, NULL), SMF_EINVAL, SMF_EINVAL, "measure fma bad");
    expect(smf_debug_fail_alloc(-2), SMF_EINVAL, SMF_EINVAL, "fail_alloc -2");
    expect(smf_debug_fail_alloc(-1), SMF_OK, SMF_OK, "fail_alloc off");
    expect(smf_destroy(NULL), SMF_EINVAL, SMF_OK, "destroy NULL");

    if (failures) fprintf(stderr, "%d unexpected return codes\n", failures);
    else printf("C ABI sanitizer driver: every call returned an expected code\n");
    return failures ? 1 : 0;
}
