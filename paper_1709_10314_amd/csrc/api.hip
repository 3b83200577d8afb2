// C ABI of libsmf: plan creation (Alg. 1 on the GPU), sampling (Alg. 2), queries.
#include <stdlib.h>
#include <string.h>

#include "smf_internal.h"

using smf::Geometry;

namespace {

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Owns the device buffers of a plan under construction; frees them unless released.
struct DevBufs {
    void* p[8] = {nullptr};
    int n = 0;
    template <typename T>
    int alloc(T** out, size_t count)
    {
        void* q = nullptr;
        if (count == 0) count = 1;
        if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            return SMF_ENOMEM;
        }
        p[n++] = q;
        *out = static_cast<T*>(q);
        return SMF_OK;
    }
    void free_all()
    {
        for (int i = 0; i < n; ++i) (void)hipFree(p[i]);
        n = 0;
    }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int setup_impl(const smf_spectrum* spec, int n_theta, int n_phi, int flags, hipStream_t st,
               smf_plan** out)
{
    if (!spec || !out) return SMF_EINVAL;
    *out = nullptr;
    if (spec->order < 1 || spec->order > 2) return SMF_EINVAL;
    if (spec->ell_max < 0 || spec->ell_max > (1 << 20)) return SMF_EINVAL;
    if (!spec->c_ell && (spec->n_kappa < 0 || spec->n_kappa > 64 || (spec->n_kappa > 0 && !spec->kappa)))
        return SMF_EINVAL;
    if (n_theta < 2 || n_theta > (1 << 16)) return SMF_EINVAL;
    if (!is_pow2(n_phi) || n_phi < 4 || n_phi > 16384) return SMF_EINVAL;
    if (flags != SMF_FP64 && flags != SMF_FP32) return SMF_EINVAL;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SMF_EHIP;
    // the FFT holds n_phi/2 complex values of the sample type in LDS
    const size_t lds = (size_t)(n_phi / 2) * (flags == SMF_FP64 ? 16 : 8);
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return SMF_EHIP;
    if (lds > (size_t)lds_max) return SMF_EINVAL;

    const Geometry g = smf::make_geometry(spec->order, n_theta, n_phi, spec->ell_max);
    DevBufs bufs;
    smf_plan* plan = (smf_plan*)calloc(1, sizeof(smf_plan));
    if (!plan) return SMF_ENOMEM;
    plan->g = g;
    plan->flags = flags;
    plan->device = dev;

    int rc = SMF_OK;
    double* kappa_dev = nullptr;
    double* cexp_dev = nullptr;
    int* bad_dev = nullptr;
    int bad = 0;
    const size_t nrec = (size_t)g.n_sets * g.m_rows * smf::factor_stride(g.order);
    hipError_t e = hipSuccess;

    if ((rc = bufs.alloc(&plan->C, (size_t)g.ell_max + 1))) goto fail;
    if ((rc = bufs.alloc(&bad_dev, 1))) goto fail;
    if (spec->c_ell) {
        if ((rc = bufs.alloc(&cexp_dev, (size_t)g.ell_max + 1))) goto fail;
        e = hipMemcpyAsync(cexp_dev, spec->c_ell, sizeof(double) * (g.ell_max + 1),
                           hipMemcpyHostToDevice, st);
    } else if (spec->n_kappa > 0) {
        if ((rc = bufs.alloc(&kappa_dev, (size_t)spec->n_kappa))) goto fail;
        e = hipMemcpyAsync(kappa_dev, spec->kappa, sizeof(double) * spec->n_kappa,
                           hipMemcpyHostToDevice, st);
    }
    if (e != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (hipMemsetAsync(bad_dev, 0, sizeof(int), st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (smf::launch_spectrum(kappa_dev, spec->c_ell ? 0 : spec->n_kappa, cexp_dev, g.ell_max,
                             plan->C, bad_dev, st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (hipMemcpyAsync(&bad, bad_dev, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (bad) { rc = SMF_ENUMERIC; goto fail; }

    if ((rc = bufs.alloc(&plan->f64, nrec))) goto fail;
    if (hipMemsetAsync(plan->f64, 0, nrec * sizeof(double), st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (flags == SMF_FP32) {
        if ((rc = bufs.alloc(&plan->f32, nrec))) goto fail;
        if (hipMemsetAsync(plan->f32, 0, nrec * sizeof(float), st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    }
    if (smf::launch_factors(g, plan->C, plan->f64, plan->f32, st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if ((rc = bufs.alloc(&plan->tw64, (size_t)2 * n_phi))) goto fail;
    if ((rc = bufs.alloc(&plan->tw32, (size_t)2 * n_phi))) goto fail;
    if (smf::launch_twiddles(n_phi, plan->tw64, plan->tw32, st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (hipStreamSynchronize(st) != hipSuccess) { rc = SMF_EHIP; goto fail; }

    // scratch used only during setup
    (void)hipFree(bad_dev);
    if (kappa_dev) (void)hipFree(kappa_dev);
    if (cexp_dev) (void)hipFree(cexp_dev);
    *out = plan;
    return SMF_OK;

fail:
    (void)hipStreamSynchronize(st);
    bufs.free_all();
    free(plan);
    return rc;
}

}  // namespace

extern "C" {

int smf_setup(const smf_spectrum* spec, int n_theta, int n_phi, int flags, void* hip_stream,
              smf_plan** out)
{
    return setup_impl(spec, n_theta, n_phi, flags, (hipStream_t)hip_stream, out);
}

static int sample_common(const smf_plan* plan, uint64_t seed, int count, void* out_dev,
                         void* hip_stream, bool fft)
{
    if (!plan || count < 0) return SMF_EINVAL;
    if (count == 0) return SMF_OK;
    if (!out_dev) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    hipStream_t st = (hipStream_t)hip_stream;
    const int fp64 = plan->flags == SMF_FP64;
    const void* fac = fp64 ? (const void*)plan->f64 : (const void*)plan->f32;
    if (smf::launch_recursion(plan->g, fp64, fac, seed, count, out_dev, st) != hipSuccess)
        return SMF_EHIP;
    if (fft) {
        const void* tw = fp64 ? (const void*)plan->tw64 : (const void*)plan->tw32;
        if (smf::launch_c2r(plan->g, fp64, tw, count, out_dev, st) != hipSuccess) return SMF_EHIP;
    }
    return SMF_OK;
}

int smf_sample(const smf_plan* plan, uint64_t seed, int count, void* out_dev, void* hip_stream)
{
    return sample_common(plan, seed, count, out_dev, hip_stream, true);
}

int smf_sample_modes(const smf_plan* plan, uint64_t seed, int count, void* g_dev, void* hip_stream)
{
    return sample_common(plan, seed, count, g_dev, hip_stream, false);
}

int smf_plan_dims(const smf_plan* plan, int* dims)
{
    if (!plan || !dims) return SMF_EINVAL;
    const Geometry& g = plan->g;
    dims[0] = g.order;
    dims[1] = g.n_theta;
    dims[2] = g.n_phi;
    dims[3] = g.ell_max;
    dims[4] = g.m_top;
    dims[5] = g.n_sets;
    dims[6] = g.s;
    dims[7] = plan->flags;
    return SMF_OK;
}

int smf_get_factors(const smf_plan* plan, double* A_host, double* B_host)
{
    if (!plan || !A_host || !B_host) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    const Geometry& g = plan->g;
    const int M = g.order, E = smf::factor_stride(M);
    const size_t nrec = (size_t)g.n_sets * g.m_rows * E;
    double* tmp = (double*)malloc(nrec * sizeof(double));
    if (!tmp) return SMF_ENOMEM;
    if (hipMemcpy(tmp, plan->f64, nrec * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
        free(tmp);
        return SMF_EHIP;
    }
    for (int j = 0; j < g.n_sets; ++j)
        for (int m = 0; m <= g.m_top; ++m) {
            const double* r = tmp + ((size_t)j * g.m_rows + m) * E;
            double* A = A_host + ((size_t)j * (g.m_top + 1) + m) * M * M;
            double* B = B_host + ((size_t)j * (g.m_top + 1) + m) * M * M;
            if (M == 1) {
                A[0] = r[0];
                B[0] = r[1];
            } else {
                A[0] = r[0]; A[1] = r[1]; A[2] = r[2]; A[3] = r[3];
                B[0] = r[4]; B[1] = 0.0; B[2] = r[5]; B[3] = r[6];
            }
        }
    free(tmp);
    return SMF_OK;
}

int smf_destroy(smf_plan* plan)
{
    if (!plan) return SMF_OK;
    DeviceGuard dg(plan->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(plan->C);
    (void)hipFree(plan->f64);
    if (plan->f32) (void)hipFree(plan->f32);
    (void)hipFree(plan->tw64);
    (void)hipFree(plan->tw32);
    free(plan);
    return SMF_OK;
}

const char* smf_error_string(int code)
{
    switch (code) {
        case SMF_OK: return "success";
        case SMF_EINVAL: return "invalid argument";
        case SMF_ENOMEM: return "device memory allocation failed";
        case SMF_EHIP: return "HIP runtime error";
        case SMF_ENUMERIC: return "spectrum has a C_l that is not finite and positive";
        default: return "unknown error code";
    }
}

}  // extern "C"
