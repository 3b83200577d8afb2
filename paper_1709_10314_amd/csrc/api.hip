// C ABI of libsmf: plan creation (Alg. 1 on the GPU), sampling (Alg. 2), queries.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <vector>

#include "batch.h"
#include "green_pair.h"
#include "smf_internal.h"

using smf::Geometry;

namespace smf {
// Host state of a batch plan: one FP32 sub-plan per field plus the device work lists.
struct BatchState {
    int n = 0;
    std::vector<smf_plan*> sub;
    std::vector<int64_t> offsets;        // n + 1 packed-output offsets (elements)
    BatchField* fields_dev = nullptr;
    uint32_t* chain_dev[3] = {nullptr, nullptr, nullptr};   // items for 1, 2, 4 m-tiles
    int n_chain[3] = {0, 0, 0};
    uint32_t* fft_dev = nullptr;
    int n_fft = 0;
    size_t lds = 0;
    int tiles_idx = 1;                   // current tile shape: 2 m-tiles per item
    int persistent = 0;                  // 1: one cooperative launch (launch_batch_persistent)
    // per-field keys and buffers of smf_sample_batch: kCallSlots tables of n entries in
    // device memory, staged through pinned host memory; slot k is reused only after the
    // event recorded behind the previous call that used it has completed
    static constexpr int kCallSlots = 4;
    BatchCall* call_dev = nullptr;
    BatchCall* call_host = nullptr;
    hipEvent_t call_ev[kCallSlots] = {};
    int call_next = 0;
    std::mutex call_mu;
};
}  // namespace smf

// ---- diagnostics ----
// Level from smf_set_log_level, else from the environment variable SMF_LOG (0 when unset): 1
// prints each plan's setup (geometry, layout choices, sizes, time) and the reason for each
// rejected argument of a setup; 2 also each sampling call's launch shape.  One line per event to
// stderr, prefixed "[smf] ".
static std::atomic<int> g_log_level{-1};

static int log_level()
{
    int l = g_log_level.load(std::memory_order_relaxed);
    if (l >= 0) return l;
    const char* e = getenv("SMF_LOG");
    int v = e ? atoi(e) : 0;
    if (v < 0) v = 0;
    int expected = -1;
    g_log_level.compare_exchange_strong(expected, v);
    return g_log_level.load(std::memory_order_relaxed);
}

__attribute__((format(printf, 2, 3))) static void log_line(int level, const char* fmt, ...)
{
    if (log_level() < level) return;
    char buf[640] = "[smf] ";
    const size_t p = strlen(buf);
    va_list ap;
    va_start(ap, fmt);
    int n = vsnprintf(buf + p, sizeof(buf) - p - 1, fmt, ap);
    va_end(ap);
    if (n < 0) return;
    size_t end = p + (size_t)n;
    if (end > sizeof(buf) - 2) end = sizeof(buf) - 2;
    buf[end] = '\n';
    buf[end + 1] = '\0';
    fputs(buf, stderr);   // one call per line, so that lines of concurrent calls do not interleave
}

// SMF_EINVAL with its reason logged at level 1
static int reject(const char* where, const char* why)
{
    log_line(1, "%s: invalid argument: %s", where, why);
    return SMF_EINVAL;
}

namespace {

// Allocation failure injection (smf_debug_fail_alloc): the number of device or pinned host
// allocations to let through before one fails, or -1 (off).
std::atomic<int> g_fail_after{-1};

bool injected_failure()
{
    int n = g_fail_after.load();
    while (n >= 0) {
        if (g_fail_after.compare_exchange_weak(n, n - 1)) return n == 0;
    }
    return false;
}

// Every device allocation of the library goes through these two.
hipError_t dev_malloc(void** p, size_t bytes)
{
    if (injected_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

hipError_t host_malloc_pinned(void** p, size_t bytes)
{
    if (injected_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipHostMalloc(p, bytes, 0);
}

void free_call_slots(smf::BatchState* b)
{
    if (b->call_dev) (void)hipFree(b->call_dev);
    if (b->call_host) (void)hipHostFree(b->call_host);
    for (int k = 0; k < smf::BatchState::kCallSlots; ++k)
        if (b->call_ev[k]) (void)hipEventDestroy(b->call_ev[k]);
    b->call_dev = nullptr;
    b->call_host = nullptr;
}


bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Owns the device buffers of a plan under construction; frees them unless released.
struct DevBufs {
    void* p[16] = {nullptr};
    int n = 0;
    template <typename T>
    int alloc(T** out, size_t count)
    {
        void* q = nullptr;
        if (n == 16) return SMF_ENOMEM;
        if (count == 0) count = 1;
        if (dev_malloc(&q, count * sizeof(T)) != hipSuccess) {
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

// An explicit grid: n_theta finite values strictly decreasing in (-1, 1).
bool grid_ok(const double* z, int n)
{
    for (int i = 0; i < n; ++i) {
        if (!(z[i] > -1.0 && z[i] < 1.0)) return false;
        if (i > 0 && !(z[i] < z[i - 1])) return false;
    }
    return true;
}

// Symmetric about the equator to the bit, z[n-1-i] == -z[i] (an odd grid then has z = 0
// at its middle ring): the south mirrors the northern sets.
bool grid_symmetric(const double* z, int n)
{
    for (int i = 0; i < n; ++i)
        if (z[n - 1 - i] != -z[i]) return false;
    return true;
}

// `scan`: also build the block transitions of the affine scan (single-field plans; the
// sub-plans of a batch only ever run the plain recursion).  z_host: explicit ring values
// (host, n_theta), or null for the ring centres.
// rows: chain rows of the plan (0: n_phi / 2, every mode slot of the FFT layout); a ring plan,
// which never transforms in place, keeps only the tiles that hold modes up to m_top.
int setup_impl(const smf_spectrum* spec, int n_theta, const double* z_host, int n_phi, int flags,
               hipStream_t st, bool scan, smf_plan** out, int rows = 0)
{
    const char* W = "smf_setup";
    if (!spec || !out) return reject(W, "spec or out is NULL");
    *out = nullptr;
    if (spec->order < 1 || spec->order > 4) return reject(W, "order must be 1, 2, 3 or 4");
    if (spec->ell_max < 0 || spec->ell_max > (1 << 20)) return reject(W, "ell_max must be in [0, 2^20]");
    if (!spec->c_ell && (spec->n_kappa < 0 || spec->n_kappa > 64 || (spec->n_kappa > 0 && !spec->kappa)))
        return reject(W, "n_kappa must be in [0, 64] with kappa given, or c_ell given");
    if (n_theta < 2 || n_theta > (1 << 16)) return reject(W, "n_theta must be in [2, 65536]");
    if (!is_pow2(n_phi) || n_phi < 4 || n_phi > 16384) return reject(W, "n_phi must be a power of two in [4, 16384]");
    const int ubasis = (flags & SMF_UBASIS) ? 1 : 0;
    const int no_mirror = (flags & SMF_NO_MIRROR) ? 1 : 0;
    const int green = (flags & SMF_GREEN) ? 1 : 0;
    const int pair = (flags & SMF_KAPPA_PAIR) ? 1 : 0;
    flags &= ~(SMF_UBASIS | SMF_NO_MIRROR | SMF_GREEN | SMF_KAPPA_PAIR);
    if (flags != SMF_FP64 && flags != SMF_FP32)
        return reject(W, "flags must hold exactly one of SMF_FP64, SMF_FP32 (SMF_FUSED is not supported)");
    if (ubasis && spec->order != 2) return reject(W, "SMF_UBASIS needs order 2");
    if (pair && (!green || spec->order != 2)) return reject(W, "SMF_KAPPA_PAIR needs SMF_GREEN at order 2");
    if (green) {
        // order 1 with one kappa, or order 2 with two distinct ones, all finite and positive, or
        // the pair alpha +- i beta given as (alpha, beta), beta > 0
        if (spec->order > 2 || ubasis || spec->c_ell || spec->n_kappa != spec->order || !spec->kappa ||
            (long long)spec->order * n_theta * (n_phi / 2 + 1) > smf::kGreenMaxTable)
            return reject(W, "SMF_GREEN needs order 1 or 2 with n_kappa = order, no c_ell, no SMF_UBASIS");
        // G_m and sin(pi lambda) grow like exp(pi sqrt|kappa|) and are formed in FP64, with their
        // products: |kappa| is held to kGreenMaxKappa, where they stay below about 1e137 (the
        // products leave the FP64 range near |kappa| = 1e5)
        constexpr double kGreenMaxKappa = 1e4;
        // and below 1e-5 the continuation about t = 1 loses digits as lambda -> 0 (5e-11 at 1e-7)
        constexpr double kGreenMinKappa = 1e-5;
        if (pair) {
            if (!std::isfinite(spec->kappa[0]) || !std::isfinite(spec->kappa[1]) || !(spec->kappa[1] > 0.0))
                return reject(W, "SMF_KAPPA_PAIR needs a finite alpha and a finite beta > 0");
            // the series of G_m cancels when its terms n^2 + n + kappa turn (alpha < 0) or rotate
            // (beta large): alpha >= -50 and beta <= 1000 keep G_m within about 1e-11
            const double mod = std::hypot(spec->kappa[0], spec->kappa[1]);
            if (!(mod <= kGreenMaxKappa) || !(mod >= kGreenMinKappa) || !(spec->kappa[0] >= -50.0) ||
                !(spec->kappa[1] <= 1000.0))
                return reject(W, "SMF_KAPPA_PAIR needs alpha >= -50, beta <= 1000 and 1e-5 <= |alpha + i beta| <= 1e4");
        } else {
            for (int i = 0; i < spec->n_kappa; ++i)
                if (!(spec->kappa[i] >= kGreenMinKappa) || !(spec->kappa[i] <= kGreenMaxKappa))
                    return reject(W, "SMF_GREEN needs kappa in [1e-5, 1e4]");
            // the partial fractions' weights +-1/(kappa_2 - kappa_1) cancel about
            // log10(kappa / |kappa_2 - kappa_1|) digits of J^m: the roots keep a relative distance
            // of 1e-3, where a field moves by 5e-11 when kappa moves by one unit in the last place
            if (spec->order == 2 && !(std::fabs(spec->kappa[1] - spec->kappa[0]) >=
                                      1e-3 * std::fmax(spec->kappa[0], spec->kappa[1])))
                return reject(W, "SMF_GREEN at order 2 needs |kappa_2 - kappa_1| >= 1e-3 max(kappa)");
        }
    }
    if (z_host && !grid_ok(z_host, n_theta))
        return reject(W, "z must be finite, strictly decreasing and inside (-1, 1)");

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SMF_EHIP;
    // the FFT holds n_phi/2 complex values of the sample type in LDS
    const size_t lds = (size_t)((n_phi / 2) + (n_phi / 32)) * (flags == SMF_FP64 ? 16 : 8);
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return SMF_EHIP;
    if (lds > (size_t)lds_max) return SMF_EINVAL;

    // no band limit with SMF_GREEN: every mode of the FFT layout is sampled, except on a ring
    // plan (rows > 0), whose synthesis stops at ell_max: its chains run the Green's-function
    // factors of the modes up to ell_max
    Geometry g = smf::make_geometry(spec->order, n_theta, n_phi, green && rows == 0 ? n_phi / 2 - 1 : spec->ell_max);
    if (rows > 0 && rows < g.m_rows) g.m_rows = rows;
    DevBufs bufs;
    smf_plan* plan = (smf_plan*)calloc(1, sizeof(smf_plan));
    if (!plan) return SMF_ENOMEM;
    plan->g = g;
    plan->flags = flags;
    plan->device = dev;
    plan->asym = (no_mirror || (z_host && !grid_symmetric(z_host, n_theta))) ? 1 : 0;
    if (z_host) {
        plan->zgrid = (double*)malloc(sizeof(double) * n_theta);
        if (!plan->zgrid) { free(plan); return SMF_ENOMEM; }
        memcpy(plan->zgrid, z_host, sizeof(double) * n_theta);
    }

    int rc = SMF_OK;
    double* kappa_dev = nullptr;
    double* cexp_dev = nullptr;
    double* z_dev = nullptr;
    double* hp_dev = nullptr;   // Green's-function setup tables (setup only)
    double* hn_dev = nullptr;
    int* bad_dev = nullptr;
    int bad = 0;
    // the spectrum as given, or for the pair alpha +- i beta 1/((l(l+1) + alpha)^2 + beta^2) on the host
    const double* c_host = spec->c_ell;
    double* c_pair = nullptr;
    // the northern table, and for a grid with no symmetry the southern walk's own table after it
    const size_t nrec1 = (size_t)g.n_sets * g.m_rows * smf::factor_stride(g.order);
    const size_t nrec = nrec1 * (plan->asym ? 2 : 1);
    hipError_t e = hipSuccess;

    if ((rc = bufs.alloc(&plan->C, (size_t)g.ell_max + 1))) goto fail;
    if ((rc = bufs.alloc(&bad_dev, 1))) goto fail;
    if (pair) {
        c_pair = (double*)malloc(sizeof(double) * ((size_t)g.ell_max + 1));
        if (!c_pair) { rc = SMF_ENOMEM; goto fail; }
        for (int l = 0; l <= g.ell_max; ++l) {
            const double t = (double)l * (l + 1.0) + spec->kappa[0];
            c_pair[l] = 1.0 / (t * t + spec->kappa[1] * spec->kappa[1]);
        }
        c_host = c_pair;
    }
    if (c_host) {
        if ((rc = bufs.alloc(&cexp_dev, (size_t)g.ell_max + 1))) goto fail;
        e = hipMemcpyAsync(cexp_dev, c_host, sizeof(double) * (g.ell_max + 1),
                           hipMemcpyHostToDevice, st);
    } else if (spec->n_kappa > 0) {
        if ((rc = bufs.alloc(&kappa_dev, (size_t)spec->n_kappa))) goto fail;
        e = hipMemcpyAsync(kappa_dev, spec->kappa, sizeof(double) * spec->n_kappa,
                           hipMemcpyHostToDevice, st);
    }
    if (e != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (hipMemsetAsync(bad_dev, 0, sizeof(int), st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (smf::launch_spectrum(kappa_dev, c_host ? 0 : spec->n_kappa, cexp_dev, g.ell_max,
                             plan->C, bad_dev, st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (hipMemcpyAsync(&bad, bad_dev, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    free(c_pair);
    c_pair = nullptr;
    if (bad) { rc = SMF_ENUMERIC; goto fail; }

    if ((rc = bufs.alloc(&plan->f64, nrec))) goto fail;
    if (hipMemsetAsync(plan->f64, 0, nrec * sizeof(double), st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    if (flags == SMF_FP32) {
        if ((rc = bufs.alloc(&plan->f32, nrec))) goto fail;
        if (hipMemsetAsync(plan->f32, 0, nrec * sizeof(float), st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    }
    if (z_host) {
        if ((rc = bufs.alloc(&z_dev, (size_t)n_theta))) goto fail;
        if (hipMemcpyAsync(z_dev, z_host, sizeof(double) * n_theta, hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = SMF_EHIP;
            goto fail;
        }
    }
    plan->south_off = plan->asym ? nrec1 : 0;
    if (green && pair) {
        // kappa_1's complex tables: 2 doubles per entry
        const size_t nt = (size_t)2 * n_theta * (g.m_rows + 1);
        if ((rc = bufs.alloc(&hp_dev, nt))) goto fail;
        if ((rc = bufs.alloc(&hn_dev, nt))) goto fail;
        if (smf::launch_green_pair(g, spec->kappa[0], spec->kappa[1], z_dev, 0, hp_dev, hn_dev, plan->f64, plan->f32,
                                   st) != hipSuccess ||
            (plan->asym && smf::launch_green_pair(g, spec->kappa[0], spec->kappa[1], z_dev, 1, hp_dev, hn_dev,
                                                  plan->f64 + nrec1, plan->f32 ? plan->f32 + nrec1 : nullptr, st) !=
                               hipSuccess)) {
            rc = SMF_EHIP;
            goto fail;
        }
    } else if (green) {
        const size_t nt = (size_t)spec->n_kappa * n_theta * (g.m_rows + 1);
        if ((rc = bufs.alloc(&hp_dev, nt))) goto fail;
        if ((rc = bufs.alloc(&hn_dev, nt))) goto fail;
        if (smf::launch_green_tables(g, spec->n_kappa, spec->kappa, z_dev, hp_dev, hn_dev, st) != hipSuccess ||
            smf::launch_factors_green(g, spec->kappa, z_dev, 0, hp_dev, hn_dev, plan->f64, plan->f32, st) !=
                hipSuccess ||
            (plan->asym && smf::launch_factors_green(g, spec->kappa, z_dev, 1, hp_dev, hn_dev, plan->f64 + nrec1,
                                                     plan->f32 ? plan->f32 + nrec1 : nullptr, st) != hipSuccess)) {
            rc = SMF_EHIP;
            goto fail;
        }
    } else {
        if (smf::launch_factors(g, plan->C, z_dev, 0, ubasis, plan->f64, plan->f32, st) != hipSuccess) {
            rc = SMF_EHIP;
            goto fail;
        }
        if (plan->asym && smf::launch_factors(g, plan->C, z_dev, 1, ubasis, plan->f64 + nrec1,
                                              plan->f32 ? plan->f32 + nrec1 : nullptr, st) != hipSuccess) {
            rc = SMF_EHIP;
            goto fail;
        }
    }
    if ((rc = bufs.alloc(&plan->tw64, (size_t)2 * n_phi))) goto fail;
    if ((rc = bufs.alloc(&plan->tw32, (size_t)2 * n_phi))) goto fail;
    if (smf::launch_twiddles(n_phi, plan->tw64, plan->tw32, st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
    plan->scan_fine = scan ? smf::scan_fine_blocks(g) : 1;
    if (plan->scan_fine > 1) {
        const size_t nphi1 = (size_t)plan->scan_fine * g.m_rows * g.order * g.order;
        const size_t nphi = nphi1 * (plan->asym ? 2 : 1);
        plan->phi_south_off = plan->asym ? nphi1 : 0;
        if ((rc = bufs.alloc(&plan->phi64, nphi))) goto fail;
        if (hipMemsetAsync(plan->phi64, 0, nphi * sizeof(double), st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
        if (flags == SMF_FP32) {
            if ((rc = bufs.alloc(&plan->phi32, nphi))) goto fail;
            if (hipMemsetAsync(plan->phi32, 0, nphi * sizeof(float), st) != hipSuccess) { rc = SMF_EHIP; goto fail; }
        }
        if (smf::launch_phi(g, plan->f64, plan->scan_fine, plan->phi64, plan->phi32, st) != hipSuccess ||
            (plan->asym && smf::launch_phi(g, plan->f64 + nrec1, plan->scan_fine, plan->phi64 + nphi1,
                                           plan->phi32 ? plan->phi32 + nphi1 : nullptr, st) != hipSuccess)) {
            rc = SMF_EHIP;
            goto fail;
        }
    }
    if (hipStreamSynchronize(st) != hipSuccess) { rc = SMF_EHIP; goto fail; }

    // scratch used only during setup
    (void)hipFree(bad_dev);
    if (kappa_dev) (void)hipFree(kappa_dev);
    if (cexp_dev) (void)hipFree(cexp_dev);
    if (z_dev) (void)hipFree(z_dev);
    if (hp_dev) (void)hipFree(hp_dev);
    if (hn_dev) (void)hipFree(hn_dev);
    *out = plan;
    log_line(1, "setup: order %d, %d x %d rings x longitudes, ell_max %d (m_top %d), %s%s%s%s%s, %d factor sets x %d mode "
             "rows (%.1f MB of factors), %s walk",
             g.order, n_theta, n_phi, g.ell_max, g.m_top, flags == SMF_FP64 ? "FP64" : "FP32", ubasis ? ", U basis" : "",
             green ? (pair ? ", Green's functions of a conjugate kappa pair" : ", Green's functions") : "", z_host ? ", explicit grid" : "", plan->asym ? ", own southern sets" : "",
             g.n_sets, g.m_rows,
             (double)nrec1 * (plan->asym ? 2 : 1) * (8.0 + (flags == SMF_FP32 ? 4.0 : 0.0)) / 1e6,
             plan->scan_fine > 1 ? "scan-capable" : "plain");
    return SMF_OK;

fail:
    (void)hipStreamSynchronize(st);
    bufs.free_all();
    free(c_pair);
    free(plan->zgrid);
    free(plan);
    log_line(1, "smf_setup: failed: %s", smf_error_string(rc));
    return rc;
}

}  // namespace

extern "C" {

int smf_setup(const smf_spectrum* spec, int n_theta, int n_phi, int flags, void* hip_stream,
              smf_plan** out)
{
    return setup_impl(spec, n_theta, nullptr, n_phi, flags, (hipStream_t)hip_stream, true, out);
}

int smf_setup_grid(const smf_spectrum* spec, int n_theta, const double* z_host, int n_phi, int flags,
                   void* hip_stream, smf_plan** out)
{
    if (!z_host) return SMF_EINVAL;
    return setup_impl(spec, n_theta, z_host, n_phi, flags, (hipStream_t)hip_stream, true, out);
}

// Layout of a call's chains: ring blocks of the affine scan (1: plain recursion) and
// chains per lane (1: one part, 2: both parts of a mode, FP32 only).  The result depends
// on the blocks only.  With w = count * 2 * ceil(m_rows / 32) one-part waves, the
// automatic choice (measured on MI355X) is: FP32 plain with two parts per lane above 1024
// waves (from 1025 to 2047 one-part waves would leave some of the 1024 SIMDs two waves and
// others one: 4096 x 8192 x 6 fields 0.560 -> 0.433 ms, 8192 x 16384 x 3 1.03 -> 0.85 ms),
// plain with one part at exactly 1024 (one wave per SIMD: 0.340 against 0.420 ms at
// 4096 x 8192 x 4), a two-part scan of 8 blocks from 512, else a one-part scan of 16 blocks; FP64 plain from 1024 waves, else a scan of the fewest
// blocks giving >= 4096 waves.  Orders 3 and 4 as FP64 (one-part scans of at most 8
// blocks), with two parts per lane in FP32 from SMF_GEN_TWO_W waves.  Scans keep
// >= kScanAutoMinSets ring steps per block.
// Orders 3 and 4: the plain recursion runs two parts per lane from this many one-part waves
// (measured: order 4 at 2048 x 4096 x 32 fields 1.88 -> 1.59 ms; at 4096 x 8192 x 8 fields,
// 2048 waves, one part per lane stays faster).
#ifndef SMF_GEN_TWO_W
#define SMF_GEN_TWO_W 4096
#endif
struct CallShape {
    int blocks, nch;
};

static CallShape call_shape(const smf_plan* plan, int count)
{
    const bool fp64 = plan->flags == SMF_FP64;
    const bool high = plan->g.order > 2;   // orders 3, 4: one part per lane, scans of <= 8 blocks
    const int cap = std::min(plan->scan_fine, smf::scan_max_blocks(fp64, plan->g.order));
    const long w = (long)count * 2 * ((plan->g.m_rows + 31) / 32);
    const int walk = plan->g.n_sets - (plan->g.even ? 2 : 1);
    const int plain_nch = (!fp64 && (high ? w >= SMF_GEN_TWO_W : w > 1024)) ? 2 : 1;
    const int scan_nch = (!fp64 && !high && w >= 512) ? 2 : 1;
    if (cap < 2 || plan->scan_req == 1) return {1, plain_nch};
    if (plan->scan_req >= 2) return {std::min(plan->scan_req, cap), scan_nch};
    if (w >= 1024) return {1, plain_nch};
    int b;
    if (fp64 || high) {
        b = 2;
        while (b < cap && w * b < 4096) b *= 2;
    } else {
        b = w >= 512 ? 8 : 16;
    }
    if (b > cap) b = cap;
    while (b >= 2 && walk / b < smf::kScanAutoMinSets) b /= 2;
    return b >= 2 ? CallShape{b, scan_nch} : CallShape{1, plain_nch};
}

// Largest field count of one call: the FFT indexes its rows (count * n_theta) with ints.
static bool count_fits(const smf_plan* plan, int count)
{
    return (long long)count * plan->g.n_theta <= 0x7FFFFFFFLL;
}

// fft: transform the modes into the field; ln (with fft): the lognormal map on the store.
static int sample_common(const smf_plan* plan, uint64_t seed, int count, void* out_dev,
                         void* hip_stream, bool fft, const smf::LognormalMap* ln = nullptr)
{
    if (!plan || plan->batch || count < 0 || !count_fits(plan, count)) return SMF_EINVAL;
    if (count == 0) return SMF_OK;
    if (!out_dev) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    hipStream_t st = (hipStream_t)hip_stream;
    const int fp64 = plan->flags == SMF_FP64;
    const void* fac = fp64 ? (const void*)plan->f64 : (const void*)plan->f32;
    const CallShape cs = call_shape(plan, count);
    log_line(2, "sample: %d field%s, %s, %d chain%s per lane%s", count, count == 1 ? "" : "s",
             cs.blocks > 1 ? "affine scan over ring blocks" : "plain walk", cs.nch, cs.nch == 1 ? "" : "s",
             fft ? ", then the transform" : "");
    if (cs.blocks > 1) {
        const void* phi = fp64 ? (const void*)plan->phi64 : (const void*)plan->phi32;
        if (smf::launch_scan(plan->g, fp64, fac, plan->south_off, phi, plan->phi_south_off, plan->scan_fine, cs.blocks,
                             seed, count, out_dev, cs.nch, st) != hipSuccess)
            return SMF_EHIP;
    } else if (smf::launch_recursion(plan->g, fp64, fac, plan->south_off, seed, count, out_dev, cs.nch, st) !=
               hipSuccess) {
        return SMF_EHIP;
    }
    if (fft) {
        const void* tw = fp64 ? (const void*)plan->tw64 : (const void*)plan->tw32;
        if (smf::launch_c2r(plan->g, fp64, tw, count, out_dev, ln, st) != hipSuccess) return SMF_EHIP;
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

int smf_sample_lognormal(const smf_plan* plan, uint64_t seed, int count, double mu, double sigma, void* out_dev,
                         void* hip_stream)
{
    if (!std::isfinite(mu) || !std::isfinite(sigma)) return SMF_EINVAL;
    const smf::LognormalMap ln = {mu, sigma};
    return sample_common(plan, seed, count, out_dev, hip_stream, true, &ln);
}

int smf_transform(const smf_plan* plan, int count, void* data_dev, void* hip_stream)
{
    if (!plan || plan->batch || count < 0 || !count_fits(plan, count)) return SMF_EINVAL;
    if (count == 0) return SMF_OK;
    if (!data_dev) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    const int fp64 = plan->flags == SMF_FP64;
    const void* tw = fp64 ? (const void*)plan->tw64 : (const void*)plan->tw32;
    return smf::launch_c2r(plan->g, fp64, tw, count, data_dev, nullptr, (hipStream_t)hip_stream) == hipSuccess
               ? SMF_OK
               : SMF_EHIP;
}

int smf_set_ring_blocks(smf_plan* plan, int blocks)
{
    if (!plan || plan->batch || blocks < 0 || blocks > smf::kScanMaxBlocks) return SMF_EINVAL;
    if (blocks > 1 && (blocks & (blocks - 1))) return SMF_EINVAL;
    plan->scan_req = blocks;
    return SMF_OK;
}

int smf_get_ring_blocks(const smf_plan* plan, int count, int* blocks)
{
    if (!plan || plan->batch || !blocks || count < 0) return SMF_EINVAL;
    *blocks = call_shape(plan, count).blocks;
    return SMF_OK;
}

int smf_plan_dims(const smf_plan* plan, int* dims)
{
    if (!plan || plan->batch || !dims) return SMF_EINVAL;
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

// One factor record to or from full M x M matrices (A row-major, B lower triangular);
// `mirror` conjugates both by D = diag((-1)^p), the storage of the southern walk's own sets.
static void unpack_record(int M, const double* r, bool mirror, double* A, double* B)
{
    if (M == 1) {
        A[0] = r[0];
        B[0] = r[1];
    } else if (M == 2) {
        A[0] = r[0]; A[1] = r[1]; A[2] = r[2]; A[3] = r[3];
        B[0] = r[4]; B[1] = 0.0; B[2] = r[5]; B[3] = r[6];
    } else {
        for (int i = 0; i < M * M; ++i) A[i] = r[i];
        int k = M * M;
        for (int p = 0; p < M; ++p)
            for (int q = 0; q < M; ++q) B[p * M + q] = q <= p ? r[k++] : 0.0;
    }
    if (mirror)
        for (int p = 0; p < M; ++p)
            for (int q = 0; q < M; ++q)
                if ((p + q) & 1) { A[p * M + q] = -A[p * M + q]; B[p * M + q] = -B[p * M + q]; }
}

static void pack_record(int M, const double* A, const double* B, bool mirror, double* r)
{
    const double sg[2] = {1.0, mirror ? -1.0 : 1.0};
    if (M == 1) {
        r[0] = A[0];
        r[1] = B[0];
    } else if (M == 2) {
        r[0] = A[0]; r[1] = sg[1] * A[1]; r[2] = sg[1] * A[2]; r[3] = A[3];
        r[4] = B[0]; r[5] = sg[1] * B[2]; r[6] = B[3];
    } else {
        int k = M * M;
        for (int p = 0; p < M; ++p)
            for (int q = 0; q < M; ++q) r[p * M + q] = sg[(p + q) & 1] * A[p * M + q];
        for (int p = 0; p < M; ++p)
            for (int q = 0; q <= p; ++q) r[k++] = sg[(p + q) & 1] * B[p * M + q];
    }
}

// Factor tables a plan holds: the northern one, and for a grid with no symmetry the
// southern walk's own one (its sets from j0 on stored mirrored).
static int n_tables(const smf_plan* plan) { return plan->asym ? 2 : 1; }

int smf_get_factors(const smf_plan* plan, double* A_host, double* B_host)
{
    if (!plan || plan->batch || !A_host || !B_host) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    const Geometry& g = plan->g;
    const int M = g.order, E = smf::factor_stride(M), j0 = g.even ? 2 : 1;
    const size_t nrec = (size_t)g.n_sets * g.m_rows * E * n_tables(plan);
    std::vector<double> tmp(nrec);
    if (hipMemcpy(tmp.data(), plan->f64, nrec * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return SMF_EHIP;
    for (int t = 0; t < n_tables(plan); ++t)
        for (int j = 0; j < g.n_sets; ++j)
            for (int m = 0; m <= g.m_top; ++m) {
                const size_t js = (size_t)t * g.n_sets + j;
                const double* r = tmp.data() + (js * g.m_rows + m) * E;
                const size_t o = (js * (g.m_top + 1) + m) * M * M;
                unpack_record(M, r, t == 1 && j >= j0, A_host + o, B_host + o);
            }
    return SMF_OK;
}

int smf_set_factors(smf_plan* plan, const double* A_host, const double* B_host, void* hip_stream)
{
    if (!plan || plan->batch || !A_host || !B_host) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    const Geometry& g = plan->g;
    const int M = g.order, E = smf::factor_stride(M), j0 = g.even ? 2 : 1;
    const size_t per = (size_t)(g.m_top + 1) * M * M;
    const size_t nsets = (size_t)g.n_sets * n_tables(plan);
    for (size_t i = 0; i < nsets * per; ++i)
        if (!std::isfinite(A_host[i]) || !std::isfinite(B_host[i])) return SMF_EINVAL;
    const size_t nrec1 = (size_t)g.n_sets * g.m_rows * E, nrec = nrec1 * n_tables(plan);
    std::vector<double> r64(nrec, 0.0);
    std::vector<float> r32;
    for (int t = 0; t < n_tables(plan); ++t)
        for (int j = 0; j < g.n_sets; ++j)
            for (int m = 0; m <= g.m_top; ++m) {
                const size_t js = (size_t)t * g.n_sets + j;
                const size_t o = (js * (g.m_top + 1) + m) * M * M;
                pack_record(M, A_host + o, B_host + o, t == 1 && j >= j0, r64.data() + (js * g.m_rows + m) * E);
            }
    hipStream_t st = (hipStream_t)hip_stream;
    if (hipMemcpyAsync(plan->f64, r64.data(), nrec * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
        return SMF_EHIP;
    if (plan->f32) {
        r32.resize(nrec);
        for (size_t i = 0; i < nrec; ++i) r32[i] = (float)r64[i];
        if (hipMemcpyAsync(plan->f32, r32.data(), nrec * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
            return SMF_EHIP;
    }
    if (plan->scan_fine > 1) {
        if (smf::launch_phi(g, plan->f64, plan->scan_fine, plan->phi64, plan->phi32, st) != hipSuccess)
            return SMF_EHIP;
        if (plan->asym &&
            smf::launch_phi(g, plan->f64 + nrec1, plan->scan_fine, plan->phi64 + plan->phi_south_off,
                            plan->phi32 ? plan->phi32 + plan->phi_south_off : nullptr, st) != hipSuccess)
            return SMF_EHIP;
    }
    return hipStreamSynchronize(st) == hipSuccess ? SMF_OK : SMF_EHIP;
}

int smf_plan_grid(const smf_plan* plan, double* z_host, int* symmetric)
{
    if (!plan || plan->batch) return SMF_EINVAL;
    if (symmetric) *symmetric = plan->asym ? 0 : 1;
    if (z_host) {
        if (plan->zgrid) {
            memcpy(z_host, plan->zgrid, sizeof(double) * plan->g.n_theta);
        } else {
            const int n = plan->g.n_theta;
            for (int i = 0; i < n; ++i) z_host[i] = std::sin(M_PI * (double)(n - 2 * i - 1) / (2.0 * n));
        }
    }
    return SMF_OK;
}

// Rings with their own pixel counts: the plan of smf_setup_grid on the smallest power of
// two n_phi >= 2 (ell_max + 1), so that the chains produce every mode, plus the ring table.
int smf_setup_rings(const smf_spectrum* spec, int n_theta, const double* z_host, const int* n_phi_ring,
                    const double* phi0, int flags, void* hip_stream, smf_plan** out)
{
    const char* W = "smf_setup_rings";
    if (!spec || !out || !n_phi_ring || !phi0 || n_theta < 2 || n_theta > (1 << 16))
        return reject(W, "NULL argument, or n_theta outside [2, 65536]");
    *out = nullptr;
    if (spec->ell_max < 0 || spec->ell_max > smf::kRingMaxEll) return reject(W, "ell_max must be in [0, 8191]");
    const bool fp64 = (flags & ~(SMF_UBASIS | SMF_NO_MIRROR | SMF_GREEN | SMF_KAPPA_PAIR)) == SMF_FP64;
    const int n_cap = fp64 ? smf::kRingMaxPixels64 : smf::kRingMaxPixels32;
    int n_max = 0;
    std::vector<int64_t> off((size_t)n_theta + 1, 0);
    for (int i = 0; i < n_theta; ++i) {
        const int n = n_phi_ring[i];
        if (n < 2 || n > n_cap || (n & 1) || !std::isfinite(phi0[i]))
            return reject(W, "each ring needs an even pixel count in [2, 8192] (FP32) or [2, 4096] (FP64) and a finite phi0");
        n_max = std::max(n_max, n);
        off[i + 1] = off[i] + n;
    }
    int n_phi = 4;
    while (n_phi < 2 * (spec->ell_max + 1)) n_phi *= 2;
    hipStream_t st = (hipStream_t)hip_stream;
    // chain rows: the 64-mode tiles that hold m <= ell_max (the rows above only held zeros)
    const int rows = ((spec->ell_max + 1 + 63) / 64) * 64;
    int rc = setup_impl(spec, n_theta, z_host, n_phi, flags, st, true, out, rows);
    if (rc != SMF_OK) return rc;
    smf_plan* plan = *out;
    // Transform class of each ring (h = n / 2):
    //  - h a power of two L with 2^kRingFftMinLog2 <= L <= 2^kRingFftMaxLog2: radix-8 passes;
    //  - Bluestein's convolution of length L >= 2h - 1 in the same range, where its estimated
    //    work (SMF_RING_BLUE_COST L log2 L) is below that of the odd-prime passes, or where the
    //    largest odd prime would take the chirp-z pass;
    //  - else rings whose largest odd prime P is at least SMF_RING_CHIRP_MIN and whose chirp-z
    //    length fits take the chirp-z pass in a launch of their own, the rest direct passes.
    std::vector<int> direct, chirp;
    std::vector<int> blue[smf::kRingFftClasses], pow2[smf::kRingFftClasses];
    smf::RingSplit rs = {0, 0, 0, 0, 0};
    const int l_cap = fp64 ? smf::kRingChirpMaxL64 : smf::kRingChirpMaxL32;
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, plan->device) != hipSuccess) {
        smf_destroy(plan);
        *out = nullptr;
        return SMF_EHIP;
    }
    auto fft_class_fits = [&](int log2l) {
        return log2l >= smf::kRingFftMinLog2 && log2l <= smf::kRingFftMaxLog2 &&
               smf::ring_fft_lds_bytes(log2l, plan->g.m_top, fp64) <= (size_t)lds_max;
    };
    // lane-operations of the odd-prime passes of the general kernel: 4 h p for the largest
    // prime (paired inputs and outputs), 10 h p for each further one
    auto odd_pass_work = [](int h) {
        int r = h;
        while ((r & 1) == 0) r >>= 1;
        std::vector<int> ps;
        for (int p = 3; r > 1;) {
            if (p * p > r) p = r;
            if (r % p) {
                p += 2;
                continue;
            }
            ps.push_back(p);
            r /= p;
        }
        double w = 0;
        for (size_t k = 0; k < ps.size(); ++k) w += (k + 1 == ps.size() ? 4.0 : 10.0) * h * ps[k];
        return w;
    };
    for (int i = 0; i < n_theta; ++i) {
        const int h = n_phi_ring[i] / 2;
        int lh = 0;
        while ((1 << lh) < h) ++lh;
        if ((1 << lh) == h && fft_class_fits(lh)) {
            pow2[lh - smf::kRingFftMinLog2].push_back(i);
            continue;
        }
        const int P = smf::ring_largest_odd_prime(h);
        int L = 1;
        while (L < 2 * P - 1) L <<= 1;
        const bool chirped = P >= SMF_RING_CHIRP_MIN && L <= l_cap;
        int lb = 0;
        while ((1 << lb) < 2 * h - 1) ++lb;
        if ((1 << lh) != h && lb >= SMF_RING_BLUE_MIN_LOG2 && fft_class_fits(lb) &&
            (chirped || SMF_RING_BLUE_COST * (double)(1 << lb) * lb < odd_pass_work(h))) {
            blue[lb - smf::kRingFftMinLog2].push_back(i);
            continue;
        }
        if (chirped) {
            chirp.push_back(i);
            rs.n_max_chirp = std::max(rs.n_max_chirp, n_phi_ring[i]);
            rs.l_max = std::max(rs.l_max, L);
        } else {
            direct.push_back(i);
            rs.n_max_direct = std::max(rs.n_max_direct, n_phi_ring[i]);
        }
    }
    // each launch takes its most expensive rings first (estimated work of the odd-prime passes:
    // h P / 2 for a direct pass, h L log2 L / P for the chirp-z one; then h log2 h)
    auto cost = [&](int i, bool chirped) {
        const double h = n_phi_ring[i] / 2;
        const int P = smf::ring_largest_odd_prime(n_phi_ring[i] / 2);
        double L = 1;
        while (L < 2 * P - 1) L *= 2;
        return (chirped ? h * L * std::log2(L) / P : h * P / 2.0) + h * std::log2(h + 1.0);
    };
    std::stable_sort(direct.begin(), direct.end(), [&](int x, int y) { return cost(x, false) > cost(y, false); });
    std::stable_sort(chirp.begin(), chirp.end(), [&](int x, int y) { return cost(x, true) > cost(y, true); });
    rs.n_direct = (int)direct.size();
    rs.n_chirp = (int)chirp.size();
    // the launch order of the ring list, and the distinct Bluestein half-lengths of each L
    std::vector<int> order;
    std::vector<int> spec_h;          // by class, largest L first
    std::vector<int64_t> spec_at;     // offset of each one's transform
    int spec_n[smf::kRingFftClasses] = {0};
    std::vector<int64_t> spec_off((size_t)n_theta, 0);
    int64_t spec_total = 0;
    for (int c = smf::kRingFftClasses - 1; c >= 0; --c) {
        rs.n_blue[c] = (int)blue[c].size();
        // rings of the same length next to each other, longest first
        std::stable_sort(blue[c].begin(), blue[c].end(), [&](int x, int y) { return n_phi_ring[x] > n_phi_ring[y]; });
        for (int i : blue[c]) {
            const int h = n_phi_ring[i] / 2;
            if (spec_n[c] == 0 || spec_h.back() != h) {
                spec_h.push_back(h);
                spec_at.push_back(spec_total);
                spec_total += (int64_t)2 << (smf::kRingFftMinLog2 + c);   // S, c and D
                ++spec_n[c];
            }
            spec_off[i] = spec_at.back();
            order.push_back(i);
        }
    }
    for (int c = smf::kRingFftClasses - 1; c >= 0; --c) {
        rs.n_pow2[c] = (int)pow2[c].size();
        order.insert(order.end(), pow2[c].begin(), pow2[c].end());
    }
    order.insert(order.end(), direct.begin(), direct.end());
    order.insert(order.end(), chirp.begin(), chirp.end());
    plan->ring_split = rs;
    if (smf::ring_lds_bytes(rs.n_max_direct, plan->g.m_top, fp64) > (size_t)lds_max ||
        smf::ring_lds_bytes(rs.n_max_chirp, plan->g.m_top, fp64, rs.l_max) > (size_t)lds_max)
        rc = SMF_EINVAL;
    plan->n_ring_max = n_max;
    plan->ring_off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_theta + 1));
    if (rc == SMF_OK && !plan->ring_off) rc = SMF_ENOMEM;
    if (rc == SMF_OK) {
        memcpy(plan->ring_off, off.data(), sizeof(int64_t) * ((size_t)n_theta + 1));
        if (dev_malloc((void**)&plan->n_ring_dev, sizeof(int) * n_theta) != hipSuccess ||
            dev_malloc((void**)&plan->phi0_dev, sizeof(double) * n_theta) != hipSuccess ||
            dev_malloc((void**)&plan->ring_off_dev, sizeof(int64_t) * ((size_t)n_theta + 1)) != hipSuccess ||
            dev_malloc((void**)&plan->ring_list_dev, sizeof(int) * n_theta) != hipSuccess)
            rc = SMF_ENOMEM;
    }
    if (rc == SMF_OK &&
        (hipMemcpyAsync(plan->n_ring_dev, n_phi_ring, sizeof(int) * n_theta, hipMemcpyHostToDevice, st) !=
             hipSuccess ||
         hipMemcpyAsync(plan->phi0_dev, phi0, sizeof(double) * n_theta, hipMemcpyHostToDevice, st) != hipSuccess ||
         hipMemcpyAsync(plan->ring_off_dev, plan->ring_off, sizeof(int64_t) * ((size_t)n_theta + 1),
                        hipMemcpyHostToDevice, st) != hipSuccess ||
         hipMemcpyAsync(plan->ring_list_dev, order.data(), sizeof(int) * n_theta, hipMemcpyHostToDevice, st) !=
             hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess))
        rc = SMF_EHIP;
    // the power-of-two transform tables and the Bluestein kernels' transforms
    if (rc == SMF_OK && smf::ring_fft_count(rs) > 0) {
        const size_t cx = fp64 ? 16 : 8;
        int* hs_dev = nullptr;
        int64_t* at_dev = nullptr;
        if (dev_malloc((void**)&plan->ring_tw64, 16 * (size_t)smf::ring_tw_entries()) != hipSuccess ||
            (!fp64 && dev_malloc((void**)&plan->ring_tw32, 8 * (size_t)smf::ring_tw_entries()) != hipSuccess) ||
            dev_malloc((void**)&plan->ring_spec_off_dev, sizeof(int64_t) * n_theta) != hipSuccess ||
            (spec_total > 0 && (dev_malloc(&plan->ring_spec_dev, cx * (size_t)spec_total) != hipSuccess ||
                                dev_malloc((void**)&hs_dev, sizeof(int) * spec_h.size()) != hipSuccess ||
                                dev_malloc((void**)&at_dev, sizeof(int64_t) * spec_at.size()) != hipSuccess)))
            rc = SMF_ENOMEM;
        if (rc == SMF_OK &&
            (smf::launch_ring_tw(plan->ring_tw64, plan->ring_tw32, st) != hipSuccess ||
             hipMemcpyAsync(plan->ring_spec_off_dev, spec_off.data(), sizeof(int64_t) * n_theta,
                            hipMemcpyHostToDevice, st) != hipSuccess))
            rc = SMF_EHIP;
        if (rc == SMF_OK && spec_total > 0) {
            if (hipMemcpyAsync(hs_dev, spec_h.data(), sizeof(int) * spec_h.size(), hipMemcpyHostToDevice, st) !=
                    hipSuccess ||
                hipMemcpyAsync(at_dev, spec_at.data(), sizeof(int64_t) * spec_at.size(), hipMemcpyHostToDevice,
                               st) != hipSuccess)
                rc = SMF_EHIP;
            int first = 0;
            for (int c = smf::kRingFftClasses - 1; c >= 0 && rc == SMF_OK; --c) {
                if (smf::launch_ring_spectra(smf::kRingFftMinLog2 + c, spec_n[c], hs_dev + first, at_dev + first,
                                             plan->ring_tw64, fp64, plan->ring_spec_dev, st) != hipSuccess)
                    rc = SMF_EHIP;
                first += spec_n[c];
            }
        }
        if (hipStreamSynchronize(st) != hipSuccess && rc == SMF_OK) rc = SMF_EHIP;
        if (hs_dev) (void)hipFree(hs_dev);
        if (at_dev) (void)hipFree(at_dev);
    }
    // streams (default priority) and events over which a synthesis of several launches spreads
    int units = rs.n_direct + rs.n_chirp > 0 ? 1 : 0;
    for (int c = 0; c < smf::kRingFftClasses; ++c) units += (rs.n_blue[c] > 0) + (rs.n_pow2[c] > 0);
    if (rc == SMF_OK && units > 1) {
        if (hipEventCreateWithFlags(&plan->ring_fork, hipEventDisableTiming) != hipSuccess) rc = SMF_EHIP;
        for (int j = 0; j < smf::kRingAuxStreams && rc == SMF_OK; ++j)
            if (hipStreamCreateWithFlags(&plan->ring_aux[j], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&plan->ring_join[j], hipEventDisableTiming) != hipSuccess)
                rc = SMF_EHIP;
    }
    if (rc != SMF_OK) {
        smf_destroy(plan);
        *out = nullptr;
        log_line(1, "smf_setup_rings: failed: %s", smf_error_string(rc));
        return rc;
    }
    if (log_level() >= 1) {
        char cls[256] = "";
        size_t used = 0;
        for (int c = smf::kRingFftClasses - 1; c >= 0; --c) {
            if (rs.n_blue[c])
                used += snprintf(cls + used, sizeof(cls) - used, " Bluestein L=%d: %d;", 1 << (smf::kRingFftMinLog2 + c),
                                 rs.n_blue[c]);
            if (rs.n_pow2[c] && used < sizeof(cls))
                used += snprintf(cls + used, sizeof(cls) - used, " power of two L=%d: %d;",
                                 1 << (smf::kRingFftMinLog2 + c), rs.n_pow2[c]);
            if (used >= sizeof(cls)) break;
        }
        char streams[64] = "one stream";
        if (plan->ring_aux[0])
            snprintf(streams, sizeof(streams), "launches spread over %d more streams", smf::kRingAuxStreams);
        log_line(1, "setup_rings: %d rings, %lld pixels per field, largest %d, chains at n_phi %d; rings by transform "
                 "class:%s general %d (chirp-z %d); %lld Bluestein half-lengths (tables %.1f MB); %s",
                 n_theta, (long long)off[n_theta], n_max, n_phi, cls, rs.n_direct + rs.n_chirp, rs.n_chirp,
                 (long long)spec_h.size(), (double)spec_total * (fp64 ? 16 : 8) / 1e6, streams);
    }
    return rc;
}

int smf_ring_layout(const smf_plan* plan, int64_t* offsets)
{
    if (!plan || plan->batch || !plan->n_ring_dev || !offsets) return SMF_EINVAL;
    memcpy(offsets, plan->ring_off, sizeof(int64_t) * ((size_t)plan->g.n_theta + 1));
    return SMF_OK;
}

static int synthesize_rings(const smf_plan* plan, int count, const void* g_dev, void* out_dev, void* hip_stream,
                            const smf::LognormalMap* ln)
{
    if (!plan || plan->batch || !plan->n_ring_dev || count < 0 || count > smf::kRingMaxCount) return SMF_EINVAL;
    if (count == 0) return SMF_OK;
    if (!g_dev || !out_dev) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    const Geometry& g = plan->g;
    const smf::RingSplit& rs = plan->ring_split;
    const bool fp64 = plan->flags == SMF_FP64;
    const hipStream_t st = (hipStream_t)hip_stream;
    const void* tw = fp64 ? (const void*)plan->ring_tw64 : (const void*)plan->ring_tw32;
    // the launches: each class of rings_fft.hip (list order), then the general kernel's pair
    struct Unit {
        bool blue;
        int log2l, rings, first;
    };
    std::vector<Unit> fft;
    int first = 0;
    for (int c = smf::kRingFftClasses - 1; c >= 0; --c) {
        if (rs.n_blue[c]) fft.push_back({true, smf::kRingFftMinLog2 + c, rs.n_blue[c], first});
        first += rs.n_blue[c];
    }
    for (int c = smf::kRingFftClasses - 1; c >= 0; --c) {
        if (rs.n_pow2[c]) fft.push_back({false, smf::kRingFftMinLog2 + c, rs.n_pow2[c], first});
        first += rs.n_pow2[c];
    }
    const bool general = rs.n_direct + rs.n_chirp > 0;
    const bool fork = SMF_RING_FORK && plan->ring_aux[0] != nullptr && fft.size() + (general ? 1 : 0) > 1;
    // with several launches the general kernel's pair stays on the caller's stream and the
    // classes go to the plan's other streams, forked from and joined back to it by events: the
    // largest first, each to the stream with the least work so far (work: rings x L log2 L per
    // transform, two for the Bluestein form), so that a memory-bound class (the power-of-two
    // rings) and the VALU-bound Bluestein classes run side by side instead of one after the
    // other; the lock keeps one call's fork, launches and join together
    static std::mutex fork_mu;
    std::unique_lock<std::mutex> lock(fork_mu, std::defer_lock);
    if (fork) {
        lock.lock();
        if (hipEventRecord(plan->ring_fork, st) != hipSuccess) return SMF_EHIP;
        for (int j = 0; j < smf::kRingAuxStreams; ++j)
            if (hipStreamWaitEvent(plan->ring_aux[j], plan->ring_fork, 0) != hipSuccess) return SMF_EHIP;
    }
    log_line(2, "synthesize_rings: %d field%s, %d transform-class launch%s%s, general kernel %s", count,
             count == 1 ? "" : "s", (int)fft.size(), fft.size() == 1 ? "" : "es", fork ? " on the plan's streams" : "",
             general ? "on the caller's stream" : "not needed");
    auto work = [](const Unit& x) { return (x.blue ? 2.0 : 1.0) * x.rings * (double)x.log2l * (double)(1 << x.log2l); };
    std::stable_sort(fft.begin(), fft.end(), [&](const Unit& x, const Unit& y) { return work(x) > work(y); });
    double load[smf::kRingAuxStreams] = {0.0};
    int rc = SMF_OK;
    for (size_t u = 0; u < fft.size() && rc == SMF_OK; ++u) {
        int j = 0;
        for (int k = 1; k < smf::kRingAuxStreams; ++k)
            if (load[k] < load[j]) j = k;
        load[j] += work(fft[u]);
        const hipStream_t su = fork ? plan->ring_aux[j] : st;
        if (smf::launch_ring_fft_class(fft[u].blue, fft[u].log2l, fft[u].rings, g.n_theta, g.m_top, g.n_phi / 2,
                                       plan->ring_off[g.n_theta], fp64, count, g_dev,
                                       plan->ring_list_dev + fft[u].first, plan->n_ring_dev, plan->phi0_dev,
                                       plan->ring_off_dev, tw, plan->ring_spec_dev, plan->ring_spec_off_dev, out_dev,
                                       ln, su) != hipSuccess)
            rc = SMF_EHIP;
    }
    if (rc == SMF_OK && general &&
        smf::launch_ring_c2r(g.n_theta, g.m_top, g.n_phi / 2, plan->ring_off[g.n_theta], rs, fp64, count, g_dev,
                             plan->ring_list_dev + first, plan->n_ring_dev, plan->phi0_dev, plan->ring_off_dev,
                             out_dev, ln, st) != hipSuccess)
        rc = SMF_EHIP;
    if (fork) {
        // the join, also after a failed launch, so that no stream is left forked
        for (int j = 0; j < smf::kRingAuxStreams; ++j)
            if (hipEventRecord(plan->ring_join[j], plan->ring_aux[j]) != hipSuccess ||
                hipStreamWaitEvent(st, plan->ring_join[j], 0) != hipSuccess)
                rc = SMF_EHIP;
    }
    return rc;
}

static int sample_rings(const smf_plan* plan, uint64_t seed, int count, void* g_work, void* out_dev,
                        void* hip_stream, const smf::LognormalMap* ln)
{
    if (!plan || plan->batch || !plan->n_ring_dev || count < 0 || count > smf::kRingMaxCount) return SMF_EINVAL;
    if (count == 0) return SMF_OK;
    if (!g_work || !out_dev || g_work == out_dev) return SMF_EINVAL;
    const int rc = sample_common(plan, seed, count, g_work, hip_stream, false);
    if (rc != SMF_OK) return rc;
    return synthesize_rings(plan, count, g_work, out_dev, hip_stream, ln);
}

// ---- the ring sampling call without a caller-given work buffer ----
// The modes go to a file-scope device array instead.  In host code `ring_scratch` names a
// host-side stand-in, not device memory: its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and only that address is used.
constexpr size_t kRingScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char ring_scratch[kRingScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// The device address of `ring_scratch` on the current device `dev`, looked up on first use.
int ring_scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return SMF_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(ring_scratch)) != hipSuccess || !p) return SMF_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SMF_OK;
}
}  // namespace

int smf_synthesize_rings(const smf_plan* plan, int count, const void* g_dev, void* out_dev, void* hip_stream)
{
    return synthesize_rings(plan, count, g_dev, out_dev, hip_stream, nullptr);
}

int smf_sample_rings(const smf_plan* plan, uint64_t seed, int count, void* g_work, void* out_dev,
                     void* hip_stream)
{
    return sample_rings(plan, seed, count, g_work, out_dev, hip_stream, nullptr);
}

int smf_sample_rings_lognormal(const smf_plan* plan, uint64_t seed, int count, double mu, double sigma,
                               void* g_work, void* out_dev, void* hip_stream)
{
    if (!std::isfinite(mu) || !std::isfinite(sigma)) return SMF_EINVAL;
    const smf::LognormalMap ln = {mu, sigma};
    return sample_rings(plan, seed, count, g_work, out_dev, hip_stream, &ln);
}

int smf_sample_rings_noalloc(const smf_plan* plan, uint64_t seed, int count, void* out_dev, void* hip_stream)
{
    if (!plan || plan->batch || !plan->n_ring_dev || count < 0 || count > smf::kRingMaxCount) return SMF_EINVAL;
    if (count == 0) return SMF_OK;
    if (!out_dev) return SMF_EINVAL;
    const Geometry& g = plan->g;
    const size_t elem = plan->flags == SMF_FP64 ? sizeof(double) : sizeof(float);
    if ((size_t)count * g.n_theta * g.n_phi * elem > kRingScratchBytes) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    void* work = nullptr;
    const int rc = ring_scratch_address(plan->device, &work);
    if (rc != SMF_OK) return rc;
    return sample_rings(plan, seed, count, work, out_dev, hip_stream, nullptr);
}

int smf_destroy(smf_plan* plan)
{
    if (!plan) return SMF_OK;
    DeviceGuard dg(plan->device);
    (void)hipDeviceSynchronize();
    if (plan->batch) {
        smf::BatchState* b = plan->batch;
        for (smf_plan* p : b->sub) smf_destroy(p);
        free_call_slots(b);
        (void)hipFree(b->fields_dev);
        for (int k = 0; k < 3; ++k) (void)hipFree(b->chain_dev[k]);
        (void)hipFree(b->fft_dev);
        delete b;
        free(plan);
        return SMF_OK;
    }
    (void)hipFree(plan->C);
    (void)hipFree(plan->f64);
    if (plan->f32) (void)hipFree(plan->f32);
    (void)hipFree(plan->tw64);
    (void)hipFree(plan->tw32);
    if (plan->phi64) (void)hipFree(plan->phi64);
    if (plan->phi32) (void)hipFree(plan->phi32);
    free(plan->zgrid);
    if (plan->n_ring_dev) (void)hipFree(plan->n_ring_dev);
    if (plan->phi0_dev) (void)hipFree(plan->phi0_dev);
    if (plan->ring_off_dev) (void)hipFree(plan->ring_off_dev);
    if (plan->ring_list_dev) (void)hipFree(plan->ring_list_dev);
    if (plan->ring_tw64) (void)hipFree(plan->ring_tw64);
    if (plan->ring_tw32) (void)hipFree(plan->ring_tw32);
    if (plan->ring_spec_dev) (void)hipFree(plan->ring_spec_dev);
    if (plan->ring_spec_off_dev) (void)hipFree(plan->ring_spec_off_dev);
    for (int j = 0; j < smf::kRingAuxStreams; ++j) {
        if (plan->ring_aux[j]) (void)hipStreamDestroy(plan->ring_aux[j]);
        if (plan->ring_join[j]) (void)hipEventDestroy(plan->ring_join[j]);
    }
    if (plan->ring_fork) (void)hipEventDestroy(plan->ring_fork);
    free(plan->ring_off);
    free(plan);
    return SMF_OK;
}

int smf_set_log_level(int level)
{
    if (level < 0) return SMF_EINVAL;
    const int prev = log_level();
    g_log_level.store(level);
    return prev;
}

int smf_debug_fail_alloc(int n)
{
    if (n < -1) return SMF_EINVAL;
    g_fail_after.store(n);
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


int smf_setup_batch(int n, const smf_spectrum* specs, const int* n_theta, const int* n_phi, int flags,
                    void* hip_stream, smf_plan** out)
{
    if (!out) return SMF_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 65535 || !specs || !n_theta || !n_phi || flags != SMF_FP32) return SMF_EINVAL;
    for (int i = 0; i < n; ++i)
        if (n_phi[i] > 4096 || n_theta[i] > 65535) return SMF_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    smf::BatchState* b = new smf::BatchState();
    b->n = n;
    b->offsets.assign(n + 1, 0);
    int rc = SMF_OK;
    std::vector<smf::BatchField> fields(n);
    std::vector<int> order_idx(n);
    std::vector<uint32_t> fft_items;
    smf_plan* plan = nullptr;
    int dev = 0;
    for (int i = 0; i < n; ++i) {
        smf_plan* p = nullptr;
        rc = setup_impl(&specs[i], n_theta[i], nullptr, n_phi[i], SMF_FP32, st, false, &p);
        if (rc != SMF_OK) goto fail;
        b->sub.push_back(p);
        b->offsets[i + 1] = b->offsets[i] + (int64_t)n_theta[i] * n_phi[i];
        const Geometry& g = p->g;
        smf::BatchField& F = fields[i];
        F.fac = p->f32;
        F.tw = p->tw32;
        F.out_off = b->offsets[i];
        F.n_theta = g.n_theta;
        F.n_phi = g.n_phi;
        F.order = g.order;
        F.m_top = g.m_top;
        F.m_rows = g.m_rows;
        F.n_sets = g.n_sets;
        F.s = g.s;
        F.even = g.even;
        F.log2h = __builtin_ctz((unsigned)g.n_phi) - 1;
        F.seed_off = i;
        b->lds = std::max(b->lds, sizeof(float) * 2 * (size_t)(g.n_phi / 2 + g.n_phi / 32));
    }
    // chain items longest chain first, for each tile shape; FFT items in the same order
    for (int i = 0; i < n; ++i) order_idx[i] = i;
    std::stable_sort(order_idx.begin(), order_idx.end(),
                     [&](int x, int y) { return fields[x].n_theta > fields[y].n_theta; });
    for (int k = 0; k < 3; ++k) {
        const int tiles = 1 << k;
        std::vector<uint32_t> items;
        for (int i : order_idx) {
            const int n_mt = (fields[i].m_rows + 31) / 32;
            for (int t = 0; t < (n_mt + tiles - 1) / tiles; ++t)
                items.push_back(((uint32_t)i << 16) | (uint32_t)t);
        }
        b->n_chain[k] = (int)items.size();
        if (dev_malloc((void**)&b->chain_dev[k], sizeof(uint32_t) * items.size()) != hipSuccess) {
            (void)hipGetLastError();
            rc = SMF_ENOMEM;
            goto fail;
        }
        if (hipMemcpy(b->chain_dev[k], items.data(), sizeof(uint32_t) * items.size(),
                      hipMemcpyHostToDevice) != hipSuccess) {
            rc = SMF_EHIP;
            goto fail;
        }
    }
    for (int i : order_idx)
        for (int r = 0; r < fields[i].n_theta; ++r) fft_items.push_back(((uint32_t)i << 16) | (uint32_t)r);
    b->n_fft = (int)fft_items.size();
    if (dev_malloc((void**)&b->fields_dev, sizeof(smf::BatchField) * n) != hipSuccess ||
        dev_malloc((void**)&b->fft_dev, sizeof(uint32_t) * fft_items.size()) != hipSuccess) {
        (void)hipGetLastError();
        rc = SMF_ENOMEM;
        goto fail;
    }
    if (dev_malloc((void**)&b->call_dev, sizeof(smf::BatchCall) * n * smf::BatchState::kCallSlots) != hipSuccess ||
        host_malloc_pinned((void**)&b->call_host, sizeof(smf::BatchCall) * n * smf::BatchState::kCallSlots) !=
            hipSuccess) {
        (void)hipGetLastError();
        rc = SMF_ENOMEM;
        goto fail;
    }
    for (int k = 0; k < smf::BatchState::kCallSlots; ++k)
        if (hipEventCreateWithFlags(&b->call_ev[k], hipEventDisableTiming) != hipSuccess) {
            rc = SMF_EHIP;
            goto fail;
        }
    if (hipMemcpy(b->fields_dev, fields.data(), sizeof(smf::BatchField) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->fft_dev, fft_items.data(), sizeof(uint32_t) * fft_items.size(),
                  hipMemcpyHostToDevice) != hipSuccess || hipGetDevice(&dev) != hipSuccess) {
        rc = SMF_EHIP;
        goto fail;
    }
    plan = (smf_plan*)calloc(1, sizeof(smf_plan));
    if (!plan) { rc = SMF_ENOMEM; goto fail; }
    plan->flags = SMF_FP32;
    plan->device = dev;
    plan->batch = b;
    *out = plan;
    return SMF_OK;
fail:
    for (smf_plan* p : b->sub) smf_destroy(p);
    free_call_slots(b);
    if (b->fields_dev) (void)hipFree(b->fields_dev);
    for (int k = 0; k < 3; ++k)
        if (b->chain_dev[k]) (void)hipFree(b->chain_dev[k]);
    if (b->fft_dev) (void)hipFree(b->fft_dev);
    delete b;
    return rc;
}

int smf_batch_layout(const smf_plan* plan, int64_t* offsets)
{
    if (!plan || !plan->batch || !offsets) return SMF_EINVAL;
    const smf::BatchState* b = plan->batch;
    for (int i = 0; i <= b->n; ++i) offsets[i] = b->offsets[i];
    return SMF_OK;
}

static int batch_launch(const smf_plan* plan, uint64_t seed, void* out_dev, hipStream_t st, int tiles_idx,
                        const smf::BatchCall* call = nullptr, int persistent = -1)
{
    const smf::BatchState* b = plan->batch;
    smf::BatchArgs a;
    a.fields = b->fields_dev;
    a.call = call;
    a.chain_items = b->chain_dev[tiles_idx];
    a.fft_items = b->fft_dev;
    a.out = (float*)out_dev;
    a.seed = seed;
    a.tiles = 1 << tiles_idx;
    a.n_chain_items = b->n_chain[tiles_idx];
    a.n_fft_items = b->n_fft;
    if (persistent < 0) persistent = b->persistent;
    if (persistent) {
        int grid = 0;
        const hipError_t e = smf::launch_batch_persistent(a, b->lds, st, &grid);
        log_line(2, "sample_batch: %d fields, one cooperative launch of %d workgroups of %d threads (%d chain items, "
                 "%d ring items)", b->n, grid, 128 * a.tiles, a.n_chain_items, a.n_fft_items);
        return e == hipSuccess ? SMF_OK : SMF_EHIP;
    }
    log_line(2, "sample_batch: %d fields, chain launch of %d workgroups of %d threads, ring launch of %d workgroups",
             b->n, a.n_chain_items, 128 * a.tiles, a.n_fft_items);
    return smf::launch_batch(a, b->lds, st) == hipSuccess ? SMF_OK : SMF_EHIP;
}

int smf_batch_set_shape(smf_plan* plan, int tiles, int persistent)
{
    if (!plan || !plan->batch || (tiles != 1 && tiles != 2 && tiles != 4) || (persistent != 0 && persistent != 1))
        return SMF_EINVAL;
    plan->batch->tiles_idx = tiles == 1 ? 0 : tiles == 2 ? 1 : 2;
    plan->batch->persistent = persistent;
    return SMF_OK;
}

int smf_batch_get_shape(const smf_plan* plan, int* tiles, int* persistent)
{
    if (!plan || !plan->batch || !tiles || !persistent) return SMF_EINVAL;
    *tiles = 1 << plan->batch->tiles_idx;
    *persistent = plan->batch->persistent;
    return SMF_OK;
}

int smf_sample_batch_packed(const smf_plan* plan, uint64_t seed, void* out_dev, void* hip_stream)
{
    if (!plan || !plan->batch || !out_dev) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    return batch_launch(plan, seed, out_dev, (hipStream_t)hip_stream, plan->batch->tiles_idx);
}

int smf_sample_batch(const smf_plan* plan, const uint64_t* seeds_host, void* const* outs_dev, void* hip_stream)
{
    if (!plan || !plan->batch || !seeds_host || !outs_dev) return SMF_EINVAL;
    smf::BatchState* b = plan->batch;
    for (int i = 0; i < b->n; ++i)
        if (!outs_dev[i] || ((uintptr_t)outs_dev[i] & 7)) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    hipStream_t st = (hipStream_t)hip_stream;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess) return SMF_EHIP;
    if (cap != hipStreamCaptureStatusNone) return SMF_EINVAL;   // the table upload is per call
    std::lock_guard<std::mutex> lk(b->call_mu);
    const int k = b->call_next;
    if (hipEventSynchronize(b->call_ev[k]) != hipSuccess) return SMF_EHIP;
    smf::BatchCall* host = b->call_host + (size_t)k * b->n;
    smf::BatchCall* dev = b->call_dev + (size_t)k * b->n;
    for (int i = 0; i < b->n; ++i) {
        host[i].key = seeds_host[i];
        host[i].out = (float*)outs_dev[i];
    }
    if (hipMemcpyAsync(dev, host, sizeof(smf::BatchCall) * b->n, hipMemcpyHostToDevice, st) != hipSuccess)
        return SMF_EHIP;
    const int rc = batch_launch(plan, 0, nullptr, st, b->tiles_idx, dev);
    if (rc != SMF_OK) return rc;
    if (hipEventRecord(b->call_ev[k], st) != hipSuccess) return SMF_EHIP;
    b->call_next = (k + 1) % smf::BatchState::kCallSlots;
    return SMF_OK;
}

int smf_autotune_batch(smf_plan* plan, uint64_t seed, void* out_dev, void* hip_stream, int* tiles_out)
{
    if (!plan || !plan->batch || !out_dev) return SMF_EINVAL;
    DeviceGuard dg(plan->device);
    smf::BatchState* b = plan->batch;
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SMF_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return SMF_EHIP; }
    int best_k = b->tiles_idx, best_p = b->persistent;
    float best = 1e30f;
    int rc = SMF_OK;
    // every tile shape in both forms: two launches, or one cooperative launch
    for (int p = 0; p < 2 && rc == SMF_OK; ++p) {
        for (int k = 0; k < 3 && rc == SMF_OK; ++k) {
            float ms_min = 1e30f;
            for (int rep = 0; rep < 3 && rc == SMF_OK; ++rep) {
                float ms = 0.f;
                if (hipEventRecord(e0, st) != hipSuccess) { rc = SMF_EHIP; break; }
                rc = batch_launch(plan, seed, out_dev, st, k, nullptr, p);
                if (rc != SMF_OK) break;
                if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = SMF_EHIP; break; }
                if (rep > 0) ms_min = std::min(ms_min, ms);   // the first run warms up
            }
            log_line(1, "autotune_batch: %d m-tiles per item, %s: %.3f ms", 1 << k,
                     p ? "one cooperative launch" : "two launches", ms_min);
            if (rc == SMF_OK && ms_min < best) {
                best = ms_min;
                best_k = k;
                best_p = p;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SMF_OK) return rc;
    b->tiles_idx = best_k;
    b->persistent = best_p;
    if (tiles_out) *tiles_out = 1 << best_k;
    return SMF_OK;
}

}  // extern "C"
