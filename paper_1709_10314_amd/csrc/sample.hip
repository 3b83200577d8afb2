// Per-plan sampling kernels: the latitude-ring state-space recursion with fused Philox
// normals (Creasey & Lang, Alg. 2; eqs. (state_initial), (state_space)) and the
// complex-to-real inverse FFT along phi of every ring (Alg. 2, last step).
#include "device_path.h"

namespace smf {
namespace {

struct RecArgs {
    int n_theta, n_phi, m_top, m_rows, n_sets, s, even;
    int n_fh;          // 2 * count (field, hemisphere) families
    int n_fg;          // workgroups per m-tile: ceil(n_fh / 4)
    int n_wg;          // n_mtiles * n_fg real workgroups
    int per_xcd;       // launched workgroups / 8
    uint32_t seed_lo, seed_hi;
};

// One lane per chain (field f, hemisphere h, mode m, part Re/Im).  A wave holds 32 modes x
// 2 parts of one (f, h), so f and h are wave-uniform (scalar registers) and so are the
// Philox key and the ring order; a workgroup holds four (f, h) families of the same 32
// modes, which read the same factor records.  Workgroups are numbered so that every
// workgroup of an m-tile lands on the same XCD (workgroup b runs on XCD b mod 8): each XCD
// streams its own slice of the factors through its own L2.
template <typename T, int M>
__global__ __launch_bounds__(256) void recursion_kernel(RecArgs a, const T* __restrict__ fac,
                                                        T* __restrict__ out)
{
    const int b = blockIdx.x;
    const int L = (b & 7) * a.per_xcd + (b >> 3);
    if (L >= a.n_wg) return;
    const int mt = L / a.n_fg;
    const int fg = L - mt * a.n_fg;
    const int fh = __builtin_amdgcn_readfirstlane(fg * 4 + (int)(threadIdx.x >> 6));
    if (fh >= a.n_fh) return;
    const int f = fh >> 1, h = fh & 1;
    const int lane = threadIdx.x & 63;
    const int m = mt * 32 + (lane >> 1), part = lane & 1;
    if (m >= a.m_rows) return;
    T* __restrict__ g = out + (size_t)f * a.n_theta * a.n_phi + 2 * m + part;
    if (m > a.m_top || (m == 0 && part == 1)) {
        zero_chain<T>(a.n_theta, a.s, h, g, (size_t)a.n_phi);
        return;
    }
    const uint64_t key = (((uint64_t)a.seed_hi << 32) | a.seed_lo) + (uint64_t)f;
    run_chain<T, M>(a.n_theta, a.s, a.even, a.n_sets, h, m, part, (uint32_t)key, (uint32_t)(key >> 32),
                    fac + (size_t)m * factor_stride(M), (size_t)a.m_rows * factor_stride(M), g,
                    (size_t)a.n_phi);
}

// Threads per row: H/8 clamped to [64, 256], and 512 for the largest rows (FP32 n_phi =
// 16384, FP64 n_phi >= 8192) so that each thread holds fewer butterflies.
template <typename T, int LOG2H>
struct FftThreads {
    static constexpr int base = (1 << LOG2H) / 8 < 64 ? 64 : ((1 << LOG2H) / 8 > 256 ? 256 : (1 << LOG2H) / 8);
    static constexpr int value = (LOG2H >= (sizeof(T) == 4 ? 13 : 12)) ? 512 : base;
};

// Rows prefetch the next row during the current one's passes while the extra registers
// fit (FP32 up to n_phi = 8192, FP64 up to 2048); larger rows load row by row.
template <typename T, int LOG2H>
struct FftPrefetch {
    static constexpr bool value = sizeof(T) == 4 ? LOG2H <= 12 : LOG2H <= 10;
};

// Register budget in waves per SIMD: 4 (128 VGPRs) for small rows, else 2 (256 VGPRs),
// and 1 for the 512-thread rows.
template <typename T, int LOG2H>
struct FftWaves {
    static constexpr int value = FftThreads<T, LOG2H>::value == 512 ? 1
                                 : (LOG2H < (sizeof(T) == 4 ? 11 : 8) ? 4 : 2);
};

// Each workgroup transforms rows blockIdx.x, blockIdx.x + gridDim.x, ...
template <typename T, int LOG2H>
__global__ __launch_bounds__((FftThreads<T, LOG2H>::value), (FftWaves<T, LOG2H>::value)) void c2r_kernel(
    T* __restrict__ data, const T* __restrict__ twr, int m_top, int rows)
{
    extern __shared__ unsigned char smem_raw[];
    c2r_rows<T, LOG2H, FftThreads<T, LOG2H>::value, FftPrefetch<T, LOG2H>::value>(
        data, twr, m_top, reinterpret_cast<Cx<T>*>(smem_raw), rows, blockIdx.x, gridDim.x);
}

// Workgroups of the row-looping FFT: enough to fill every CU several times over.
constexpr int kFftGrid = 2048;

template <typename T, int LOG2H>
hipError_t launch_c2r_t(const T* tw, int m_top, int rows, T* data, hipStream_t st)
{
    const size_t lds = sizeof(Cx<T>) * lds_slots(1 << LOG2H);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)c2r_kernel<T, LOG2H>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int grid = rows < kFftGrid ? rows : kFftGrid;
    hipLaunchKernelGGL((c2r_kernel<T, LOG2H>), dim3(grid), dim3(FftThreads<T, LOG2H>::value), lds, st, data, tw,
                       m_top, rows);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_c2r(int log2h, const T* tw, int m_top, int rows, T* data, hipStream_t st)
{
    switch (log2h) {
        case 1: return launch_c2r_t<T, 1>(tw, m_top, rows, data, st);
        case 2: return launch_c2r_t<T, 2>(tw, m_top, rows, data, st);
        case 3: return launch_c2r_t<T, 3>(tw, m_top, rows, data, st);
        case 4: return launch_c2r_t<T, 4>(tw, m_top, rows, data, st);
        case 5: return launch_c2r_t<T, 5>(tw, m_top, rows, data, st);
        case 6: return launch_c2r_t<T, 6>(tw, m_top, rows, data, st);
        case 7: return launch_c2r_t<T, 7>(tw, m_top, rows, data, st);
        case 8: return launch_c2r_t<T, 8>(tw, m_top, rows, data, st);
        case 9: return launch_c2r_t<T, 9>(tw, m_top, rows, data, st);
        case 10: return launch_c2r_t<T, 10>(tw, m_top, rows, data, st);
        case 11: return launch_c2r_t<T, 11>(tw, m_top, rows, data, st);
        case 12: return launch_c2r_t<T, 12>(tw, m_top, rows, data, st);
        case 13: return launch_c2r_t<T, 13>(tw, m_top, rows, data, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_recursion(const Geometry& g, int fp64, const void* fac, uint64_t seed, int count,
                            void* out, hipStream_t st)
{
    RecArgs a;
    a.n_theta = g.n_theta;
    a.n_phi = g.n_phi;
    a.m_top = g.m_top;
    a.m_rows = g.m_rows;
    a.n_sets = g.n_sets;
    a.s = g.s;
    a.even = g.even;
    a.n_fh = 2 * count;
    a.n_fg = (a.n_fh + 3) / 4;
    const int n_mt = (g.m_rows + 31) / 32;
    a.n_wg = n_mt * a.n_fg;
    a.per_xcd = (a.n_wg + 7) / 8;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    const dim3 grid((unsigned)(a.per_xcd * 8));
    if (fp64) {
        if (g.order == 1)
            hipLaunchKernelGGL((recursion_kernel<double, 1>), grid, dim3(256), 0, st, a,
                               (const double*)fac, (double*)out);
        else
            hipLaunchKernelGGL((recursion_kernel<double, 2>), grid, dim3(256), 0, st, a,
                               (const double*)fac, (double*)out);
    } else {
        if (g.order == 1)
            hipLaunchKernelGGL((recursion_kernel<float, 1>), grid, dim3(256), 0, st, a,
                               (const float*)fac, (float*)out);
        else
            hipLaunchKernelGGL((recursion_kernel<float, 2>), grid, dim3(256), 0, st, a,
                               (const float*)fac, (float*)out);
    }
    return hipGetLastError();
}

hipError_t launch_c2r(const Geometry& g, int fp64, const void* tw, int count, void* data,
                      hipStream_t st)
{
    const int log2h = __builtin_ctz((unsigned)g.n_phi) - 1;
    const int rows = count * g.n_theta;
    if (rows == 0) return hipSuccess;
    if (fp64) return dispatch_c2r<double>(log2h, (const double*)tw, g.m_top, rows, (double*)data, st);
    return dispatch_c2r<float>(log2h, (const float*)tw, g.m_top, rows, (float*)data, st);
}

}  // namespace smf
