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
    int n_wg;          // m-tiles * n_fg workgroups with work
    int per_xcd;       // launched workgroups / 8
    uint32_t seed_lo, seed_hi;
    size_t south_off;  // elements to the southern walk's own factor table (0: mirrored)
};

// Chains per lane (NCH): 2 runs both parts of a mode in one lane (the two chains share
// every factor record and store one (Re, Im) pair per ring), 1 runs one part per lane
// (twice the waves, half the serial work per wave).  Both give identical results; the
// host picks per call (FP64 always uses 1: two FP64 chains do not fit the register
// budget).
//
// One lane per (field f, hemisphere h, mode m[, part]).  A wave holds 64 modes (two parts
// per lane) or 32 modes x 2 parts of one (f, h), so f and h are wave-uniform (scalar
// registers) and so are the Philox key and the ring order; a workgroup holds four (f, h)
// families of the same modes, which read the same factor records.  Workgroups are
// numbered so that every workgroup of an m-tile lands on the same XCD (workgroup b runs on
// XCD b mod 8): each XCD streams its own slice of the factors through its own L2.
template <typename T, int M, int NCH>
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
    const int m = NCH == 2 ? mt * 64 + lane : mt * 32 + (lane >> 1);
    const int part = NCH == 2 ? 0 : lane & 1;
    if (m >= a.m_rows) return;
    T* __restrict__ g = out + (size_t)f * a.n_theta * a.n_phi + 2 * m + part;
    if (m > a.m_top || (NCH == 1 && m == 0 && part == 1)) {
        zero_chain<T, NCH>(a.n_theta, a.s, h, g, (size_t)a.n_phi);
        return;
    }
    const uint64_t key = (((uint64_t)a.seed_hi << 32) | a.seed_lo) + (uint64_t)f;
    run_chain<T, M, NCH>(a.n_theta, a.s, a.even, a.n_sets, h, m, part, (uint32_t)key, (uint32_t)(key >> 32),
                         fac + (size_t)m * factor_stride(M), (size_t)a.m_rows * factor_stride(M), g,
                         (size_t)a.n_phi, a.south_off);
}

// Markov orders 3 and 4, laid out as the recursion above: NCH = 2 runs both parts of a
// mode in one lane (64 modes per wave), NCH = 1 one part (32 modes x 2 parts per wave);
// four (f, h) families per workgroup, m-tiles kept on one XCD.
template <typename T, int M, int NCH>
__global__ __launch_bounds__(256) void recursion_gen_kernel(RecArgs a, const T* __restrict__ fac,
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
    const int m = NCH == 2 ? mt * 64 + lane : mt * 32 + (lane >> 1);
    const int part = NCH == 2 ? 0 : lane & 1;
    if (m >= a.m_rows) return;
    T* __restrict__ g = out + (size_t)f * a.n_theta * a.n_phi + 2 * m + part;
    if (m > a.m_top || (NCH == 1 && m == 0 && part == 1)) {
        zero_chain<T, NCH>(a.n_theta, a.s, h, g, (size_t)a.n_phi);
        return;
    }
    const uint64_t key = (((uint64_t)a.seed_hi << 32) | a.seed_lo) + (uint64_t)f;
    run_chain_gen<T, M, NCH>(a.n_theta, a.s, a.even, a.n_sets, h, m, part, (uint32_t)key, (uint32_t)(key >> 32),
                        fac + (size_t)m * factor_stride(M), (size_t)a.m_rows * factor_stride(M), g,
                        (size_t)a.n_phi, a.south_off);
}

// ------------------------------------------------------------------ affine scan
// The recursion x_{k+1} = A_k x_k + B_k w_k (eq. (state_space)) is affine in x, so a chain
// cut into ring blocks can run its blocks in parallel: block b started from zero gives c_b
// (its end state driven by its own noise only), and the true start of block b is the fold
// x_b = Phi_{b-1} x_{b-1} + c_{b-1} over the earlier blocks, with Phi the block transitions
// stored at setup.  Block 0 starts from the real start state and stores its rings at once;
// the other blocks walk twice, first without stores for c_b, then from x_b with stores,
// recomputing the same counter-based normals (no workspace, about twice the arithmetic).
//
// A workgroup is one (field, hemisphere, m-tile) with one wave per ring block, laid out as
// the plain recursion's waves (64 modes with both parts per lane in FP32, 32 modes x 2
// parts in FP64): every wave covers the same chains, so its loads and stores are as
// contiguous as the plain recursion's, and the block end states meet in LDS across one
// barrier.
struct ScanArgs {
    int n_theta, n_phi, m_top, m_rows, n_sets, s, even;
    int n_fh, n_wg, per_xcd;
    int fine_per, fine;    // fine blocks per ring block; fine blocks in the plan
    uint32_t seed_lo, seed_hi;
    size_t south_off, phi_south_off;   // the southern walk's own tables (0: mirrored)
};

// Prefetch depth of a scan wave: a workgroup of B >= 8 waves leaves 2048 / B VGPRs per
// lane, so the deeper scans keep shallower pipelines.
template <typename T, int B, int NCH>
struct ScanDepth {
    static constexpr int value = sizeof(T) == 8 ? (B >= 8 ? 2 : 4)
                                 : (B >= 16 ? 2 : (NCH == 2 || B >= 8 ? 4 : 8));
};

template <typename T, int M, int B, int NCH>
__global__ __launch_bounds__(64 * B) void scan_kernel(ScanArgs a, const T* __restrict__ fac,
                                                      const T* __restrict__ phi, T* __restrict__ out)
{
    __shared__ T ends[B * 64 * NCH * M];
    const int bx = blockIdx.x;
    const int L = (bx & 7) * a.per_xcd + (bx >> 3);
    if (L >= a.n_wg) return;
    const int mt = L / a.n_fh;
    const int fh = L - mt * a.n_fh;
    const int f = fh >> 1, h = fh & 1;
    const int blk = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int m = NCH == 2 ? mt * 64 + lane : mt * 32 + (lane >> 1);
    const int part = NCH == 2 ? 0 : lane & 1;
    const bool in_range = m < a.m_rows;
    const bool active = in_range && m <= a.m_top && (NCH == 2 || !(m == 0 && part == 1));
    const size_t row = (size_t)a.n_phi;
    T* __restrict__ g = out + (size_t)f * a.n_theta * a.n_phi + 2 * (in_range ? m : 0) + part;
    if (in_range && !active && blk == 0) zero_chain<T, NCH>(a.n_theta, a.s, h, g, row);

    const uint64_t key = (((uint64_t)a.seed_hi << 32) | a.seed_lo) + (uint64_t)f;
    const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
    const int mm = active ? m : 0;
    const T* __restrict__ fm = fac + (size_t)mm * factor_stride(M);
    const T* __restrict__ fw = fm + (h ? a.south_off : 0);   // the walk's records
    const T* __restrict__ ph = phi + (h ? a.phi_south_off : 0);
    const size_t set_stride = (size_t)a.m_rows * factor_stride(M);
    T sc[NCH];
    chain_scales<T, NCH>(m, (uint32_t)part, sc);
    const uint32_t um = (uint32_t)mm, up = (uint32_t)part;
    const int j0 = a.even ? 2 : 1;
    const long walk = a.n_sets - j0;
    const int jb = j0 + (int)(walk * (blk * a.fine_per) / a.fine);
    const int je = j0 + (int)(walk * ((blk + 1) * a.fine_per) / a.fine);
    const int r_first = h == 0 ? a.s - jb + a.even : a.s + jb;
    const int r_last = h == 0 ? a.s - (je - 1) + a.even : a.s + (je - 1);
    constexpr int P = ScanDepth<T, B, NCH>::value;

    // pass 1: block 0 from the start state (final, stored); the others from zero
    T x0[NCH], x1[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) x0[c] = x1[c] = T(0);
    if (active) {
        if (blk == 0) {
            chain_start<T, M, NCH>(a.s, a.even, h, um, up, k0, k1, sc, fm, set_stride, g, row, true, x0, x1);
            if (h == 0)
                walk_hemisphere<T, M, P, true, NCH, true>(a.s, a.even, r_first, r_last, mm, up, k0, k1, sc, fw,
                                                          set_stride, a.n_sets, g, row, x0, x1);
            else
                walk_hemisphere<T, M, P, false, NCH, true>(a.s, a.even, r_first, r_last, mm, up, k0, k1, sc, fw,
                                                           set_stride, a.n_sets, g, row, x0, x1);
        } else {
            if (h == 0)
                walk_hemisphere<T, M, P, true, NCH, false>(a.s, a.even, r_first, r_last, mm, up, k0, k1, sc, fw,
                                                           set_stride, a.n_sets, g, row, x0, x1);
            else
                walk_hemisphere<T, M, P, false, NCH, false>(a.s, a.even, r_first, r_last, mm, up, k0, k1, sc, fw,
                                                            set_stride, a.n_sets, g, row, x0, x1);
        }
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        ends[((blk * 64 + lane) * NCH + c) * M] = x0[c];
        if (M == 2) ends[((blk * 64 + lane) * NCH + c) * M + 1] = x1[c];
    }
    __syncthreads();
    if (blk == 0 || !active) return;

    // fold: the start of this block, per chain
    T y0[NCH], y1[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        y0[c] = ends[(lane * NCH + c) * M];
        y1[c] = M == 2 ? ends[(lane * NCH + c) * M + 1] : T(0);
    }
    for (int k = 1; k < blk; ++k) {
        for (int i = k * a.fine_per; i < (k + 1) * a.fine_per; ++i) {
            const T* __restrict__ p = ph + ((size_t)i * a.m_rows + mm) * (M * M);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if (M == 1) {
                    y0[c] = p[0] * y0[c];
                } else {
                    const T t0 = fma(p[0], y0[c], p[1] * y1[c]);
                    const T t1 = fma(p[2], y0[c], p[3] * y1[c]);
                    y0[c] = t0;
                    y1[c] = t1;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            y0[c] += ends[((k * 64 + lane) * NCH + c) * M];
            if (M == 2) y1[c] += ends[((k * 64 + lane) * NCH + c) * M + 1];
        }
    }
    // pass 2: this block again from its true start, with stores
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        x0[c] = y0[c];
        x1[c] = y1[c];
    }
    if (h == 0)
        walk_hemisphere<T, M, P, true, NCH, true>(a.s, a.even, r_first, r_last, mm, up, k0, k1, sc, fw, set_stride,
                                                  a.n_sets, g, row, x0, x1);
    else
        walk_hemisphere<T, M, P, false, NCH, true>(a.s, a.even, r_first, r_last, mm, up, k0, k1, sc, fw, set_stride,
                                                   a.n_sets, g, row, x0, x1);
}

// The affine scan for orders 3 and 4: the layout of scan_kernel with one part per lane
// (32 modes x 2 parts per wave, one wave per ring block), the general-order walk with one
// group per stage, block end states of M components in LDS, and the fold through the M x M
// block transitions.
template <typename T, int M, int B>
__global__ __launch_bounds__(64 * B) void scan_gen_kernel(ScanArgs a, const T* __restrict__ fac,
                                                          const T* __restrict__ phi, T* __restrict__ out)
{
    __shared__ T ends[B * 64 * M];
    const int bx = blockIdx.x;
    const int L = (bx & 7) * a.per_xcd + (bx >> 3);
    if (L >= a.n_wg) return;
    const int mt = L / a.n_fh;
    const int fh = L - mt * a.n_fh;
    const int f = fh >> 1, h = fh & 1;
    const int blk = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int m = mt * 32 + (lane >> 1);
    const int part = lane & 1;
    const bool in_range = m < a.m_rows;
    const bool active = in_range && m <= a.m_top && !(m == 0 && part == 1);
    const size_t row = (size_t)a.n_phi;
    T* __restrict__ g = out + (size_t)f * a.n_theta * a.n_phi + 2 * (in_range ? m : 0) + part;
    if (in_range && !active && blk == 0) zero_chain<T, 1>(a.n_theta, a.s, h, g, row);

    const uint64_t key = (((uint64_t)a.seed_hi << 32) | a.seed_lo) + (uint64_t)f;
    const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
    const int mm = active ? m : 0;
    const T* __restrict__ fm = fac + (size_t)mm * factor_stride(M);
    const T* __restrict__ fw = fm + (h ? a.south_off : 0);
    const T* __restrict__ ph = phi + (h ? a.phi_south_off : 0);
    const size_t set_stride = (size_t)a.m_rows * factor_stride(M);
    T sc[1];
    chain_scales<T, 1>(mm, (uint32_t)part, sc);
    const uint32_t um = (uint32_t)mm, up = (uint32_t)part;
    const int j0 = a.even ? 2 : 1;
    const long walk = a.n_sets - j0;
    const int jb = j0 + (int)(walk * (blk * a.fine_per) / a.fine);
    const int je = j0 + (int)(walk * ((blk + 1) * a.fine_per) / a.fine);
    const int r_first = h == 0 ? a.s - jb + a.even : a.s + jb;
    const int r_last = h == 0 ? a.s - (je - 1) + a.even : a.s + (je - 1);

    // pass 1: block 0 from the start state (final, stored); the others from zero
    T x[1][M];
#pragma unroll
    for (int p = 0; p < M; ++p) x[0][p] = T(0);
    if (active) {
        if (blk == 0) {
            chain_start_gen<T, M, 1>(a.s, a.even, h, um, up, k0, k1, sc, fm, set_stride, g, row, true, x);
            if (h == 0)
                walk_gen<T, M, 1, true, true, 1>(a.s, a.even, r_first, r_last, um, up, k0, k1, sc, fw, set_stride,
                                              a.n_sets, g, row, x);
            else
                walk_gen<T, M, 1, false, true, 1>(a.s, a.even, r_first, r_last, um, up, k0, k1, sc, fw, set_stride,
                                               a.n_sets, g, row, x);
        } else {
            if (h == 0)
                walk_gen<T, M, 1, true, false, 1>(a.s, a.even, r_first, r_last, um, up, k0, k1, sc, fw, set_stride,
                                               a.n_sets, g, row, x);
            else
                walk_gen<T, M, 1, false, false, 1>(a.s, a.even, r_first, r_last, um, up, k0, k1, sc, fw, set_stride,
                                                a.n_sets, g, row, x);
        }
    }
#pragma unroll
    for (int p = 0; p < M; ++p) ends[(blk * 64 + lane) * M + p] = x[0][p];
    __syncthreads();
    if (blk == 0 || !active) return;

    // fold: the start of this block
    T y[1][M];
#pragma unroll
    for (int p = 0; p < M; ++p) y[0][p] = ends[lane * M + p];
    for (int k = 1; k < blk; ++k) {
        for (int i = k * a.fine_per; i < (k + 1) * a.fine_per; ++i) {
            const T* __restrict__ q = ph + ((size_t)i * a.m_rows + mm) * (M * M);
            T t[M];
#pragma unroll
            for (int p = 0; p < M; ++p) {
                T acc = q[p * M + M - 1] * y[0][M - 1];
#pragma unroll
                for (int c = M - 2; c >= 0; --c) acc = fma(q[p * M + c], y[0][c], acc);
                t[p] = acc;
            }
#pragma unroll
            for (int p = 0; p < M; ++p) y[0][p] = t[p];
        }
#pragma unroll
        for (int p = 0; p < M; ++p) y[0][p] += ends[(k * 64 + lane) * M + p];
    }
    // pass 2: this block again from its true start, with stores
    if (h == 0)
        walk_gen<T, M, 1, true, true, 1>(a.s, a.even, r_first, r_last, um, up, k0, k1, sc, fw, set_stride, a.n_sets, g,
                                      row, y);
    else
        walk_gen<T, M, 1, false, true, 1>(a.s, a.even, r_first, r_last, um, up, k0, k1, sc, fw, set_stride, a.n_sets,
                                       g, row, y);
}

template <typename T, int M>
void launch_scan_gen_t(const ScanArgs& a, int blocks, const T* fac, const T* phi, T* out, hipStream_t st)
{
    const dim3 grid((unsigned)(a.per_xcd * 8));
    switch (blocks) {
        case 2: hipLaunchKernelGGL((scan_gen_kernel<T, M, 2>), grid, dim3(128), 0, st, a, fac, phi, out); break;
        case 4: hipLaunchKernelGGL((scan_gen_kernel<T, M, 4>), grid, dim3(256), 0, st, a, fac, phi, out); break;
        default: hipLaunchKernelGGL((scan_gen_kernel<T, M, 8>), grid, dim3(512), 0, st, a, fac, phi, out); break;
    }
}

template <typename T, int M, int NCH>
void launch_scan_t(const ScanArgs& a, int blocks, const T* fac, const T* phi, T* out, hipStream_t st)
{
    const dim3 grid((unsigned)(a.per_xcd * 8));
    switch (blocks) {
        case 2: hipLaunchKernelGGL((scan_kernel<T, M, 2, NCH>), grid, dim3(128), 0, st, a, fac, phi, out); break;
        case 4: hipLaunchKernelGGL((scan_kernel<T, M, 4, NCH>), grid, dim3(256), 0, st, a, fac, phi, out); break;
        case 8: hipLaunchKernelGGL((scan_kernel<T, M, 8, NCH>), grid, dim3(512), 0, st, a, fac, phi, out); break;
        default:
            if constexpr (sizeof(T) == 4)   // FP64 scans stop at 8 blocks
                hipLaunchKernelGGL((scan_kernel<T, M, 16, NCH>), grid, dim3(1024), 0, st, a, fac, phi, out);
            break;
    }
}

// Threads per row: H/8 clamped to [64, 256], and 512 for the largest rows (FP32 n_phi =
// 16384, FP64 n_phi >= 8192) so that each thread holds fewer butterflies.
template <typename T, int LOG2H>
struct FftThreads {
    static constexpr int base = (1 << LOG2H) / 8 < 64 ? 64 : ((1 << LOG2H) / 8 > 256 ? 256 : (1 << LOG2H) / 8);
    static constexpr int value = (LOG2H >= (sizeof(T) == 4 ? 13 : 12)) ? 512 : base;
};

// Rows prefetch the next row during the current one's passes while the extra registers
// fit (FP32 every size, FP64 up to n_phi = 8192); FP64 rows of 16384 load row by row.
template <typename T, int LOG2H>
struct FftPrefetch {
    static constexpr bool value = sizeof(T) == 4 ? LOG2H <= 13 : LOG2H <= 12;
};

// Register budget in waves per SIMD: 4 (128 VGPRs) for small rows, else SMF_FFT_WAVES_BIG
// (2: 256 VGPRs), and 1 for the 512-thread rows.
#ifndef SMF_FFT_WAVES_BIG
#define SMF_FFT_WAVES_BIG 2
#endif
template <typename T, int LOG2H>
struct FftWaves {
    static constexpr int value = FftThreads<T, LOG2H>::value == 512 ? 1
                                 : (LOG2H < (sizeof(T) == 4 ? 11 : 8) ? 4 : SMF_FFT_WAVES_BIG);
};

// Each workgroup transforms rows blockIdx.x, blockIdx.x + gridDim.x, ...
template <typename T, int LOG2H>
__global__ __launch_bounds__((FftThreads<T, LOG2H>::value), (FftWaves<T, LOG2H>::value)) void c2r_kernel(
    T* __restrict__ data, const T* __restrict__ twr, int m_top, int rows, Epilogue<T> ep)
{
    extern __shared__ unsigned char smem_raw[];
    c2r_rows<T, LOG2H, FftThreads<T, LOG2H>::value, FftPrefetch<T, LOG2H>::value>(
        data, twr, m_top, reinterpret_cast<Cx<T>*>(smem_raw), rows, blockIdx.x, gridDim.x, ep);
}

// Waves per SIMD of the radix-16 kernel: 2 (it needs about 244 VGPRs; with 128 or 168 it
// spills)
#ifndef SMF_R16_WAVES
#define SMF_R16_WAVES 2
#endif
// Rows of n_phi = 8192 by three radix-16 passes (c2r_row_r16), 256 threads, FP32.
template <typename T>
__global__ __launch_bounds__(256, SMF_R16_WAVES) void c2r16_kernel(T* __restrict__ data,
                                                                             const T* __restrict__ twr, int m_top,
                                                                             int rows, Epilogue<T> ep)
{
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
    for (int r = blockIdx.x; r < rows; r += gridDim.x) c2r_row_r16<T>(data + (size_t)r * 8192, twr, m_top, buf, ep);
}

// Workgroups of the row-looping FFT: enough to fill every CU several times over.
constexpr int kFftGrid = 2048;

// FP32 rows of n_phi = 8192 take the radix-16 kernel (0.446 against 0.454 ms for the 8-field
// 4096 x 8192 workload; with the mirror partners loaded from global memory instead of
// exchanged through LDS it took 0.574 ms)
#ifndef SMF_FFT_R16
#define SMF_FFT_R16 1
#endif

template <typename T, int LOG2H>
hipError_t launch_c2r_t(const T* tw, int m_top, int rows, T* data, const Epilogue<T>& ep, hipStream_t st)
{
    const size_t lds = sizeof(Cx<T>) * lds_slots(1 << LOG2H);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)c2r_kernel<T, LOG2H>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int grid = rows < kFftGrid ? rows : kFftGrid;
    hipLaunchKernelGGL((c2r_kernel<T, LOG2H>), dim3(grid), dim3(FftThreads<T, LOG2H>::value), lds, st, data, tw,
                       m_top, rows, ep);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_c2r(int log2h, const T* tw, int m_top, int rows, T* data, const Epilogue<T>& ep,
                        hipStream_t st)
{
    if constexpr (sizeof(T) == 4) {
        if (SMF_FFT_R16 && log2h == 12) {
            const size_t lds = sizeof(Cx<T>) * lds_slots(4096);
            const int grid = rows < kFftGrid ? rows : kFftGrid;
            hipLaunchKernelGGL((c2r16_kernel<T>), dim3(grid), dim3(256), lds, st, data, tw, m_top, rows, ep);
            return hipGetLastError();
        }
    }
    switch (log2h) {
        case 1: return launch_c2r_t<T, 1>(tw, m_top, rows, data, ep, st);
        case 2: return launch_c2r_t<T, 2>(tw, m_top, rows, data, ep, st);
        case 3: return launch_c2r_t<T, 3>(tw, m_top, rows, data, ep, st);
        case 4: return launch_c2r_t<T, 4>(tw, m_top, rows, data, ep, st);
        case 5: return launch_c2r_t<T, 5>(tw, m_top, rows, data, ep, st);
        case 6: return launch_c2r_t<T, 6>(tw, m_top, rows, data, ep, st);
        case 7: return launch_c2r_t<T, 7>(tw, m_top, rows, data, ep, st);
        case 8: return launch_c2r_t<T, 8>(tw, m_top, rows, data, ep, st);
        case 9: return launch_c2r_t<T, 9>(tw, m_top, rows, data, ep, st);
        case 10: return launch_c2r_t<T, 10>(tw, m_top, rows, data, ep, st);
        case 11: return launch_c2r_t<T, 11>(tw, m_top, rows, data, ep, st);
        case 12: return launch_c2r_t<T, 12>(tw, m_top, rows, data, ep, st);
        case 13: return launch_c2r_t<T, 13>(tw, m_top, rows, data, ep, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_recursion(const Geometry& g, int fp64, const void* fac, size_t south_off, uint64_t seed,
                            int count, void* out, int nch, hipStream_t st)
{
    if (nch != 1 && (nch != 2 || fp64)) return hipErrorInvalidValue;
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
    const int modes_per_wave = nch == 2 ? 64 : 32;
    const int n_mt = (g.m_rows + modes_per_wave - 1) / modes_per_wave;
    a.n_wg = n_mt * a.n_fg;
    a.per_xcd = (a.n_wg + 7) / 8;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.south_off = south_off;
    const dim3 grid((unsigned)(a.per_xcd * 8));
    if (g.order >= 3) {
        if (fp64) {
            if (g.order == 3)
                hipLaunchKernelGGL((recursion_gen_kernel<double, 3, 1>), grid, dim3(256), 0, st, a, (const double*)fac,
                                   (double*)out);
            else
                hipLaunchKernelGGL((recursion_gen_kernel<double, 4, 1>), grid, dim3(256), 0, st, a, (const double*)fac,
                                   (double*)out);
        } else if (nch == 2) {
            if (g.order == 3)
                hipLaunchKernelGGL((recursion_gen_kernel<float, 3, 2>), grid, dim3(256), 0, st, a, (const float*)fac,
                                   (float*)out);
            else
                hipLaunchKernelGGL((recursion_gen_kernel<float, 4, 2>), grid, dim3(256), 0, st, a, (const float*)fac,
                                   (float*)out);
        } else {
            if (g.order == 3)
                hipLaunchKernelGGL((recursion_gen_kernel<float, 3, 1>), grid, dim3(256), 0, st, a, (const float*)fac,
                                   (float*)out);
            else
                hipLaunchKernelGGL((recursion_gen_kernel<float, 4, 1>), grid, dim3(256), 0, st, a, (const float*)fac,
                                   (float*)out);
        }
    } else if (fp64) {
        if (g.order == 1)
            hipLaunchKernelGGL((recursion_kernel<double, 1, 1>), grid, dim3(256), 0, st, a,
                               (const double*)fac, (double*)out);
        else
            hipLaunchKernelGGL((recursion_kernel<double, 2, 1>), grid, dim3(256), 0, st, a,
                               (const double*)fac, (double*)out);
    } else if (nch == 2) {
        if (g.order == 1)
            hipLaunchKernelGGL((recursion_kernel<float, 1, 2>), grid, dim3(256), 0, st, a,
                               (const float*)fac, (float*)out);
        else
            hipLaunchKernelGGL((recursion_kernel<float, 2, 2>), grid, dim3(256), 0, st, a,
                               (const float*)fac, (float*)out);
    } else {
        if (g.order == 1)
            hipLaunchKernelGGL((recursion_kernel<float, 1, 1>), grid, dim3(256), 0, st, a,
                               (const float*)fac, (float*)out);
        else
            hipLaunchKernelGGL((recursion_kernel<float, 2, 1>), grid, dim3(256), 0, st, a,
                               (const float*)fac, (float*)out);
    }
    return hipGetLastError();
}

hipError_t launch_scan(const Geometry& g, int fp64, const void* fac, size_t south_off, const void* phi,
                       size_t phi_south_off, int fine_blocks,
                       int blocks, uint64_t seed, int count, void* out, int nch, hipStream_t st)
{
    if (blocks < 2 || blocks > scan_max_blocks(fp64, g.order) || (blocks & (blocks - 1)) || fine_blocks % blocks)
        return hipErrorInvalidValue;
    if (nch != 1 && (nch != 2 || fp64 || g.order > 2)) return hipErrorInvalidValue;
    ScanArgs a;
    a.n_theta = g.n_theta;
    a.n_phi = g.n_phi;
    a.m_top = g.m_top;
    a.m_rows = g.m_rows;
    a.n_sets = g.n_sets;
    a.s = g.s;
    a.even = g.even;
    a.n_fh = 2 * count;
    a.fine_per = fine_blocks / blocks;
    a.fine = fine_blocks;
    a.south_off = south_off;
    a.phi_south_off = phi_south_off;
    const int modes_per_wave = nch == 2 ? 64 : 32;
    const int n_mt = (g.m_rows + modes_per_wave - 1) / modes_per_wave;
    a.n_wg = n_mt * a.n_fh;
    a.per_xcd = (a.n_wg + 7) / 8;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    if (g.order >= 3) {
        if (fp64) {
            if (g.order == 3) launch_scan_gen_t<double, 3>(a, blocks, (const double*)fac, (const double*)phi, (double*)out, st);
            else launch_scan_gen_t<double, 4>(a, blocks, (const double*)fac, (const double*)phi, (double*)out, st);
        } else {
            if (g.order == 3) launch_scan_gen_t<float, 3>(a, blocks, (const float*)fac, (const float*)phi, (float*)out, st);
            else launch_scan_gen_t<float, 4>(a, blocks, (const float*)fac, (const float*)phi, (float*)out, st);
        }
    } else if (fp64) {
        if (g.order == 1) launch_scan_t<double, 1, 1>(a, blocks, (const double*)fac, (const double*)phi, (double*)out, st);
        else launch_scan_t<double, 2, 1>(a, blocks, (const double*)fac, (const double*)phi, (double*)out, st);
    } else if (nch == 2) {
        if (g.order == 1) launch_scan_t<float, 1, 2>(a, blocks, (const float*)fac, (const float*)phi, (float*)out, st);
        else launch_scan_t<float, 2, 2>(a, blocks, (const float*)fac, (const float*)phi, (float*)out, st);
    } else {
        if (g.order == 1) launch_scan_t<float, 1, 1>(a, blocks, (const float*)fac, (const float*)phi, (float*)out, st);
        else launch_scan_t<float, 2, 1>(a, blocks, (const float*)fac, (const float*)phi, (float*)out, st);
    }
    return hipGetLastError();
}

hipError_t launch_c2r(const Geometry& g, int fp64, const void* tw, int count, void* data,
                      const LognormalMap* ln, hipStream_t st)
{
    const int log2h = __builtin_ctz((unsigned)g.n_phi) - 1;
    const int rows = count * g.n_theta;
    if (rows == 0) return hipSuccess;
    if (fp64) {
        const Epilogue<double> ep = {ln ? ln->mu : 0.0, ln ? ln->sigma : 0.0, ln ? 1 : 0};
        return dispatch_c2r<double>(log2h, (const double*)tw, g.m_top, rows, (double*)data, ep, st);
    }
    const Epilogue<float> ep = {ln ? (float)ln->mu : 0.0f, ln ? (float)ln->sigma : 0.0f, ln ? 1 : 0};
    return dispatch_c2r<float>(log2h, (const float*)tw, g.m_top, rows, (float*)data, ep, st);
}

}  // namespace smf
