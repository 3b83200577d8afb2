// Batched sampling of many fields of uneven shape, spectrum and order 1..4 (FP32) in two
// launches: one over the chain items of every field (Creasey & Lang, Alg. 2; eqs.
// (state_initial), (state_space)), then one over every ring of every field (the inverse
// FFT, Alg. 2 last step).  Both grids are flat work lists built at setup: a workgroup
// looks its item up and runs it, with no queue, no counters and no waiting, so the call
// is a pair of ordinary launches that a HIP graph can capture.
//
// A chain item is (field, group of `tiles` m-tiles); the workgroup holds 2 x tiles waves
// (hemisphere x m-tile).  Chain items are listed longest chain first so that the
// in-order dispatch starts the long fields early.  The number of m-tiles per item is the
// tile shape the autotuner picks.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "batch.h"
#include "device_path.h"

namespace smf {
namespace {

constexpr int kFftThreads = 256;

template <int LOG2H>
__device__ __forceinline__ void fft_item(float* row, const float* tw, int m_top, Cx<float>* buf)
{
    c2r_row<float, LOG2H, kFftThreads>(row, tw, m_top, buf, Epilogue<float>{0.0f, 0.0f, 0});
}

__device__ void dispatch_fft(int log2h, float* row, const float* tw, int m_top, Cx<float>* buf)
{
    switch (log2h) {
        case 1: fft_item<1>(row, tw, m_top, buf); break;
        case 2: fft_item<2>(row, tw, m_top, buf); break;
        case 3: fft_item<3>(row, tw, m_top, buf); break;
        case 4: fft_item<4>(row, tw, m_top, buf); break;
        case 5: fft_item<5>(row, tw, m_top, buf); break;
        case 6: fft_item<6>(row, tw, m_top, buf); break;
        case 7: fft_item<7>(row, tw, m_top, buf); break;
        case 8: fft_item<8>(row, tw, m_top, buf); break;
        case 9: fft_item<9>(row, tw, m_top, buf); break;
        case 10: fft_item<10>(row, tw, m_top, buf); break;
        case 11: fft_item<11>(row, tw, m_top, buf); break;
        default: break;
    }
}

// Chain item `item` by the calling wave w (hemisphere w & 1, m-tile tiles * sub + (w >> 1)).
// No barriers: each wave returns on its own.
__device__ __forceinline__ void chain_item(const BatchArgs& a, int item, int w)
{
    const uint32_t code = a.chain_items[item];
    const int fi = (int)(code >> 16);
    const int sub = (int)(code & 0xFFFF);
    const BatchField& F = a.fields[fi];
    const int h = w & 1;
    const int lane = threadIdx.x & 63;
    const int m = (a.tiles * sub + (w >> 1)) * 32 + (lane >> 1), part = lane & 1;
    if (m >= F.m_rows) return;
    float* g = (a.call ? a.call[fi].out : a.out + F.out_off) + 2 * m + part;
    if (m > F.m_top || (m == 0 && part == 1)) {
        zero_chain<float>(F.n_theta, F.s, h, g, (size_t)F.n_phi);
        return;
    }
    const uint64_t key = a.call ? a.call[fi].key : a.seed + (uint64_t)F.seed_off;
    const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
    const size_t stride = (size_t)F.m_rows * factor_stride(F.order);
    switch (F.order) {
        case 1:
            run_chain<float, 1>(F.n_theta, F.s, F.even, F.n_sets, h, m, part, k0, k1,
                                F.fac + (size_t)m * factor_stride(1), stride, g, (size_t)F.n_phi);
            break;
        case 2:
            run_chain<float, 2>(F.n_theta, F.s, F.even, F.n_sets, h, m, part, k0, k1,
                                F.fac + (size_t)m * factor_stride(2), stride, g, (size_t)F.n_phi);
            break;
        case 3:
            run_chain_gen<float, 3>(F.n_theta, F.s, F.even, F.n_sets, h, m, part, k0, k1,
                                    F.fac + (size_t)m * factor_stride(3), stride, g, (size_t)F.n_phi);
            break;
        default:
            run_chain_gen<float, 4>(F.n_theta, F.s, F.even, F.n_sets, h, m, part, k0, k1,
                                    F.fac + (size_t)m * factor_stride(4), stride, g, (size_t)F.n_phi);
            break;
    }
}

// One workgroup per chain item.
__global__ __launch_bounds__(kMaxChainThreads) void batch_chain_kernel(BatchArgs a)
{
    chain_item(a, blockIdx.x, __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)));
}

// One workgroup per ring of every field.
__global__ __launch_bounds__(kFftThreads) void batch_fft_kernel(BatchArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    const uint32_t code = a.fft_items[blockIdx.x];
    const int fi = (int)(code >> 16);
    const int ring = (int)(code & 0xFFFF);
    const BatchField& F = a.fields[fi];
    float* base = a.call ? a.call[fi].out : a.out + F.out_off;
    dispatch_fft(F.log2h, base + (size_t)ring * F.n_phi, F.tw, F.m_top,
                 reinterpret_cast<Cx<float>*>(smem_raw));
}

// The persistent form: one cooperative launch of as many workgroups of NT = 128 * tiles threads
// as the device holds at once.  Each workgroup runs the chain items blockIdx.x, blockIdx.x +
// gridDim.x, ... (listed longest first, so the stride deals them out evenly), then every
// workgroup meets at the grid barrier, after which all chain outputs are visible, and runs
// the ring items the same way with all its threads.  The barrier is the runtime's cooperative
// grid barrier, valid because the launch is cooperative and sized to co-residency.
template <int NT>
__device__ __forceinline__ void fft_item_nt(int log2h, float* row, const float* tw, int m_top, Cx<float>* buf)
{
    const Epilogue<float> ep = {0.0f, 0.0f, 0};
    switch (log2h) {
        case 1: c2r_row<float, 1, NT>(row, tw, m_top, buf, ep); break;
        case 2: c2r_row<float, 2, NT>(row, tw, m_top, buf, ep); break;
        case 3: c2r_row<float, 3, NT>(row, tw, m_top, buf, ep); break;
        case 4: c2r_row<float, 4, NT>(row, tw, m_top, buf, ep); break;
        case 5: c2r_row<float, 5, NT>(row, tw, m_top, buf, ep); break;
        case 6: c2r_row<float, 6, NT>(row, tw, m_top, buf, ep); break;
        case 7: c2r_row<float, 7, NT>(row, tw, m_top, buf, ep); break;
        case 8: c2r_row<float, 8, NT>(row, tw, m_top, buf, ep); break;
        case 9: c2r_row<float, 9, NT>(row, tw, m_top, buf, ep); break;
        case 10: c2r_row<float, 10, NT>(row, tw, m_top, buf, ep); break;
        case 11: c2r_row<float, 11, NT>(row, tw, m_top, buf, ep); break;
        default: break;
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void batch_persistent_kernel(BatchArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int it = blockIdx.x; it < a.n_chain_items; it += gridDim.x) chain_item(a, it, w);
    cooperative_groups::this_grid().sync();
    Cx<float>* buf = reinterpret_cast<Cx<float>*>(smem_raw);
    for (int it = blockIdx.x; it < a.n_fft_items; it += gridDim.x) {
        const uint32_t code = a.fft_items[it];
        const int fi = (int)(code >> 16);
        const int ring = (int)(code & 0xFFFF);
        const BatchField& F = a.fields[fi];
        float* base = a.call ? a.call[fi].out : a.out + F.out_off;
        fft_item_nt<NT>(F.log2h, base + (size_t)ring * F.n_phi, F.tw, F.m_top, buf);
        __syncthreads();   // the row's last LDS reads before the next row's writes
    }
}

template <int NT>
hipError_t launch_persistent_t(const BatchArgs& a, size_t lds, hipStream_t st, int* grid_out)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)batch_persistent_kernel<NT>, NT, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1 || cus < 1) return hipErrorCooperativeLaunchTooLarge;
    const long items = std::max<long>(a.n_chain_items, a.n_fft_items);
    const int grid = (int)std::min<long>((long)per_cu * cus, std::max<long>(items, 1));
    if (grid_out) *grid_out = grid;
    BatchArgs args = a;
    void* params[] = {&args};
    return hipLaunchCooperativeKernel((const void*)batch_persistent_kernel<NT>, dim3(grid), dim3(NT), params,
                                      (unsigned)lds, st);
}

}  // namespace

hipError_t launch_batch_persistent(const BatchArgs& a, size_t lds, hipStream_t st, int* grid_out)
{
    switch (a.tiles) {
        case 1: return launch_persistent_t<128>(a, lds, st, grid_out);
        case 2: return launch_persistent_t<256>(a, lds, st, grid_out);
        case 4: return launch_persistent_t<512>(a, lds, st, grid_out);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch(const BatchArgs& a, size_t lds, hipStream_t st)
{
    if (a.n_chain_items > 0) {
        hipLaunchKernelGGL(batch_chain_kernel, dim3(a.n_chain_items), dim3(64 * 2 * a.tiles), 0, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.n_fft_items > 0) {
        hipLaunchKernelGGL(batch_fft_kernel, dim3(a.n_fft_items), dim3(kFftThreads), lds, st, a);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace smf
