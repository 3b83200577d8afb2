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

// One workgroup per chain item; wave w -> hemisphere w & 1, m-tile tiles * sub + (w >> 1).
__global__ __launch_bounds__(kMaxChainThreads) void batch_chain_kernel(BatchArgs a)
{
    const uint32_t code = a.chain_items[blockIdx.x];
    const int fi = (int)(code >> 16);
    const int sub = (int)(code & 0xFFFF);
    const BatchField& F = a.fields[fi];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
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

}  // namespace

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
