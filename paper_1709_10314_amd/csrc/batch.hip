// Batched sampling of many fields of uneven shape, spectrum and order in one persistent
// launch (FP32).  Each field runs Alg. 2 of Creasey & Lang: its ring chains (eqs.
// (state_initial), (state_space)) and then the inverse FFT of each of its rings.
//
// Work items are pulled from one atomic counter.  Items 0..n_rec-1 are chain items
// (field, pair of m-tiles; four waves = 2 hemispheres x 2 m-tiles), ordered longest chain
// first; items n_rec.. are FFT items (field, ring) in the same field order.  An FFT item
// waits until its field's chain items are all done (per-field counter, release/acquire
// at agent scope so the modes written on another XCD are visible).  Chain items never
// wait, and every chain item is taken before any FFT item, so the waits always end; they
// are bounded anyway, and a wait that runs out sets the error word instead of hanging.
#include "batch.h"
#include "device_path.h"

namespace smf {
namespace {

constexpr int kBatchThreads = 256;

template <int LOG2H>
__device__ __forceinline__ void fft_item(float* row, const float* tw, int m_top, Cx<float>* buf)
{
    c2r_row<float, LOG2H, kBatchThreads>(row, tw, m_top, buf);
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

__global__ __launch_bounds__(kBatchThreads) void batch_reset_kernel(int* counters, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        counters[i] = 0;
}

__global__ __launch_bounds__(kBatchThreads) void batch_kernel(BatchArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    Cx<float>* buf = reinterpret_cast<Cx<float>*>(smem_raw);
    __shared__ int s_item;
    int* queue = a.counters;
    int* err = a.counters + 1;
    int* done = a.counters + 2;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(queue, 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= a.n_items) return;
        const uint32_t code = a.items[item];
        const int fi = (int)(code >> 16);
        const int sub = (int)(code & 0xFFFF);
        const BatchField F = a.fields[fi];
        if (item < a.n_rec) {
            // chain item: wave w -> hemisphere w & 1, m-tile 2 sub + (w >> 1)
            const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
            const int h = w & 1;
            const int lane = tid & 63;
            const int m = (2 * sub + (w >> 1)) * 32 + (lane >> 1), part = lane & 1;
            if (m < F.m_rows) {
                float* g = a.out + F.out_off + 2 * m + part;
                if (m > F.m_top || (m == 0 && part == 1)) {
                    zero_chain<float>(F.n_theta, F.s, h, g, (size_t)F.n_phi);
                } else {
                    const uint64_t key = a.seed + (uint64_t)F.seed_off;
                    const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
                    const size_t stride = (size_t)F.m_rows * factor_stride(F.order);
                    if (F.order == 1)
                        run_chain<float, 1>(F.n_theta, F.s, F.even, h, m, part, k0, k1,
                                            F.fac + (size_t)m * factor_stride(1), stride, g,
                                            (size_t)F.n_phi);
                    else
                        run_chain<float, 2>(F.n_theta, F.s, F.even, h, m, part, k0, k1,
                                            F.fac + (size_t)m * factor_stride(2), stride, g,
                                            (size_t)F.n_phi);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0) __hip_atomic_fetch_add(done + fi, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // FFT item: ring `sub` of field fi, once all chain items of fi are done
            if (tid == 0) {
                int spins = 0;
                if (a.spin_limit < 0) atomicOr(err, 1);   // wait skipped on request
                else while (__hip_atomic_load(done + fi, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < F.n_rec_items) {
                    __builtin_amdgcn_s_sleep(8);
                    if (++spins > a.spin_limit) {
                        atomicOr(err, 1);
                        break;
                    }
                }
            }
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            dispatch_fft(F.log2h, a.out + F.out_off + (size_t)sub * F.n_phi, F.tw, F.m_top, buf);
            __syncthreads();
        }
    }
}

}  // namespace

hipError_t launch_batch(const BatchArgs& a, int grid, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(kBatchThreads), 0, st, a.counters,
                       a.n_fields + 2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(kBatchThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t batch_max_blocks_per_cu(size_t lds, int* blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void*)batch_kernel, kBatchThreads,
                                                        lds);
}

}  // namespace smf
