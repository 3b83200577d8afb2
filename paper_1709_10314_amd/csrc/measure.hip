// Throughput references for the roofline of the chain kernels, measured on the device they
// run on: the sampler's white noise alone (Philox4x32-10 words through Box-Muller in FP32,
// the instruction mix of the recursion without its loads and stores) and plain FP32 fused
// multiply-adds (the vector ALU's issue rate for the unpacked instructions this library is
// built with).  Each lane reduces what it made to one float and stores it, so nothing is
// dead code; the caller times the launch.
#include "rng.h"
#include "smf_internal.h"

namespace smf {
namespace {

constexpr int kMeasureThreads = 256;
// Philox blocks per stage, as many as a lane of the two-part order-2 walk runs per stage
constexpr int kMeasureStage = 8;

__global__ __launch_bounds__(kMeasureThreads) void normals_peak_kernel(uint32_t k0, uint32_t k1, int stages,
                                                                       float* __restrict__ out)
{
    const uint32_t lane = blockIdx.x * kMeasureThreads + threadIdx.x;
    float acc = 0.0f;
    for (int st = 0; st < stages; ++st) {
        uint32_t c0[kMeasureStage], c2[kMeasureStage];
#pragma unroll
        for (int i = 0; i < kMeasureStage; ++i) {
            c0[i] = (uint32_t)(st * kMeasureStage + i);
            c2[i] = (uint32_t)i & 1u;
        }
        PhiloxBlock w[kMeasureStage];
        philox4x32_10_n<kMeasureStage>(c0, lane, c2, k0, k1, w);
#pragma unroll
        for (int i = 0; i < kMeasureStage; ++i) {
            float a, b, c, d;
            BoxMuller<float>::pair(w[i].w[0], w[i].w[1], 0.70710678118654752440f, a, b);
            BoxMuller<float>::pair(w[i].w[2], w[i].w[3], 0.70710678118654752440f, c, d);
            acc += (a + b) + (c + d);
        }
    }
    out[lane] = acc;
}

// 8 independent chains of x <- x * a + b per lane
constexpr int kFmaChains = 8;

__global__ __launch_bounds__(kMeasureThreads) void fma_peak_kernel(float a, float b, int iters,
                                                                   float* __restrict__ out)
{
    const uint32_t lane = blockIdx.x * kMeasureThreads + threadIdx.x;
    float x[kFmaChains];
#pragma unroll
    for (int i = 0; i < kFmaChains; ++i) x[i] = (float)(lane + i) * 1e-9f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int i = 0; i < kFmaChains; ++i) x[i] = fmaf(x[i], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kFmaChains; ++i) s += x[i];
    out[lane] = s;
}

}  // namespace
}  // namespace smf

extern "C" {

int smf_measure_normals(uint64_t seed, int workgroups, int stages, void* out_dev, void* hip_stream)
{
    if (workgroups < 1 || stages < 1 || !out_dev) return SMF_EINVAL;
    hipLaunchKernelGGL(smf::normals_peak_kernel, dim3((unsigned)workgroups), dim3(smf::kMeasureThreads), 0,
                       (hipStream_t)hip_stream, (uint32_t)seed, (uint32_t)(seed >> 32), stages, (float*)out_dev);
    return hipGetLastError() == hipSuccess ? SMF_OK : SMF_EHIP;
}

int smf_measure_fma(int workgroups, int iters, void* out_dev, void* hip_stream)
{
    if (workgroups < 1 || iters < 1 || !out_dev) return SMF_EINVAL;
    hipLaunchKernelGGL(smf::fma_peak_kernel, dim3((unsigned)workgroups), dim3(smf::kMeasureThreads), 0,
                       (hipStream_t)hip_stream, 0.999999f, 1e-7f, iters, (float*)out_dev);
    return hipGetLastError() == hipSuccess ? SMF_OK : SMF_EHIP;
}

}  // extern "C"
