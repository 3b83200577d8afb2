// Counter-based white noise for the ring recursion: Philox4x32-10 (Salmon, Moraes, Dror,
// Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and Box-Muller.
//
// Counter map: the normal xi_q that produces ring r of chain (m, part) of a field keyed
// K = seed + field is word w = (r M + q) mod 4 of the Philox block with counter
// (floor((r M + q) / 4), m, part, 0) and key (lo32(K), hi32(K)).  Words are turned into
// uniforms u = (x + 1/2) 2^-32 and paired (0,1), (2,3) by Box-Muller:
//   n_{2i} = sqrt(-2 ln u_{2i}) cos(2 pi u_{2i+1}),  n_{2i+1} = sqrt(-2 ln u_{2i}) sin(2 pi u_{2i+1}).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smf {

struct PhiloxBlock {
    uint32_t w[4];
};

// a ^ b ^ c in one gfx950 three-input bitwise op (truth table 0x96: odd parity)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ PhiloxBlock philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                     uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t pb = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    PhiloxBlock b;
    b.w[0] = c0; b.w[1] = c1; b.w[2] = c2; b.w[3] = c3;
    return b;
}

// N independent Philox blocks with counters (c0[i], c1, c2[i], 0), advanced one round at a
// time.
template <int N>
struct PhiloxLanes {
    uint32_t a[N], b[N], c[N], d[N];
    uint32_t k0, k1;

    __device__ __forceinline__ PhiloxLanes(const uint32_t* c0, uint32_t c1, const uint32_t* c2, uint32_t key0,
                                           uint32_t key1)
        : k0(key0), k1(key1)
    {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            a[i] = c0[i];
            b[i] = c1;
            c[i] = c2[i];
            d[i] = 0u;
        }
    }

    // one round of all N blocks, then the Weyl key bump
    __device__ __forceinline__ void round()
    {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const uint64_t pa = (uint64_t)a[i] * 0xD2511F53u;
            const uint64_t pb = (uint64_t)c[i] * 0xCD9E8D57u;
            const uint32_t n0 = xor3((uint32_t)(pb >> 32), b[i], k0);
            const uint32_t n2 = xor3((uint32_t)(pa >> 32), d[i], k1);
            b[i] = (uint32_t)pb;
            d[i] = (uint32_t)pa;
            a[i] = n0;
            c[i] = n2;
        }
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }

    __device__ __forceinline__ PhiloxBlock block(int i) const
    {
        PhiloxBlock w;
        w.w[0] = a[i]; w.w[1] = b[i]; w.w[2] = c[i]; w.w[3] = d[i];
        return w;
    }
};

// All ten rounds of N blocks in lockstep; the scheduling barrier after each round keeps
// the compiler from serialising the blocks, so their multiply/xor chains interleave.
template <int N>
__device__ __forceinline__ void philox4x32_10_n(const uint32_t* c0, uint32_t c1, const uint32_t* c2, uint32_t k0,
                                                uint32_t k1, PhiloxBlock* out)
{
    PhiloxLanes<N> ph(c0, c1, c2, k0, k1);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        ph.round();
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = ph.block(i);
}

template <typename T>
struct BoxMuller;

// FP64 natural log of u in (0, 1]: u = m 2^e with m in [sqrt(1/2), sqrt(2)), and
// ln m = 2 atanh(f), f = (m - 1) / (m + 1), |f| <= 0.1716, from the series
// 2 (f + f^3/3 + ... + f^23/23) (truncation below 1e-18); ln 2 split in two parts.
// Within 1 ulp of the correctly rounded log over the uniforms Box-Muller uses.
__device__ __forceinline__ double log_unit(double u)
{
    int e;
    double m = frexp(u, &e);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double f2 = f * f;
    double p = 1.0 / 23.0;
    p = fma(p, f2, 1.0 / 21.0);
    p = fma(p, f2, 1.0 / 19.0);
    p = fma(p, f2, 1.0 / 17.0);
    p = fma(p, f2, 1.0 / 15.0);
    p = fma(p, f2, 1.0 / 13.0);
    p = fma(p, f2, 1.0 / 11.0);
    p = fma(p, f2, 1.0 / 9.0);
    p = fma(p, f2, 1.0 / 7.0);
    p = fma(p, f2, 1.0 / 5.0);
    p = fma(p, f2, 1.0 / 3.0);
    const double lm = fma(2.0 * f * f2, p, 2.0 * f);
    const double ln2_hi = 0x1.62e42fefa39efp-1, ln2_lo = 0x1.abc9e3b39803fp-56;
    return fma((double)e, ln2_hi, fma((double)e, ln2_lo, lm));
}

// sin(pi x), cos(pi x) for x in [0, 2]: x = n/2 + r with n = rint(2x), |r| <= 1/4 (the
// subtraction is exact), Taylor series of sin and cos of y = pi r to degree 17 / 18
// (truncation below 1e-16 of y), then the quarter-turn n mod 4.  Absolute error within
// 4e-16.
__device__ __forceinline__ void sincospi_turn(double x, double& s, double& c)
{
    const double n = rint(2.0 * x);
    const double r = fma(-0.5, n, x);
    const double y = r * 3.14159265358979323846;
    const double y2 = y * y;
    double ps = -1.0 / 355687428096000.0;   // -1/17!
    ps = fma(ps, y2, 1.0 / 1307674368000.0);
    ps = fma(ps, y2, -1.0 / 6227020800.0);
    ps = fma(ps, y2, 1.0 / 39916800.0);
    ps = fma(ps, y2, -1.0 / 362880.0);
    ps = fma(ps, y2, 1.0 / 5040.0);
    ps = fma(ps, y2, -1.0 / 120.0);
    ps = fma(ps, y2, 1.0 / 6.0);
    const double sy = fma(-y * y2, ps, y);
    double pc = 1.0 / 6402373705728000.0;   // 1/18!
    pc = fma(pc, y2, -1.0 / 20922789888000.0);
    pc = fma(pc, y2, 1.0 / 87178291200.0);
    pc = fma(pc, y2, -1.0 / 479001600.0);
    pc = fma(pc, y2, 1.0 / 3628800.0);
    pc = fma(pc, y2, -1.0 / 40320.0);
    pc = fma(pc, y2, 1.0 / 720.0);
    pc = fma(pc, y2, -1.0 / 24.0);
    pc = fma(pc, y2, 0.5);
    const double cy = fma(-y2, pc, 1.0);
    const int q = (int)n & 3;
    s = q == 0 ? sy : (q == 1 ? cy : (q == 2 ? -sy : -cy));
    c = q == 0 ? cy : (q == 1 ? -sy : (q == 2 ? -cy : sy));
}

// FP64: the log and sin/cos above, the correctly rounded sqrt.
template <>
struct BoxMuller<double> {
    // (sc r cos, sc r sin) of the pair (x0, x1)
    __device__ __forceinline__ static void pair(uint32_t x0, uint32_t x1, double sc, double& a, double& b)
    {
        const double u0 = ((double)x0 + 0.5) * 0x1p-32;
        const double u1 = ((double)x1 + 0.5) * 0x1p-32;
        const double r = sc * sqrt(-2.0 * log_unit(u0));
        double s, c;
        sincospi_turn(2.0 * u1, s, c);
        a = r * c;
        b = r * s;
    }
};

// FP32: the hardware transcendentals.  v_log_f32 is log2, so -2 ln u = -2 ln(2) log2 u;
// v_sin_f32 / v_cos_f32 take their argument in turns, so sin(2 pi u) = v_sin_f32(u).
template <>
struct BoxMuller<float> {
    __device__ __forceinline__ static void pair(uint32_t x0, uint32_t x1, float sc, float& a, float& b)
    {
        // (x + 1/2) 2^-32 with one rounding of x to 24 bits: relative error ~2^-24
        const float u0 = fmaf((float)x0, 0x1p-32f, 0x1p-33f);
        const float u1 = fmaf((float)x1, 0x1p-32f, 0x1p-33f);
        const float r = sc * __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));
        a = r * __builtin_amdgcn_cosf(u1);
        b = r * __builtin_amdgcn_sinf(u1);
    }
};

}  // namespace smf
