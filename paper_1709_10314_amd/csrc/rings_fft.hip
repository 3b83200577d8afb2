// Two more transform classes of the ring synthesis (the sum T(z_i, phi0_i + 2 pi j / n_i) of
// Alg. 2's last step on rings that carry their own pixel count n_i), for rings whose
// half-length h = n_i / 2 is large:
//   - h a power of two L (1024 <= L <= 4096): the complex inverse DFT of length h as radix-16,
//     radix-16 and radix-L/256 Stockham passes, the data in registers except between passes;
//   - h with a large odd prime factor: the whole length-h DFT by Bluestein's chirp-z identity
//     k q = (k^2 + q^2 - (q - k)^2) / 2, i.e. z_q = e^{i pi q^2 / h} sum_k (Z_k e^{i pi k^2 / h})
//     e^{-i pi (q - k)^2 / h}, a cyclic convolution of length L >= 2h - 1 done by two
//     power-of-two transforms of length L (the same passes) and a product with the transform
//     of the chirp; that transform, the chirp and the chirp times the split's twiddle depend
//     on h only and are computed once, at setup, in FP64.
// Folding the modes onto the ring's frequencies and the real-to-complex split are those of the
// general ring kernel (rings.hip); here each thread folds the bins of its transform inputs, and
// the split's mirror partners come through LDS.
#include <algorithm>

#include "device_path.h"
#include "smf_internal.h"

namespace smf {
namespace {

// Consecutive work items kept on one XCD (two rings of one length in eight fields)
constexpr int kXcdChunk = 16;

struct RingFftArgs {
    int n_theta;
    int m_top;
    int g_row;          // complex values per ring in the mode buffer
    int64_t total;      // pixels of one field
    const int* list;    // rings of this launch
    int rings;          // entries of list
    int count;          // fields
};

// First element of the twiddle table of length L = 2^LOG2L: e^{2 pi i t / (2L)}, t < 2L,
// tables for L = 2^kRingFftMinLog2 .. 2^kRingFftMaxLog2 stored one after the other.
__host__ __device__ constexpr int ring_tw_base(int log2l)
{
    return 2 * ((1 << log2l) - (1 << kRingFftMinLog2));
}

template <typename T>
__device__ __forceinline__ Cx<T> conj_c(Cx<T> a) { return {a.re, -a.im}; }

// ---- register-resident radix-16 form (L = 256 R3, R3 = 4, 8, 16; NT = L / 16 threads) ----
// Thread t holds x_{t + NT r} (r < 16) in registers: pass 1 (radix 16, Ns = 1) takes them
// straight from the split, pass 2 (radix 16, Ns = 16) goes through LDS, pass 3 (radix R3,
// Ns = 256) reads LDS and leaves the results z_{t + NT r} in registers, which is again the
// input layout of pass 1: the two transforms of the Bluestein form meet in registers.

// Passes 1 and 2; the data are in LDS after pass 2 (a barrier at the end).
template <typename T, int LOG2L>
__device__ __forceinline__ void r16_pass12(Cx<T>* buf, const Cx<T>* __restrict__ tw, int t, Cx<T> (&v)[16])
{
    constexpr int L = 1 << LOG2L;
    constexpr int NT = L / 16;
    // pass 1 (Ns = 1): no twiddles; outputs 16 t + q
    dft_inv16<T>(v);
#pragma unroll
    for (int q = 0; q < 16; ++q) buf[lds_slot(16 * t + q)] = v[q];
    __syncthreads();
    // pass 2 (Ns = 16): k = t mod 16, twiddles e^{2 pi i k r / 256} = tw[k r L / 128]; outputs
    // (t - k) 16 + k + 16 q
    const int k = t & 15;
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = buf[lds_slot(t + NT * r)];
    __syncthreads();
    twiddle16<T>(v, tw, k * (L / 128));
    dft_inv16<T>(v);
    const int o = (t - k) * 16 + k;
#pragma unroll
    for (int q = 0; q < 16; ++q) buf[lds_slot(o + 16 * q)] = v[q];
    __syncthreads();
}

// Pass 3: radix R3 over butterflies b = t + NT j (j < 256 / NT), inputs x_{b + 256 r},
// twiddles e^{2 pi i b r / L} = tw[2 b r]; outputs z_{b + 256 q} = z_{t + NT (j + (256 / NT) q)}
// to v[j + (256 / NT) q].  The caller must barrier before the buffer is written again.
template <typename T, int LOG2L>
__device__ __forceinline__ void r16_pass3(const Cx<T>* buf, const Cx<T>* __restrict__ tw, int t, Cx<T> (&v)[16])
{
    constexpr int L = 1 << LOG2L;
    constexpr int NT = L / 16;
    constexpr int R3 = L / 256;
    constexpr int PER = 256 / NT;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int b = t + NT * j;
        Cx<T> u[R3];
#pragma unroll
        for (int r = 0; r < R3; ++r) u[r] = buf[lds_slot(b + 256 * r)];
        if constexpr (R3 == 16) {
            twiddle16<T>(u, tw, 2 * b);
            dft_inv16<T>(u);
        } else {
            Cx<T> w[R3];
            butterfly_twiddles<T, R3>(tw, 2 * b, w);
#pragma unroll
            for (int r = 1; r < R3; ++r) u[r] = cmul(u[r], w[r]);
            dft_inv<T, R3>(u);
        }
#pragma unroll
        for (int q = 0; q < R3; ++q) v[j + PER * q] = u[q];
    }
}

// One workgroup of L / 16 threads per (ring, field); blockIdx.x picks the ring from the
// launch's list, blockIdx.y is the field.  BLUE: the Bluestein form (h <= L / 2); otherwise
// h = L.  Thread t folds bins k = t + NT r with the phase e^{i k phi0} factored out:
// B_k = e^{i k phi0} (U_k + conj X_k), U_k = sum_p g_{k+pn} E^p, X_k = sum_p g_{n-k+pn} E^{p+1},
// E = e^{i n phi0}, and e^{i k phi0} = e^{i (t mod 16) phi0} e^{i 16 (t / 16) phi0} e^{i NT r phi0},
// three table values (FP64 sincos, rounded to the type once) multiplied in the type.  LDS: the
// buffer, the phase tables (16 values each, then E and e^{i h phi0}) and B_h.  The Bluestein form
// reads its length's block of the plan's table: S (L values), then c_k = e^{i pi k^2 / h} and
// D_k = i e^{2 pi i k / n} c_k (L / 2 values each, k < h used).
// Waves per SIMD the radix-16 ring kernels are compiled for (their register budget; 0: the
// compiler's choice)
#ifndef SMF_RING_R16_WAVES
#define SMF_RING_R16_WAVES 0
#endif
// 1: the radix-16 ring kernels also load the modes n - k ahead of the tables (FP32)
#ifndef SMF_RING_PRE_NEG
#define SMF_RING_PRE_NEG 1
#endif
#if SMF_RING_R16_WAVES > 0
#define SMF_R16_ATTR __attribute__((amdgpu_waves_per_eu(SMF_RING_R16_WAVES)))
#else
#define SMF_R16_ATTR
#endif

// The Bluestein form keeps the chirp of its bins in registers for the outputs (FP32, L = 4096:
// measured faster, within 128 VGPRs) or reloads it after the second transform (measured faster
// at the shorter lengths, whose transforms then get more registers)
template <typename T, int LOG2L, bool BLUE>
__host__ __device__ constexpr bool r16_keeps_chirp()
{
    return BLUE && sizeof(T) == 4 && LOG2L == 12;
}

template <typename T, int LOG2L, bool BLUE>
__global__ __launch_bounds__((1 << LOG2L) / 16, (r16_keeps_chirp<T, LOG2L, BLUE>() ? 4 : 1)) SMF_R16_ATTR void ring_r16_kernel(RingFftArgs a, const T* __restrict__ g,
                                                                     const int* __restrict__ n_ring,
                                                                     const double* __restrict__ phi0,
                                                                     const int64_t* __restrict__ off,
                                                                     const Cx<T>* __restrict__ tw_all,
                                                                     const Cx<T>* __restrict__ spec,
                                                                     const int64_t* __restrict__ spec_off,
                                                                     T* __restrict__ out, Epilogue<T> ep)
{
    constexpr int L = 1 << LOG2L;
    constexpr int NT = L / 16;
    constexpr int RB = BLUE ? 8 : 16;        // bins per thread (Bluestein: k < h <= L / 2)
    constexpr bool PRE = sizeof(T) == 4;     // first-period modes loaded ahead of the tables
    extern __shared__ unsigned char smem_raw[];
    // work item w = (list position) * count + field.  Workgroup b runs on XCD b mod 8; the
    // items are dealt to the XCDs in chunks of kXcdChunk consecutive items, chunk c to XCD c mod 8,
    // so that the workgroups of one ring length (next to each other in the list, every field)
    // share their XCD's L2 for the Bluestein kernel's transform while the XCDs get equal shares
    // of the list.  Blocks past the last item return before any barrier.
    const int n_items = a.rings * a.count;
    const int slot = (int)(blockIdx.x >> 3);
    const int w = ((slot / kXcdChunk) * 8 + (int)(blockIdx.x & 7)) * kXcdChunk + slot % kXcdChunk;
    if (w >= n_items) return;
    const int i = a.list[w / a.count];
    const int f = w - (w / a.count) * a.count;
    const int n = n_ring[i];
    const int h = n >> 1;
    const int t = threadIdx.x;
    const int mt = a.m_top;
    const Cx<T>* tw = tw_all + ring_tw_base(LOG2L);
    Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
    Cx<T>* Ph = buf + lds_slots(L);   // [0, 16): e^{i b phi0}; [16, 32): e^{i 16 b phi0};
                                      // [32, 48): e^{i NT b phi0}; 48: E; 49: e^{i h phi0}
    Cx<T>* Bh = Ph + 50;
    const double p0 = phi0[i];
    using V2 = typename Vec2<T>::type;
    const V2* gv = reinterpret_cast<const V2*>(g + ((size_t)f * a.n_theta + i) * (size_t)a.g_row * 2);
    const V2 zero2 = {T(0), T(0)};
    auto mode = [&](int m) {
        const V2 x = gv[m];
        return Cx<T>{x.x, x.y};
    };

    V2 xa[PRE ? RB : 1], xb[PRE && SMF_RING_PRE_NEG ? RB : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int k = t + NT * r;
            const int mk = k == 0 ? n : n - k;
            xa[r] = (k < h && k <= mt) ? gv[k] : zero2;
            if constexpr (SMF_RING_PRE_NEG) xb[r] = (k < h && mk <= mt) ? gv[mk] : zero2;
        }
    }
    const bool phased = p0 != 0.0;   // uniform: rings starting at longitude 0 need no phases
    if (phased && t < 50) {
        double sn, cs;
        const int a = t & 15, sel = t >> 4;
        const double m = sel == 0 ? a : sel == 1 ? 16.0 * a : sel == 2 ? (double)NT * a : t == 48 ? n : h;
        sincos(m * p0, &sn, &cs);
        Ph[t] = {(T)cs, (T)sn};
    }
    __syncthreads();
    const Cx<T> one = {T(1), T(0)};
    const Cx<T> En = phased ? Ph[48] : one;
    const Cx<T> base = phased ? cmul(Ph[t & 15], Ph[16 + (t >> 4)]) : one;   // e^{i t phi0}
    const Cx<T>* S = spec + (BLUE ? spec_off[i] : 0);   // S, then c (at L), then D (at 3 L / 2)

    // fold, one period of the modes at a time over all of this thread's bins (so that a
    // period's loads are in flight together): Y_k = U_k + conj X_k, then B_k = e^{i k phi0} Y_k,
    // written to LDS for the mirror partners of the split; thread 0 also sums the Nyquist bin h,
    // U_h = sum_p g_{h+pn} E^p, B_h = e^{i h phi0} (U_h + conj(E U_h))
    Cx<T> v[16];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int k = t + NT * r;
        const int mk = k == 0 ? n : n - k;
        Cx<T> u, x;
        if constexpr (PRE) {
            u = {xa[r].x, xa[r].y};
            if constexpr (SMF_RING_PRE_NEG)
                x = {xb[r].x, xb[r].y};
            else
                x = (k < h && mk <= mt) ? mode(mk) : Cx<T>{T(0), T(0)};
        } else {
            u = (k < h && k <= mt) ? mode(k) : Cx<T>{T(0), T(0)};
            x = (k < h && mk <= mt) ? mode(mk) : Cx<T>{T(0), T(0)};
        }
        v[r] = cadd(u, conj_c(cmul(x, En)));
    }
    // the Bluestein tables of this thread's bins, loaded while the fold goes on (zero from h on);
    // c_k is also the chirp of output q = k
    constexpr bool KEEP_C = r16_keeps_chirp<T, LOG2L, BLUE>();
    Cx<T> cc[BLUE ? RB : 1], dd[BLUE ? RB : 1];
    if constexpr (BLUE) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            cc[r] = S[L + t + NT * r];
            dd[r] = S[L + L / 2 + t + NT * r];
        }
    }
    Cx<T> uh = (t == 0 && h <= mt) ? mode(h) : Cx<T>{T(0), T(0)};
    Cx<T> Ep = En, Eq = cmul(En, En);   // E^p, E^{p+1}
    for (int p = 1; p * n <= mt; ++p) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int k = t + NT * r;
            const int m1 = k + p * n, m2 = (k == 0 ? n : n - k) + p * n;
            Cx<T> u = {T(0), T(0)}, x = {T(0), T(0)};
            if (k < h && m1 <= mt) u = mode(m1);
            if (k < h && m2 <= mt) x = mode(m2);
            v[r] = cadd(v[r], cadd(cmul(u, Ep), conj_c(cmul(x, Eq))));
        }
        if (t == 0 && h + p * n <= mt) uh = cadd(uh, cmul(mode(h + p * n), Ep));
        Ep = Eq;
        Eq = cmul(Eq, En);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int k = t + NT * r;
        if (k < h) {
            if (phased) v[r] = cmul(cmul(base, Ph[32 + r]), v[r]);
            buf[lds_slot(k)] = v[r];
        }
    }
    if (t == 0) Bh[0] = cmul(phased ? Ph[49] : one, cadd(uh, conj_c(cmul(uh, En))));
    __syncthreads();
    // split: Z_k = (B_k + conj B_{h-k}) + i w^k (B_k - conj B_{h-k}), w = e^{2 pi i / n}; the
    // Bluestein form takes Z_k c_k = (B_k + conj B_{h-k}) c_k + (B_k - conj B_{h-k}) D_k
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int k = t + NT * r;
        Cx<T> z = {T(0), T(0)};
        if (k < h) {
            const Cx<T> b1 = v[r];
            const Cx<T> b2 = conj_c(k == 0 ? Bh[0] : buf[lds_slot(h - k)]);
            if constexpr (BLUE)
                z = cadd(cmul(cadd(b1, b2), cc[r]), cmul(csub(b1, b2), dd[r]));
            else
                z = cadd(cadd(b1, b2), mul_i(cmul(tw[k], csub(b1, b2))));
        }
        v[r] = z;
    }
#pragma unroll
    for (int r = RB; r < 16; ++r) v[r] = {T(0), T(0)};
    __syncthreads();   // every partner read before pass 1 writes the buffer
    r16_pass12<T, LOG2L>(buf, tw, t, v);
    r16_pass3<T, LOG2L>(buf, tw, t, v);

    V2* o = reinterpret_cast<V2*>(out + (size_t)f * a.total + off[i]);
    if constexpr (!BLUE) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const Cx<T> x = epilogue(ep, v[r]);
            V2 w;
            w.x = x.re;
            w.y = x.im;
            o[t + NT * r] = w;
        }
    } else {
        // the product with the chirp's transform S (divided by L), then the forward transform
        // as conj(inverse(conj(.))), z_q = c_q (the convolution at q) for q < h
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = conj_c(cmul(v[r], S[t + NT * r]));
        __syncthreads();   // pass 3's reads before pass 1 writes the buffer
        r16_pass12<T, LOG2L>(buf, tw, t, v);
        r16_pass3<T, LOG2L>(buf, tw, t, v);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int q = t + NT * r;
            if (q < h) {
                const Cx<T> x = epilogue(ep, cmul(conj_c(v[r]), KEEP_C ? cc[r] : S[L + q]));
                V2 w;
                w.x = x.re;
                w.y = x.im;
                o[q] = w;
            }
        }
    }
}

// The transform tables of a ring plan: tw[base(l) + t] = e^{2 pi i t / 2^(l+1)}, t < 2^(l+1),
// for l = kRingFftMinLog2 .. kRingFftMaxLog2, from FP64 sincospi, in FP64 and rounded to FP32.
__global__ void ring_tw_kernel(double* __restrict__ tw64, float* __restrict__ tw32)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ring_tw_base(kRingFftMaxLog2 + 1)) return;
    int l = kRingFftMinLog2;
    while (t >= ring_tw_base(l + 1)) ++l;
    const int k = t - ring_tw_base(l);
    double s, c;
    sincospi((double)k / (double)(1 << l), &s, &c);
    tw64[2 * t] = c;
    tw64[2 * t + 1] = s;
    if (tw32) {
        tw32[2 * t] = (float)c;
        tw32[2 * t + 1] = (float)s;
    }
}

// S = inverse DFT_L(b) / L of Bluestein's kernel b_j = e^{-i pi j^2 / h} (j < h), b_{L-j} = b_j
// (0 < j < h), zero elsewhere, then the chirp c_j = e^{i pi j^2 / h} and D_j = i e^{i pi j / h} c_j
// (j < L / 2; zero from h on); one workgroup per listed length h, in FP64, stored in the plan's
// type at out + off[w] (2 L complex values).
template <typename T, int LOG2L>
__global__ __launch_bounds__((1 << LOG2L) / 8) void ring_spectrum_kernel(const int* __restrict__ hs,
                                                                         const int64_t* __restrict__ offs,
                                                                         const Cx<double>* __restrict__ tw_all,
                                                                         T* __restrict__ out)
{
    constexpr int L = 1 << LOG2L;
    constexpr int NT = L / 8;
    extern __shared__ unsigned char smem_raw[];
    Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem_raw);
    const int h = hs[blockIdx.x];
    const int64_t n = 2 * (int64_t)h;
    for (int j = threadIdx.x; j < L; j += NT) {
        Cx<double> v = {0.0, 0.0};
        const int jj = j < h ? j : (j > L - h ? L - j : -1);
        if (jj >= 0) {
            double s, c;
            sincospi(-(double)(((int64_t)jj * jj) % n) / (double)h, &s, &c);
            v = {c, s};
        }
        buf[lds_slot(j)] = v;
    }
    __syncthreads();
    run_passes<double, LOG2L, NT, 0>(buf, tw_all + ring_tw_base(LOG2L));
    Cx<T>* o = reinterpret_cast<Cx<T>*>(out) + offs[blockIdx.x];
    const double inv = 1.0 / (double)L;
    for (int j = threadIdx.x; j < L; j += NT) {
        const Cx<double> v = buf[lds_slot(j)];
        o[j] = {(T)(v.re * inv), (T)(v.im * inv)};
    }
    // the phases reduced modulo n = 2 h exactly in integers before the FP64 sincospi
    for (int j = threadIdx.x; j < L / 2; j += NT) {
        Cx<T> c = {T(0), T(0)}, d = {T(0), T(0)};
        if (j < h) {
            double s, co;
            sincospi((double)(((int64_t)j * j) % n) / (double)h, &s, &co);
            c = {(T)co, (T)s};
            sincospi((double)(((int64_t)j * j + j) % n) / (double)h, &s, &co);
            d = {(T)(-s), (T)co};
        }
        o[L + j] = c;
        o[L + L / 2 + j] = d;
    }
}

// LDS of ring_r16_kernel
size_t r16_kernel_lds(int log2l, bool fp64)
{
    const size_t cx = fp64 ? 16 : 8;
    return cx * ((size_t)lds_slots(1 << log2l) + 50 + 2);
}

template <typename T, int LOG2L, bool BLUE>
hipError_t launch_fft_t(const RingFftArgs& a, int rings, int count, const T* g, const int* n_ring,
                        const double* phi0, const int64_t* off, const void* tw, const void* spec,
                        const int64_t* spec_off, T* out, const Epilogue<T>& ep, hipStream_t st)
{
    if (rings == 0) return hipSuccess;
    const size_t lds = r16_kernel_lds(LOG2L, sizeof(T) == 8);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)ring_r16_kernel<T, LOG2L, BLUE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    // fields in chunks whose work items (rings x fields) fit a 2^30-workgroup grid
    const int per_round = 8 * kXcdChunk;
    const int chunk = (int)std::min<int64_t>(count, ((int64_t)1 << 30) / rings);
    for (int f0 = 0; f0 < count; f0 += chunk) {
        RingFftArgs ab = a;
        ab.rings = rings;
        ab.count = std::min(chunk, count - f0);
        const int items = rings * ab.count;
        hipLaunchKernelGGL((ring_r16_kernel<T, LOG2L, BLUE>), dim3(((items + per_round - 1) / per_round) * per_round),
                           dim3((1 << LOG2L) / 16), lds, st, ab, g + (size_t)f0 * a.n_theta * a.g_row * 2, n_ring,
                           phi0, off, (const Cx<T>*)tw, (const Cx<T>*)spec, spec_off, out + (size_t)f0 * a.total, ep);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, bool BLUE>
hipError_t launch_fft_l(int log2l, const RingFftArgs& a, int rings, int count, const T* g, const int* n_ring,
                        const double* phi0, const int64_t* off, const void* tw, const void* spec,
                        const int64_t* spec_off, T* out, const Epilogue<T>& ep, hipStream_t st)
{
    switch (log2l) {
    case 10: return launch_fft_t<T, 10, BLUE>(a, rings, count, g, n_ring, phi0, off, tw, spec, spec_off, out, ep, st);
    case 11: return launch_fft_t<T, 11, BLUE>(a, rings, count, g, n_ring, phi0, off, tw, spec, spec_off, out, ep, st);
    case 12: return launch_fft_t<T, 12, BLUE>(a, rings, count, g, n_ring, phi0, off, tw, spec, spec_off, out, ep, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int LOG2L>
hipError_t launch_spectrum_t(int lengths, const int* hs, const int64_t* offs, const double* tw64, void* out,
                             hipStream_t st)
{
    if (lengths == 0) return hipSuccess;
    const size_t lds = sizeof(Cx<double>) * (size_t)lds_slots(1 << LOG2L);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)ring_spectrum_kernel<T, LOG2L>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((ring_spectrum_kernel<T, LOG2L>), dim3(lengths), dim3((1 << LOG2L) / 8), lds, st, hs, offs,
                       (const Cx<double>*)tw64, (T*)out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spectrum_l(int log2l, int lengths, const int* hs, const int64_t* offs, const double* tw64,
                             void* out, hipStream_t st)
{
    switch (log2l) {
    case 10: return launch_spectrum_t<T, 10>(lengths, hs, offs, tw64, out, st);
    case 11: return launch_spectrum_t<T, 11>(lengths, hs, offs, tw64, out, st);
    case 12: return launch_spectrum_t<T, 12>(lengths, hs, offs, tw64, out, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int ring_tw_entries() { return ring_tw_base(kRingFftMaxLog2 + 1); }

int ring_fft_count(const RingSplit& rs)
{
    int n = 0;
    for (int c = 0; c < kRingFftClasses; ++c) n += rs.n_blue[c] + rs.n_pow2[c];
    return n;
}

size_t ring_fft_lds_bytes(int log2l, int m_top, bool fp64)
{
    (void)m_top;
    return r16_kernel_lds(log2l, fp64);
}

hipError_t launch_ring_tw(double* tw64, float* tw32, hipStream_t st)
{
    const int n = ring_tw_entries();
    hipLaunchKernelGGL(ring_tw_kernel, dim3((n + 255) / 256), dim3(256), 0, st, tw64, tw32);
    return hipGetLastError();
}

hipError_t launch_ring_spectra(int log2l, int lengths, const int* hs_dev, const int64_t* offs_dev,
                               const double* tw64, bool fp64, void* out, hipStream_t st)
{
    if (log2l < kRingFftMinLog2 || log2l > kRingFftMaxLog2 || lengths < 0) return hipErrorInvalidValue;
    return fp64 ? launch_spectrum_l<double>(log2l, lengths, hs_dev, offs_dev, tw64, out, st)
                : launch_spectrum_l<float>(log2l, lengths, hs_dev, offs_dev, tw64, out, st);
}

hipError_t launch_ring_fft_class(bool blue, int log2l, int rings, int n_theta, int m_top, int g_row, int64_t total,
                                 bool fp64, int count, const void* g, const int* list, const int* n_ring,
                                 const double* phi0, const int64_t* off, const void* tw, const void* spec,
                                 const int64_t* spec_off, void* out, const LognormalMap* ln, hipStream_t st)
{
    if (count <= 0 || count > 65535 || rings < 0) return hipErrorInvalidValue;
    const RingFftArgs a = {n_theta, m_top, g_row, total, list, rings, count};
    if (fp64) {
        const Epilogue<double> ep = {ln ? ln->mu : 0.0, ln ? ln->sigma : 0.0, ln ? 1 : 0};
        return blue ? launch_fft_l<double, true>(log2l, a, rings, count, (const double*)g, n_ring, phi0, off, tw, spec,
                                                 spec_off, (double*)out, ep, st)
                    : launch_fft_l<double, false>(log2l, a, rings, count, (const double*)g, n_ring, phi0, off, tw,
                                                  spec, spec_off, (double*)out, ep, st);
    }
    const Epilogue<float> ep = {ln ? (float)ln->mu : 0.0f, ln ? (float)ln->sigma : 0.0f, ln ? 1 : 0};
    return blue ? launch_fft_l<float, true>(log2l, a, rings, count, (const float*)g, n_ring, phi0, off, tw, spec,
                                            spec_off, (float*)out, ep, st)
                : launch_fft_l<float, false>(log2l, a, rings, count, (const float*)g, n_ring, phi0, off, tw, spec,
                                             spec_off, (float*)out, ep, st);
}

}  // namespace smf
