// Alg. 2's last step on rings that each carry their own pixel count n_i and first-pixel
// longitude phi0_i (iso-latitude grids such as HEALPix, which Sec. 1 names):
//   T(z_i, phi0_i + 2 pi j / n_i) = sum_{|m| <= m_top} c_m e^{2 pi i m j / n_i},
//   c_m = g_m e^{i m phi0_i},  c_{-m} = conj(c_m),
// every mode kept.  Folding the modes onto the ring's n_i frequencies (B_k = sum of c_m
// over m = k mod n_i) turns the sum into one complex-to-real inverse DFT of length n_i,
// which runs as a complex inverse DFT of length h = n_i / 2 (the split of the ring C2R),
// Stockham passes in LDS: a pass for each odd prime factor of h (the largest first; direct,
// or for a large prime P Bluestein's chirp-z form, the length-P DFT as a convolution done by
// power-of-two FFTs), then radix-4 and radix-2 butterflies.
#include "device_path.h"

namespace smf {
namespace {

struct RingArgs {
    int n_theta;
    int m_top;
    int g_row;        // complex values per ring in the mode buffer (n_phi / 2)
    int64_t total;    // pixels of one field
    const int* list;  // rings of this launch (blockIdx.x indexes it)
};

constexpr int kRingThreads = 256;

template <typename T>
__device__ __forceinline__ Cx<T> conj_c(Cx<T> a) { return {a.re, -a.im}; }

// q = x / d and r = x - q d for 0 <= x < 2^24, 0 < d, x / d < 2^22, from a float product with the
// reciprocal (off by at most one, which the remainder's range check corrects).
struct FastDiv {
    int d;
    float inv;
};
__device__ __forceinline__ FastDiv fast_div(int d) { return {d, 1.0f / (float)d}; }
__device__ __forceinline__ int fdiv(int x, FastDiv f, int& r)
{
    int q = (int)((float)x * f.inv);
    r = x - q * f.d;
    if (r < 0) {
        --q;
        r += f.d;
    } else if (r >= f.d) {
        ++q;
        r -= f.d;
    }
    return q;
}

// Re-anchoring interval of the twiddle recurrence of the direct passes.
constexpr int kRingAnchor = 16;
// Bins per thread whose first-period modes are loaded ahead of the table work.
constexpr int kRingPre = 8;

// e^{+2 pi i k / n} for 0 <= k < n: Ft[k / 64] * Et[k mod 64] (two roundings of the type).
template <typename T>
__device__ __forceinline__ Cx<T> ring_tw(const Cx<T>* Et, const Cx<T>* Ft, int k)
{
    return cmul(Ft[k >> 6], Et[k & 63]);
}

// In-place FFTs of a power-of-two length L in LDS for the chirp-z pass, radix-4 stages (spans
// L/4, L/16, ...) and, when log2 L is odd, a last radix-2 stage on neighbouring pairs.  The
// forward one (e^{-2 pi i}) runs the stages by decimation in frequency and leaves the
// digit-reversed order; the inverse (e^{+2 pi i}, unscaled) undoes them in reverse order and
// returns natural order, so a product taken between the two needs no permutation.
// Twiddles e^{2 pi i k / L} = FL[k / 64] EL[k mod 64]; each stage ends with a barrier.
template <typename T>
__device__ void lds_fft_fwd(Cx<T>* x, int L, const Cx<T>* EL, const Cx<T>* FL, int tid)
{
    for (int Q = L >> 2; Q >= 1; Q >>= 2) {
        const int stride = L / (4 * Q);
        for (int t = tid; t < (L >> 2); t += kRingThreads) {
            const int gi = t / Q;
            const int pos = t - gi * Q;
            const int base = gi * 4 * Q + pos;
            const Cx<T> v0 = x[base], v1 = x[base + Q], v2 = x[base + 2 * Q], v3 = x[base + 3 * Q];
            const Cx<T> s02 = cadd(v0, v2), d02 = csub(v0, v2), s13 = cadd(v1, v3);
            const Cx<T> id13 = mul_i(csub(v1, v3));
            const Cx<T> w1 = ring_tw(EL, FL, pos * stride);
            const Cx<T> w2 = cmul(w1, w1);
            const Cx<T> w3 = cmul(w1, w2);
            x[base] = cadd(s02, s13);
            x[base + Q] = cmul(csub(d02, id13), Cx<T>{w1.re, -w1.im});
            x[base + 2 * Q] = cmul(csub(s02, s13), Cx<T>{w2.re, -w2.im});
            x[base + 3 * Q] = cmul(cadd(d02, id13), Cx<T>{w3.re, -w3.im});
        }
        __syncthreads();
    }
    if (__builtin_ctz(L) & 1) {
        for (int t = tid; t < (L >> 1); t += kRingThreads) {
            const Cx<T> u = x[2 * t], v = x[2 * t + 1];
            x[2 * t] = cadd(u, v);
            x[2 * t + 1] = csub(u, v);
        }
        __syncthreads();
    }
}

template <typename T>
__device__ void lds_fft_inv(Cx<T>* x, int L, const Cx<T>* EL, const Cx<T>* FL, int tid)
{
    const bool odd = __builtin_ctz(L) & 1;
    if (odd) {
        for (int t = tid; t < (L >> 1); t += kRingThreads) {
            const Cx<T> u = x[2 * t], v = x[2 * t + 1];
            x[2 * t] = cadd(u, v);
            x[2 * t + 1] = csub(u, v);
        }
        __syncthreads();
    }
    for (int Q = odd ? 2 : 1; Q <= (L >> 2); Q <<= 2) {
        const int stride = L / (4 * Q);
        for (int t = tid; t < (L >> 2); t += kRingThreads) {
            const int gi = t / Q;
            const int pos = t - gi * Q;
            const int base = gi * 4 * Q + pos;
            const Cx<T> w1 = ring_tw(EL, FL, pos * stride);
            const Cx<T> w2 = cmul(w1, w1);
            const Cx<T> w3 = cmul(w1, w2);
            const Cx<T> v0 = x[base], v1 = cmul(x[base + Q], w1), v2 = cmul(x[base + 2 * Q], w2),
                        v3 = cmul(x[base + 3 * Q], w3);
            const Cx<T> s02 = cadd(v0, v2), d02 = csub(v0, v2), s13 = cadd(v1, v3);
            const Cx<T> id13 = mul_i(csub(v1, v3));
            x[base] = cadd(s02, s13);
            x[base + Q] = cadd(d02, id13);
            x[base + 2 * Q] = csub(s02, s13);
            x[base + 3 * Q] = csub(d02, id13);
        }
        __syncthreads();
    }
}

// One workgroup per (ring, field): blockIdx.x picks the ring from the launch's list,
// blockIdx.y is the field.  LDS holds two buffers of h + 1 complex values and small tables of
// the ring's twiddles and phases; with BLUE (the rings whose largest odd prime P takes the
// chirp-z pass) also two convolution buffers of L >= 2P - 1 values and the tables of their
// twiddles.
template <typename T, bool BLUE>
__global__ __launch_bounds__(kRingThreads) void ring_c2r_kernel(RingArgs a, const T* __restrict__ g,
                                                                const int* __restrict__ n_ring,
                                                                const double* __restrict__ phi0,
                                                                const int64_t* __restrict__ off,
                                                                T* __restrict__ out, Epilogue<T> ep)
{
    extern __shared__ unsigned char smem_raw[];
    const int i = a.list[blockIdx.x];
    const int f = blockIdx.y;
    const int n = n_ring[i];
    const int h = n >> 1;
    const int tid = threadIdx.x;
    const int mt = a.m_top;
    Cx<T>* buf0 = reinterpret_cast<Cx<T>*>(smem_raw);
    Cx<T>* buf1 = buf0 + (h + 1);
    // small tables from FP64 sincos, rounded to the type: Et_b = e^{2 pi i b / n},
    // Ft_a = e^{2 pi i 64 a / n} (twiddles Ft Et), Gt_b = e^{i b phi0}, Ht_a = e^{i 64 a phi0}
    // (b < 64; a mode's phase is Ht Gt); laid out in an FP64-sized region E, F, G, H
    Cx<double>* E = reinterpret_cast<Cx<double>*>(buf1 + (h + 1));
    const int na = n / 64 + 1;
    const int ma = mt / 64 + 1;
    Cx<double>* F = E + 64;
    Cx<double>* G = F + na;
    Cx<double>* H = G + 64;
    Cx<T>* Et = reinterpret_cast<Cx<T>*>(H + ma);
    Cx<T>* Ft = Et + 64;
    Cx<T>* part = Ft + na;   // partial sums of the fold, kRingThreads values
    Cx<T>* Gt = reinterpret_cast<Cx<T>*>(G);
    Cx<T>* Ht = Gt + 64;
    const double p0 = phi0[i];
    const bool phased = p0 != 0.0;   // uniform: rings starting at longitude 0 need no phases

    // the modes of the first period of this thread's first kRingPre bins (m = k and m = n - k),
    // loaded before the tables are built so that their latency overlaps that work
    using V2 = typename Vec2<T>::type;
    const T* gr = g + ((size_t)f * a.n_theta + i) * (size_t)a.g_row * 2;
    const V2* gv = reinterpret_cast<const V2*>(gr);
    const int nb = h + 1;
    const int gs = nb >= kRingThreads ? 1 : kRingThreads / nb;
    V2 pre_p[kRingPre], pre_n[kRingPre];
    if (gs == 1) {
#pragma unroll
        for (int r = 0; r < kRingPre; ++r) {
            const int k = tid + r * kRingThreads;
            const int mn = k == 0 ? n : n - k;
            pre_p[r] = (k < nb && k <= mt) ? gv[k] : V2{T(0), T(0)};
            pre_n[r] = (k < nb && mn <= mt) ? gv[mn] : V2{T(0), T(0)};
        }
    }

    for (int k = tid; k < (phased ? 128 + na + ma : 64 + na); k += kRingThreads) {
        double s, c;
        if (k < 64)
            sincospi(2.0 * (double)k / (double)n, &s, &c);
        else if (k < 64 + na)
            sincospi(128.0 * (double)(k - 64) / (double)n, &s, &c);
        else if (k < 128 + na)
            sincos((double)(k - 64 - na) * p0, &s, &c);
        else
            sincos((double)(64 * (k - 128 - na)) * p0, &s, &c);
        if (k < 64 + na)
            Et[k] = {(T)c, (T)s};
        else
            Gt[k - 64 - na] = {(T)c, (T)s};   // Gt then Ht
    }
    __syncthreads();

    // fold: B_k = sum_{m = k mod n} c_m + sum_{m = -k mod n, m >= 1} conj(c_m),  k <= h.
    // A ring with at most kRingThreads / 2 bins gives each bin `gs` threads, which sum every
    // gs-th period of its modes; the partial sums are added in a fixed order.
    // c_m = g_m e^{i m phi0}
    auto cph = [&](int m, V2 x) {
        const Cx<T> v = {x.x, x.y};
        return phased ? cmul(v, cmul(Ht[m >> 6], Gt[m & 63])) : v;
    };
    const V2 zero2 = {T(0), T(0)};
    auto fold_bin = [&](int k, int g0) {
        Cx<T> acc = {T(0), T(0)};
#pragma unroll 4
        for (int m = k + g0 * n; m <= mt; m += gs * n) acc = cadd(acc, cph(m, gv[m]));
#pragma unroll 4
        for (int m = (k == 0 ? n : n - k) + g0 * n; m <= mt; m += gs * n) acc = cadd(acc, conj_c(cph(m, gv[m])));
        return acc;
    };
    if (gs == 1) {
        // bins from the prefetched first period, then the further periods (modes above n), one
        // period at a time over this thread's bins so that a period's loads are in flight together
        Cx<T> acc[kRingPre];
#pragma unroll
        for (int r = 0; r < kRingPre; ++r) {
            const int k = tid + r * kRingThreads;
            const int mn = k == 0 ? n : n - k;
            acc[r] = {T(0), T(0)};
            if (k < nb && k <= mt) acc[r] = cph(k, pre_p[r]);
            if (k < nb && mn <= mt) acc[r] = cadd(acc[r], conj_c(cph(mn, pre_n[r])));
        }
        for (int p = 1; p * n <= mt; ++p) {
#pragma unroll
            for (int r = 0; r < kRingPre; ++r) {
                const int k = tid + r * kRingThreads;
                const int m1 = k + p * n, m2 = (k == 0 ? n : n - k) + p * n;
                const V2 x1 = (k < nb && m1 <= mt) ? gv[m1] : zero2;
                const V2 x2 = (k < nb && m2 <= mt) ? gv[m2] : zero2;
                if (k < nb && m1 <= mt) acc[r] = cadd(acc[r], cph(m1, x1));
                if (k < nb && m2 <= mt) acc[r] = cadd(acc[r], conj_c(cph(m2, x2)));
            }
        }
#pragma unroll
        for (int r = 0; r < kRingPre; ++r) {
            const int k = tid + r * kRingThreads;
            if (k < nb) buf1[k] = acc[r];
        }
        for (int k = tid + kRingPre * kRingThreads; k < nb; k += kRingThreads) buf1[k] = fold_bin(k, 0);
    } else {
        if (tid < nb * gs) part[tid] = fold_bin(tid % nb, tid / nb);
        __syncthreads();
        if (tid < nb) {
            Cx<T> acc = part[tid];
            for (int q = 1; q < gs; ++q) acc = cadd(acc, part[q * nb + tid]);
            buf1[tid] = acc;
        }
    }
    __syncthreads();

    // split: Z_k = (B_k + conj B_{h-k}) + i w^k (B_k - conj B_{h-k}),  k < h
    for (int k = tid; k < h; k += kRingThreads) {
        const Cx<T> x = buf1[k], y = buf1[h - k];
        const Cx<T> yc = {y.re, -y.im};
        const Cx<T> d = cmul(ring_tw(Et, Ft, k), csub(x, yc));
        buf0[k] = cadd(cadd(x, yc), mul_i(d));
    }
    __syncthreads();

    // inverse DFT of length h, Stockham: after a pass of radix R the data hold
    // sub-transforms of length Ns * R in natural order
    Cx<T>* src = buf0;
    Cx<T>* dst = buf1;
    int Ns = 1;
    int rem = h;
    while ((rem & 1) == 0) rem >>= 1;
    int p = 3;
    if (rem > 1) {
        // the largest odd prime factor P first: with Ns = 1 the twiddles of inputs t and
        // P - t are conjugate, so each pair costs one twiddle and four multiply-adds
        int big = 3, r = rem;
        while (r > 1) {
            if (p * p > r) p = r;
            if (r % p) {
                p += 2;
                continue;
            }
            big = p;
            r /= p;
        }
        const int P = big;
        const int step = n / P;
        const int hp = h / P;
        const int half = (P + 1) / 2;
        if (BLUE) {
            // chirp-z: with c_k = e^{i pi k^2 / P} (= e^{2 pi i ((k^2 mod 2P) hp) / n}),
            // X_q = c_q sum_t (x_t c_t) conj(c_{q-t}), a cyclic convolution of length
            // L >= 2P - 1 with the spectrum of conj(c) computed once per ring
            int L = 1;
            while (L < 2 * P - 1) L <<= 1;
            Cx<T>* wa = part + kRingThreads;
            Cx<T>* wd = wa + L;
            Cx<T>* EL = wd + L;
            Cx<T>* FL = EL + 64;
            for (int k = tid; k < 64 + L / 64 + 1; k += kRingThreads) {
                double sn, cs;
                sincospi((k < 64 ? 2.0 * (double)k : 128.0 * (double)(k - 64)) / (double)L, &sn, &cs);
                EL[k] = {(T)cs, (T)sn};
            }
            auto chirp = [&](int k) { return ring_tw(Et, Ft, (int)(((long)k * k) % (2 * P)) * hp); };
            for (int k = tid; k < L; k += kRingThreads) {
                Cx<T> v = {T(0), T(0)};
                if (k < P)
                    v = chirp(k);
                else if (k > L - P)
                    v = chirp(L - k);
                wd[k] = {v.re, -v.im};
            }
            __syncthreads();
            lds_fft_fwd(wd, L, EL, FL, tid);
            const T inv = T(1) / (T)L;
            for (int b = 0; b < hp; ++b) {
                for (int k = tid; k < L; k += kRingThreads)
                    wa[k] = k < P ? cmul(src[b + k * hp], chirp(k)) : Cx<T>{T(0), T(0)};
                __syncthreads();
                lds_fft_fwd(wa, L, EL, FL, tid);
                for (int k = tid; k < L; k += kRingThreads) wa[k] = cmul(wa[k], wd[k]);
                __syncthreads();
                lds_fft_inv(wa, L, EL, FL, tid);
                for (int q = tid; q < P; q += kRingThreads) {
                    const Cx<T> r = cmul(wa[q], chirp(q));
                    dst[b * P + q] = {r.re * inv, r.im * inv};
                }
                __syncthreads();
            }
        } else {
            // outputs q and P - q have conjugate twiddles too: one thread makes both
            const FastDiv fh = fast_div(half), fp = fast_div(P);
            for (int idx = tid; idx < hp * half; idx += kRingThreads) {
                int q;
                const int b = fdiv(idx, fh, q);
                const Cx<T> w1 = ring_tw(Et, Ft, q * step);
                Cx<T> acc = src[b];
                Cx<T> acc2 = acc;
                Cx<T> W = w1;
                for (int t = 1; 2 * t < P; ++t) {
                    if (t % kRingAnchor == 0) {
                        int tq;
                        (void)fdiv(t * q, fp, tq);
                        W = ring_tw(Et, Ft, tq * step);
                    } else if (t > 1) {
                        W = cmul(W, w1);
                    }
                    const Cx<T> x = src[b + t * hp], y = src[b + (P - t) * hp];
                    const Cx<T> sp = cadd(x, y), df = csub(x, y);
                    acc.re += sp.re * W.re - df.im * W.im;
                    acc.im += sp.im * W.re + df.re * W.im;
                    acc2.re += sp.re * W.re + df.im * W.im;
                    acc2.im += sp.im * W.re - df.re * W.im;
                }
                dst[b * P + q] = acc;
                if (q > 0) dst[b * P + P - q] = acc2;
            }
        }
        __syncthreads();
        Cx<T>* tmp = src;
        src = dst;
        dst = tmp;
        Ns = P;
        rem /= P;
        p = 3;
    }
    while (rem > 1) {
        if (p * p > rem) p = rem;
        if (rem % p) {
            p += 2;
            continue;
        }
        // direct pass of odd radix p: output u of each sub-transform sums its p inputs with
        // twiddles W_t = e^{2 pi i t u / (Ns p)}, stepped by W_t = W_{t-1} W_1 and taken from
        // the tables every kRingAnchor terms
        const int NsR = Ns * p;
        const int step = n / NsR;
        const int hp = h / p;
        const FastDiv fr = fast_div(NsR), fs = fast_div(Ns);
        for (int idx = tid; idx < h; idx += kRingThreads) {
            int u, us;
            const int b = fdiv(idx, fr, u);
            (void)fdiv(u, fs, us);
            const int j = b * Ns + us;
            const Cx<T> w1 = ring_tw(Et, Ft, u * step);
            Cx<T> acc = src[j];
            Cx<T> W = w1;
            for (int t = 1; t < p; ++t) {
                if (t % kRingAnchor == 0) {
                    int tu;
                    (void)fdiv(t * u, fr, tu);
                    W = ring_tw(Et, Ft, tu * step);
                } else if (t > 1) {
                    W = cmul(W, w1);
                }
                acc = cadd(acc, cmul(src[j + t * hp], W));
            }
            dst[idx] = acc;
        }
        __syncthreads();
        Cx<T>* tmp = src;
        src = dst;
        dst = tmp;
        Ns = NsR;
        rem /= p;
    }
    while (h / Ns >= 4) {
        const int q = h >> 2;
        const int step = n / (4 * Ns);
        const FastDiv fs = fast_div(Ns);
        for (int j = tid; j < q; j += kRingThreads) {
            int kq;
            const int jb = fdiv(j, fs, kq);
            // one table twiddle per butterfly; its square and cube by complex multiplies
            const Cx<T> w1 = ring_tw(Et, Ft, kq * step);
            const Cx<T> w2 = cmul(w1, w1);
            Cx<T> v[4];
            v[0] = src[j];
            v[1] = cmul(src[j + q], w1);
            v[2] = cmul(src[j + 2 * q], w2);
            v[3] = cmul(src[j + 3 * q], cmul(w1, w2));
            dft_inv<T, 4>(v);
            const int base = jb * 4 * Ns + kq;
#pragma unroll
            for (int t = 0; t < 4; ++t) dst[base + t * Ns] = v[t];
        }
        __syncthreads();
        Cx<T>* tmp = src;
        src = dst;
        dst = tmp;
        Ns *= 4;
    }
    if (h / Ns == 2) {
        const int q = h >> 1;
        const int step = n / (2 * Ns);
        const FastDiv fs = fast_div(Ns);
        for (int j = tid; j < q; j += kRingThreads) {
            int kq;
            const int jb = fdiv(j, fs, kq);
            Cx<T> v[2] = {src[j], cmul(src[j + q], ring_tw(Et, Ft, kq * step))};
            dft_inv<T, 2>(v);
            const int base = jb * 2 * Ns + kq;
            dst[base] = v[0];
            dst[base + Ns] = v[1];
        }
        __syncthreads();
        src = dst;
    }

    // T_{2j} = Re z_j, T_{2j+1} = Im z_j (through the lognormal map when it is on)
    V2* o = reinterpret_cast<V2*>(out + (size_t)f * a.total + off[i]);
    for (int j = tid; j < h; j += kRingThreads) {
        const Cx<T> v = epilogue(ep, src[j]);
        V2 w;
        w.x = v.re;
        w.y = v.im;
        o[j] = w;
    }
}

template <typename T, bool BLUE>
hipError_t launch_ring_c2r_t(const RingArgs& a, int rings, int count, size_t lds, const T* g, const int* n_ring,
                             const double* phi0, const int64_t* off, T* out, const Epilogue<T>& ep, hipStream_t st)
{
    if (rings == 0) return hipSuccess;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)ring_c2r_kernel<T, BLUE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((ring_c2r_kernel<T, BLUE>), dim3(rings, count), dim3(kRingThreads), lds, st, a, g, n_ring,
                       phi0, off, out, ep);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ring_pair(const RingArgs& a, const RingSplit& rs, int count, const T* g, const int* n_ring,
                            const double* phi0, const int64_t* off, T* out, const LognormalMap* ln, hipStream_t st)
{
    const bool fp64 = sizeof(T) == 8;
    const Epilogue<T> ep = {ln ? (T)ln->mu : T(0), ln ? (T)ln->sigma : T(0), ln ? 1 : 0};
    RingArgs ab = a;
    ab.list = a.list + rs.n_direct;
    hipError_t e = launch_ring_c2r_t<T, false>(a, rs.n_direct, count, ring_lds_bytes(rs.n_max_direct, a.m_top, fp64),
                                               g, n_ring, phi0, off, out, ep, st);
    if (e != hipSuccess) return e;
    return launch_ring_c2r_t<T, true>(ab, rs.n_chirp, count,
                                      ring_lds_bytes(rs.n_max_chirp, a.m_top, fp64, rs.l_max), g, n_ring, phi0, off,
                                      out, ep, st);
}

}  // namespace

size_t ring_lds_bytes(int n_max, int m_top, bool fp64, int l_max)
{
    const size_t cx = fp64 ? 16 : 8;
    const size_t small = 128 + (size_t)(n_max / 64 + 1) + (size_t)(m_top / 64 + 1);
    size_t b = cx * ((size_t)2 * (n_max / 2 + 1) + 64 + (size_t)(n_max / 64 + 1) + kRingThreads) + 16 * small;
    if (l_max > 0) b += cx * ((size_t)2 * l_max + 64 + (size_t)(l_max / 64 + 1));
    return b;
}

int ring_largest_odd_prime(int h)
{
    int r = h;
    while (r > 0 && (r & 1) == 0) r >>= 1;
    int big = 1, p = 3;
    while (r > 1) {
        if (p * p > r) p = r;
        if (r % p) {
            p += 2;
            continue;
        }
        big = p;
        r /= p;
    }
    return big;
}

hipError_t launch_ring_c2r(int n_theta, int m_top, int g_row, int64_t total, const RingSplit& rs, bool fp64,
                           int count, const void* g, const int* list, const int* n_ring, const double* phi0,
                           const int64_t* off, void* out, const LognormalMap* ln, hipStream_t st)
{
    if (count <= 0 || count > 65535 || n_theta <= 0 || rs.n_direct + rs.n_chirp > n_theta) return hipErrorInvalidValue;
    const RingArgs a = {n_theta, m_top, g_row, total, list};
    if (fp64)
        return launch_ring_pair<double>(a, rs, count, (const double*)g, n_ring, phi0, off, (double*)out, ln, st);
    return launch_ring_pair<float>(a, rs, count, (const float*)g, n_ring, phi0, off, (float*)out, ln, st);
}

}  // namespace smf
