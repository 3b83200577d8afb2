// Device bodies of the sampling path, shared by the per-plan kernels (sample.hip) and the
// batch kernels (batch.hip):
//   chain_start, walk_hemisphere, run_chain
//              -- the latitude-ring recursion of one (field, hemisphere, mode) for one part
//                 or both parts per lane, with fused Philox normals (Creasey & Lang,
//                 Alg. 2; eqs. (state_initial), (state_space); the mirror remark after
//                 Alg. 1); the affine scan walks ring blocks with the same pieces
//   run_chain_gen
//              -- the same recursion for Markov orders 3 and 4, one part per lane
//   c2r_row, c2r_rows
//              -- the complex-to-real inverse FFT of one ring / of many rings per
//                 workgroup, in place (Alg. 2, last step)
#pragma once

#include "rng.h"
#include "smf_internal.h"

namespace smf {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

// ------------------------------------------------------------------ recursion

// Four normals of one Philox block (counter (blk, m, part, 0)), each scaled by sc
// (1 for m = 0, 1/sqrt(2) for the Re/Im parts of m > 0).
template <typename T>
__device__ __forceinline__ void block_normals(uint32_t blk, uint32_t m, uint32_t part, uint32_t k0,
                                              uint32_t k1, T sc, T n[4])
{
    const PhiloxBlock w = philox4x32_10(blk, m, part, 0u, k0, k1);
    BoxMuller<T>::pair(w.w[0], w.w[1], sc, n[0], n[1]);
    BoxMuller<T>::pair(w.w[2], w.w[3], sc, n[2], n[3]);
}

// One state-space step x <- A x + B w (eq. (state_space)) with the factor record `rec`.
// The products are fused in a fixed order (explicit fma), so a step rounds the same way
// wherever it is inlined.
template <typename T, int M>
__device__ __forceinline__ void chain_step(const T* __restrict__ rec, T& x0, T& x1, T w0, T w1)
{
    if (M == 1) {
        using V2 = typename Vec2<T>::type;
        const V2 v = *reinterpret_cast<const V2*>(rec);
        x0 = fma(v.x, x0, v.y * w0);
    } else {
        const T a00 = rec[0], a01 = rec[1], a10 = rec[2], a11 = rec[3];
        const T b00 = rec[4], b10 = rec[5], b11 = rec[6];
        const T y0 = fma(a00, x0, fma(a01, x1, b00 * w0));
        const T y1 = fma(a10, x0, fma(a11, x1, fma(b10, w0, b11 * w1)));
        x0 = y0;
        x1 = y1;
    }
}

template <typename T>
__device__ __forceinline__ T pick4(const T n[4], int w)
{
    return w == 0 ? n[0] : (w == 1 ? n[1] : (w == 2 ? n[2] : n[3]));
}

// Factor record of one step, loaded ahead of use (register prefetch pipeline).
template <typename T, int M>
struct Rec {
    T v[M == 1 ? 2 : 7];
};

template <typename T, int M>
__device__ __forceinline__ Rec<T, M> load_rec(const T* __restrict__ rec)
{
    Rec<T, M> R;
    if constexpr (M == 1) {
        using V2 = typename Vec2<T>::type;
        const V2 v = *reinterpret_cast<const V2*>(rec);
        R.v[0] = v.x;
        R.v[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < 7; ++i) R.v[i] = rec[i];
    }
    return R;
}

// x <- A x + B w with a prefetched record (same fused order as chain_step)
template <typename T, int M>
__device__ __forceinline__ void chain_step_rec(const Rec<T, M>& R, T& x0, T& x1, T w0, T w1)
{
    if constexpr (M == 1) {
        x0 = fma(R.v[0], x0, R.v[1] * w0);
    } else {
        const T y0 = fma(R.v[0], x0, fma(R.v[1], x1, R.v[4] * w0));
        const T y1 = fma(R.v[2], x0, fma(R.v[3], x1, fma(R.v[5], w0, R.v[6] * w1)));
        x0 = y0;
        x1 = y1;
    }
}

// Philox groups kept in flight by the register prefetch pipeline of a chain walk, per
// precision and chains per lane.
#ifndef SMF_CHAIN_P32
#define SMF_CHAIN_P32 4
#endif
#ifndef SMF_CHAIN_P32_ONE
#define SMF_CHAIN_P32_ONE 8
#endif
#ifndef SMF_CHAIN_P64
#define SMF_CHAIN_P64 2
#endif
template <typename T, int NCH = 1>
struct ChainDepth {
    static constexpr int value = sizeof(T) == 4 ? (NCH == 2 ? SMF_CHAIN_P32 : SMF_CHAIN_P32_ONE) : SMF_CHAIN_P64;
};

// Rings are walked in groups of G = 4/M that share one Philox block (counter block
// (ring M) / 4).  Ring r uses set j = s - r + even walking north and j = r - s walking
// south; the southern noise is D w (second component negated).
//
// A lane runs NCH chains of one mode that share every factor record: NCH = 1 is the
// chain of one part (`up0`), NCH = 2 the Re and Im chains (parts 0 and 1), whose values
// are adjacent in the output and stored as one pair.  `sc[c]` scales chain c's normals
// (1 for m = 0, 1/sqrt(2) for the parts of m > 0, 0 for the imaginary part of m = 0,
// which keeps that chain exactly zero).
//
// A group that is cut by the start or the last ring is stepped with direct loads.  Full
// groups run through a register prefetch pipeline: the G records of full group q are
// loaded while group q - P is computed (slot q mod P, a compile-time index after
// unrolling by P), so the loads of P*G rings are in flight during a group's arithmetic.
// The unrolled body has no branches, which lets the compiler count outstanding loads
// exactly instead of draining them.  Prefetches past the walk are clamped to valid sets
// and never used.
template <typename T, int M, bool NORTH>
__device__ __forceinline__ int set_of_ring(int r, int s, int even, int n_sets)
{
    int j = NORTH ? s - r + even : r - s;
    return j < 0 ? 0 : (j >= n_sets ? n_sets - 1 : j);
}

// x0 of the NCH chains into ring slot `off` of g
template <typename T, int NCH>
__device__ __forceinline__ void store_ring(T* __restrict__ g, size_t off, const T (&x0)[NCH])
{
    if constexpr (NCH == 1) {
        g[off] = x0[0];
    } else {
        using V2 = typename Vec2<T>::type;
        V2 v;
        v.x = x0[0];
        v.y = x0[1];
        *reinterpret_cast<V2*>(g + off) = v;
    }
}

template <typename T, int M, bool NORTH, int NCH>
__device__ __forceinline__ void step_group_direct(int base, int lo, int hi, int s, int even, int n_sets,
                                                  uint32_t um, uint32_t up0, uint32_t k0, uint32_t k1,
                                                  const T (&sc)[NCH], const T* __restrict__ fm,
                                                  size_t set_stride, T* __restrict__ g, size_t row,
                                                  T (&x0)[NCH], T (&x1)[NCH], bool store)
{
    constexpr int G = 4 / M;
    T nb[NCH][4];
#pragma unroll
    for (int c = 0; c < NCH; ++c) block_normals<T>((uint32_t)((base * M) >> 2), um, up0 + c, k0, k1, sc[c], nb[c]);
#pragma unroll
    for (int tt = 0; tt < G; ++tt) {
        const int t = NORTH ? G - 1 - tt : tt;
        const int r = base + t;
        if (r >= lo && r <= hi) {
            const Rec<T, M> R = load_rec<T, M>(fm + (size_t)set_of_ring<T, M, NORTH>(r, s, even, n_sets) * set_stride);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const T w0 = nb[c][t * M];
                const T w1 = M == 2 ? (NORTH ? nb[c][t * M + 1] : -nb[c][t * M + 1]) : T(0);
                chain_step_rec<T, M>(R, x0[c], x1[c], w0, w1);
            }
            if (store) store_ring<T, NCH>(g, (size_t)r * row, x0);
        }
    }
}

// Walks rings r_first..r_last (north: descending, south: ascending), storing each ring's
// x0 unless STORE is false (then only the end state is wanted; a compile-time choice keeps
// the pipelined loop body free of branches).
template <typename T, int M, int P, bool NORTH, int NCH, bool STORE = true>
__device__ __forceinline__ void walk_hemisphere(int s, int even, int r_first, int r_last, int m, uint32_t up0,
                                                uint32_t k0, uint32_t k1, const T (&sc)[NCH],
                                                const T* __restrict__ fm, size_t set_stride, int n_sets,
                                                T* __restrict__ g, size_t row, T (&x0)[NCH], T (&x1)[NCH])
{
    constexpr bool store = STORE;
    constexpr int G = 4 / M;
    const uint32_t um = (uint32_t)m;
    if (NORTH ? r_first < r_last : r_first > r_last) return;
    // cut first group, then full groups q = 0..ng-1 with bases b0 - q G (north) or
    // b0 + q G (south), then a cut last group
    int b0, ng;
    if (NORTH) {
        int top = r_first;
        const int base = (top / G) * G;
        if (top != base + G - 1 || base < r_last) {
            step_group_direct<T, M, true, NCH>(base, base > r_last ? base : r_last, top, s, even, n_sets, um, up0,
                                               k0, k1, sc, fm, set_stride, g, row, x0, x1, store);
            top = base - 1;
        }
        ng = top + 1 - r_last >= G ? (top + 1 - r_last) / G : 0;
        b0 = top + 1 - G;
    } else {
        int lo = r_first;
        const int base = (lo / G) * G;
        if (lo != base || base + G - 1 > r_last) {
            step_group_direct<T, M, false, NCH>(base, lo, base + G - 1 < r_last ? base + G - 1 : r_last, s, even,
                                                n_sets, um, up0, k0, k1, sc, fm, set_stride, g, row, x0, x1, store);
            lo = base + G;
        }
        ng = r_last - lo + 1 >= G ? (r_last - lo + 1) / G : 0;
        b0 = lo;
    }
    if (ng > 0) {
        Rec<T, M> buf[P][G];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int base = NORTH ? b0 - p * G : b0 + p * G;
#pragma unroll
            for (int t = 0; t < G; ++t)
                buf[p][t] = load_rec<T, M>(fm + (size_t)set_of_ring<T, M, NORTH>(base + t, s, even, n_sets) * set_stride);
        }
        int q = 0;
        for (; q + P <= ng; q += P) {
            // the P x NCH Philox blocks of this stage in lockstep, then their normals
            uint32_t blk[P * NCH], prt[P * NCH];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int base = NORTH ? b0 - (q + p) * G : b0 + (q + p) * G;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    blk[p * NCH + c] = (uint32_t)((base * M) >> 2);
                    prt[p * NCH + c] = up0 + c;
                }
            }
            PhiloxBlock wb[P * NCH];
            philox4x32_10_n<P * NCH>(blk, um, prt, k0, k1, wb);
            T nbs[P][NCH][4];
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const PhiloxBlock& w = wb[p * NCH + c];
                    BoxMuller<T>::pair(w.w[0], w.w[1], sc[c], nbs[p][c][0], nbs[p][c][1]);
                    BoxMuller<T>::pair(w.w[2], w.w[3], sc[c], nbs[p][c][2], nbs[p][c][3]);
                }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int base = NORTH ? b0 - (q + p) * G : b0 + (q + p) * G;
#pragma unroll
                for (int tt = 0; tt < G; ++tt) {
                    const int t = NORTH ? G - 1 - tt : tt;
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        const T w0 = nbs[p][c][t * M];
                        const T w1 = M == 2 ? (NORTH ? nbs[p][c][t * M + 1] : -nbs[p][c][t * M + 1]) : T(0);
                        chain_step_rec<T, M>(buf[p][t], x0[c], x1[c], w0, w1);
                    }
                    if (store) store_ring<T, NCH>(g, (size_t)(base + t) * row, x0);
                }
                const int nbase = NORTH ? base - P * G : base + P * G;
#pragma unroll
                for (int t = 0; t < G; ++t)
                    buf[p][t] = load_rec<T, M>(fm + (size_t)set_of_ring<T, M, NORTH>(nbase + t, s, even, n_sets) * set_stride);
            }
        }
        // fewer than P full groups left: their records are already in the slots
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (q + p < ng) {
                const int base = NORTH ? b0 - (q + p) * G : b0 + (q + p) * G;
                T nb[NCH][4];
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    block_normals<T>((uint32_t)((base * M) >> 2), um, up0 + c, k0, k1, sc[c], nb[c]);
#pragma unroll
                for (int tt = 0; tt < G; ++tt) {
                    const int t = NORTH ? G - 1 - tt : tt;
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        const T w0 = nb[c][t * M];
                        const T w1 = M == 2 ? (NORTH ? nb[c][t * M + 1] : -nb[c][t * M + 1]) : T(0);
                        chain_step_rec<T, M>(buf[p][t], x0[c], x1[c], w0, w1);
                    }
                    if (store) store_ring<T, NCH>(g, (size_t)(base + t) * row, x0);
                }
            }
        }
    }
    // cut last group
    if (NORTH) {
        const int end = b0 - ng * G + G - 1;   // highest ring not yet produced
        if (end >= r_last) {
            const int base = (end / G) * G;
            step_group_direct<T, M, true, NCH>(base, r_last, end, s, even, n_sets, um, up0, k0, k1, sc, fm,
                                               set_stride, g, row, x0, x1, store);
        }
    } else {
        const int lo = b0 + ng * G;
        if (lo <= r_last)
            step_group_direct<T, M, false, NCH>(lo, lo, r_last, s, even, n_sets, um, up0, k0, k1, sc, fm,
                                                set_stride, g, row, x0, x1, store);
    }
}

// The state a hemisphere's main walk starts from: the start draw at ring s (eq.
// (state_initial)), stored there by the northern chain; for the southern chain also the
// crossing step to ring s+1 (even n_theta, set 1, stored), then the switch to y = D x.
// Every chain of a (mode, part) redraws the start from the same counters.
template <typename T, int M, int NCH>
__device__ __forceinline__ void chain_start(int s, int even, int h, uint32_t um, uint32_t up0, uint32_t k0,
                                            uint32_t k1, const T (&sc)[NCH], const T* __restrict__ fm,
                                            size_t set_stride, T* __restrict__ g, size_t row, bool store,
                                            T (&x0)[NCH], T (&x1)[NCH])
{
    const int w = (s * M) & 3;
    const int r = s + 1;
    const int wc = (r * M) & 3;
    const bool same_block = ((r * M) >> 2) == ((s * M) >> 2);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        T nz[4];
        block_normals<T>((uint32_t)((s * M) >> 2), um, up0 + c, k0, k1, sc[c], nz);
        const T w0 = pick4(nz, w);
        if (M == 1) {
            x0[c] = fm[1] * w0;
            x1[c] = T(0);
        } else {
            const T w1 = w == 0 ? nz[1] : nz[3];
            x0[c] = fm[4] * w0;
            x1[c] = fm[5] * w0 + fm[6] * w1;
        }
        if (h == 1 && even) {
            // crossing s -> s+1 with set 1, in the true coordinates
            T c0, c1 = T(0);
            if (same_block) {
                c0 = pick4(nz, wc);
                if (M == 2) c1 = wc == 0 ? nz[1] : nz[3];
            } else {
                T nc[4];
                block_normals<T>((uint32_t)((r * M) >> 2), um, up0 + c, k0, k1, sc[c], nc);
                c0 = pick4(nc, wc);
                if (M == 2) c1 = wc == 0 ? nc[1] : nc[3];
            }
            chain_step<T, M>(fm + set_stride, x0[c], x1[c], c0, c1);
        }
        if (h == 1) x1[c] = -x1[c];   // y = D x
    }
    if (store) {
        if (h == 0) store_ring<T, NCH>(g, (size_t)s * row, x0);
        else if (even) store_ring<T, NCH>(g, (size_t)r * row, x0);
    }
}

// Chain scales of a lane running NCH chains of mode m from part up0 (see above).
template <typename T, int NCH>
__device__ __forceinline__ void chain_scales(int m, uint32_t up0, T (&sc)[NCH])
{
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        sc[c] = m == 0 ? ((up0 + c) == 0 ? T(1) : T(0)) : T(0.70710678118654752440);
}

// The NCH chains of one lane.  `fm` points at the mode's record in factor set 0 (sets
// `set_stride` apart); `g` at the lane's slot of ring 0 of its field (rings `row` elements
// apart).  The northern chain (h = 0) draws the start state at ring s and steps to ring 0;
// the southern chain (h = 1) redraws the same start state (same counters), takes the
// crossing step (even n_theta) and steps to ring n-1 with the mirrored factors, carried
// as y = D x so that the stored northern records apply unchanged with D w as the noise.
// On a grid with no symmetry the southern walk reads its own records, stored mirrored the
// same way, `south_off` elements after the northern ones.  The ring order is uniform
// across the wave.
template <typename T, int M, int NCH = 1, int P = ChainDepth<T, NCH>::value>
__device__ __forceinline__ void run_chain(int n, int s, int even, int n_sets, int h, int m, int up0,
                                          uint32_t k0, uint32_t k1, const T* __restrict__ fm,
                                          size_t set_stride, T* __restrict__ g, size_t row, size_t south_off = 0)
{
    T sc[NCH], x0[NCH], x1[NCH];
    chain_scales<T, NCH>(m, (uint32_t)up0, sc);
    chain_start<T, M, NCH>(s, even, h, (uint32_t)m, (uint32_t)up0, k0, k1, sc, fm, set_stride, g, row, true, x0,
                           x1);
    if (h == 0)
        walk_hemisphere<T, M, P, true, NCH>(s, even, s - 1, 0, m, (uint32_t)up0, k0, k1, sc, fm, set_stride,
                                            n_sets, g, row, x0, x1);
    else
        walk_hemisphere<T, M, P, false, NCH>(s, even, even ? s + 2 : s + 1, n - 1, m, (uint32_t)up0, k0, k1, sc,
                                             fm + south_off, set_stride, n_sets, g, row, x0, x1);
}

// Zero NCH adjacent slots of one hemisphere (modes above m_top, the imaginary part of g_0).
template <typename T, int NCH = 1>
__device__ __forceinline__ void zero_chain(int n, int s, int h, T* __restrict__ g, size_t row)
{
    const int r_lo = h ? s + 1 : 0, r_hi = h ? n : s + 1;
    T z[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) z[c] = T(0);
    for (int r = r_lo; r < r_hi; ++r) store_ring<T, NCH>(g, (size_t)r * row, z);
}

// ------------------------------------------------------------------ orders 3 and 4
// The same recursion for a state of M = 3 or 4 components (value and z-derivatives up to
// M-1).  A lane runs NCH chains of one mode that share every record load: one part
// (NCH = 1, part `up0`) or both parts (NCH = 2, parts 0 and 1, stored as one pair), as in
// the order-1/2 walk.  Ring r uses the normals r M + q, q < M, of the counter map (block
// (r M + q) / 4, word (r M + q) mod 4), so G rings whose G M normals fill NB whole Philox
// blocks form a group: M = 3 -> 4 rings in 3 blocks, M = 4 -> 1 ring in 1 block.  Groups
// are aligned to multiples of G in the ring index; a walk starts and ends with cut groups
// whose rings outside the walk are skipped.
template <int M>
struct GenGroup {
    static constexpr int G = M % 4 == 0 ? 1 : (M % 2 == 0 ? 2 : 4);
    static constexpr int NB = G * M / 4;
};

// A factor record (A row-major, B's lower triangle by rows, b_index) loaded as 16-byte
// chunks: V values cover the M*M + M(M+1)/2 used ones.
template <typename T, int M>
struct RecGen {
    static constexpr int USED = M * M + M * (M + 1) / 2;
    static constexpr int CH = (USED * (int)sizeof(T) + 15) / 16;
    static constexpr int V = CH * 16 / (int)sizeof(T);
    T v[V];
};

template <typename T, int M>
__device__ __forceinline__ RecGen<T, M> load_rec_gen(const T* __restrict__ rec)
{
    RecGen<T, M> R;
    const uint4* __restrict__ p = reinterpret_cast<const uint4*>(rec);
#pragma unroll
    for (int c = 0; c < RecGen<T, M>::CH; ++c) *reinterpret_cast<uint4*>(&R.v[c * 16 / sizeof(T)]) = p[c];
    return R;
}

// x <- A x + B w, each component accumulated by explicit fma in a fixed order.
template <typename T, int M>
__device__ __forceinline__ void chain_step_gen(const RecGen<T, M>& R, T (&x)[M], const T (&w)[M])
{
    T y[M];
#pragma unroll
    for (int p = 0; p < M; ++p) {
        T acc = R.v[b_index<M>(p, p)] * w[p];
#pragma unroll
        for (int q = p - 1; q >= 0; --q) acc = fma(R.v[b_index<M>(p, q)], w[q], acc);
#pragma unroll
        for (int q = M - 1; q >= 0; --q) acc = fma(R.v[p * M + q], x[q], acc);
        y[p] = acc;
    }
#pragma unroll
    for (int p = 0; p < M; ++p) x[p] = y[p];
}

// The 4 NB normals of the group starting at ring `base` for each of the lane's chains
// (part up0 + c, scaled by sc[c]); the NCH * NB Philox blocks run in lockstep.
template <typename T, int M, int NCH>
__device__ __forceinline__ void group_normals(int base, uint32_t um, uint32_t up0, uint32_t k0, uint32_t k1,
                                              const T (&sc)[NCH], T (&nb)[NCH][4 * GenGroup<M>::NB])
{
    constexpr int NB = GenGroup<M>::NB;
    uint32_t blk[NCH * NB], prt[NCH * NB];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            blk[c * NB + k] = (uint32_t)((base * M) >> 2) + (uint32_t)k;
            prt[c * NB + k] = up0 + c;
        }
    PhiloxBlock wb[NCH * NB];
    philox4x32_10_n<NCH * NB>(blk, um, prt, k0, k1, wb);
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const PhiloxBlock& w = wb[c * NB + k];
            BoxMuller<T>::pair(w.w[0], w.w[1], sc[c], nb[c][4 * k], nb[c][4 * k + 1]);
            BoxMuller<T>::pair(w.w[2], w.w[3], sc[c], nb[c][4 * k + 2], nb[c][4 * k + 3]);
        }
}

// The M normals of ring base + t from a group's normals (t uniform, not a constant:
// selected, not indexed), the odd ones negated south of the start (D w).
template <typename T, int M, bool NORTH>
__device__ __forceinline__ void ring_normals(const T (&nb)[4 * GenGroup<M>::NB], int t, T (&w)[M])
{
#pragma unroll
    for (int q = 0; q < M; ++q) w[q] = T(0);
#pragma unroll
    for (int u = 0; u < GenGroup<M>::G; ++u)
        if (u == t) {
#pragma unroll
            for (int q = 0; q < M; ++q) w[q] = (!NORTH && (q & 1)) ? -nb[u * M + q] : nb[u * M + q];
        }
}

// The value component of the lane's chains into ring slot `off` (one pair for NCH = 2).
template <typename T, int M, int NCH>
__device__ __forceinline__ void store_gen(T* __restrict__ g, size_t off, const T (&x)[NCH][M])
{
    T v[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) v[c] = x[c][0];
    store_ring<T, NCH>(g, off, v);
}

// One ring of the lane's chains with the ring's record and its group's normals (t: the
// ring's compile-time position in the group).
template <typename T, int M, bool NORTH, int NCH>
__device__ __forceinline__ void step_ring_gen(const RecGen<T, M>& R, const T (&nb)[NCH][4 * GenGroup<M>::NB], int t,
                                              T (&x)[NCH][M])
{
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        T w[M];
#pragma unroll
        for (int q = 0; q < M; ++q) w[q] = (!NORTH && (q & 1)) ? -nb[c][t * M + q] : nb[c][t * M + q];
        chain_step_gen<T, M>(R, x[c], w);
    }
}

// Rings [lo, hi] of the group at `base`, in walk order.  The group's records are loaded
// before its Philox rounds, so their latency overlaps the rounds.  STORE = false walks
// without stores (only the end state is wanted).
template <typename T, int M, bool NORTH, bool STORE, int NCH>
__device__ __forceinline__ void step_group_gen(int base, int lo, int hi, int s, int even, int n_sets, uint32_t um,
                                               uint32_t up0, uint32_t k0, uint32_t k1, const T (&sc)[NCH],
                                               const T* __restrict__ fm, size_t set_stride, T* __restrict__ g,
                                               size_t row, T (&x)[NCH][M])
{
    constexpr int G = GenGroup<M>::G;
    RecGen<T, M> R[G];
#pragma unroll
    for (int t = 0; t < G; ++t)
        R[t] = load_rec_gen<T, M>(fm + (size_t)set_of_ring<T, M, NORTH>(base + t, s, even, n_sets) * set_stride);
    T nb[NCH][4 * GenGroup<M>::NB];
    group_normals<T, M, NCH>(base, um, up0, k0, k1, sc, nb);
#pragma unroll
    for (int tt = 0; tt < G; ++tt) {
        const int t = NORTH ? G - 1 - tt : tt;
        const int r = base + t;
        if (r >= lo && r <= hi) {
            step_ring_gen<T, M, NORTH, NCH>(R[t], nb, t, x);
            if constexpr (STORE) store_gen<T, M, NCH>(g, (size_t)r * row, x);
        }
    }
}

// Groups per stage of a general-order walk: the stage's Philox blocks run in lockstep and
// the records of the next stage's groups are in flight during its steps (0: each group
// loads its records just before its own Philox rounds).  Measured on MI355X at 4096 x 8192
// (FP32, 1 and 8 fields) and 1024 x 2048 (FP64, 16 fields).
#ifndef SMF_GEN_P3_32
#define SMF_GEN_P3_32 2
#endif
#ifndef SMF_GEN_P4_32
#define SMF_GEN_P4_32 1
#endif
#ifndef SMF_GEN_P3_64
#define SMF_GEN_P3_64 2
#endif
#ifndef SMF_GEN_P4_64
#define SMF_GEN_P4_64 2
#endif
#ifndef SMF_GEN_P3_TWO
#define SMF_GEN_P3_TWO 2
#endif
#ifndef SMF_GEN_P4_TWO
#define SMF_GEN_P4_TWO 1
#endif
template <typename T, int M, int NCH = 1>
struct GenDepth {
    static constexpr int value = NCH == 2 ? (M == 3 ? SMF_GEN_P3_TWO : SMF_GEN_P4_TWO)
                                 : sizeof(T) == 8 ? (M == 3 ? SMF_GEN_P3_64 : SMF_GEN_P4_64)
                                                  : (M == 3 ? SMF_GEN_P3_32 : SMF_GEN_P4_32);
};

// Walks rings r_first..r_last (north: descending, south: ascending) as walk_hemisphere does
// for orders 1 and 2: a cut first group stepped directly, full groups through a P-slot
// record pipeline (slot q mod P, refilled with group q + P after use), a cut last group.
template <typename T, int M, int P, bool NORTH, bool STORE, int NCH>
__device__ __forceinline__ void walk_gen(int s, int even, int r_first, int r_last, uint32_t um, uint32_t up0,
                                         uint32_t k0, uint32_t k1, const T (&sc)[NCH], const T* __restrict__ fm,
                                         size_t set_stride, int n_sets, T* __restrict__ g, size_t row,
                                         T (&x)[NCH][M])
{
    constexpr int G = GenGroup<M>::G, NB = GenGroup<M>::NB;
    if (NORTH ? r_first < r_last : r_first > r_last) return;
    int b0, ng;
    if (NORTH) {
        int top = r_first;
        const int base = (top / G) * G;
        if (top != base + G - 1 || base < r_last) {
            step_group_gen<T, M, true, STORE, NCH>(base, base > r_last ? base : r_last, top, s, even, n_sets, um, up0,
                                                   k0, k1, sc, fm, set_stride, g, row, x);
            top = base - 1;
        }
        ng = top + 1 - r_last >= G ? (top + 1 - r_last) / G : 0;
        b0 = top + 1 - G;
    } else {
        int lo = r_first;
        const int base = (lo / G) * G;
        if (lo != base || base + G - 1 > r_last) {
            step_group_gen<T, M, false, STORE, NCH>(base, lo, base + G - 1 < r_last ? base + G - 1 : r_last, s, even,
                                                    n_sets, um, up0, k0, k1, sc, fm, set_stride, g, row, x);
            lo = base + G;
        }
        ng = r_last - lo + 1 >= G ? (r_last - lo + 1) / G : 0;
        b0 = lo;
    }
    if (ng > 0) {
        RecGen<T, M> buf[P][G];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int base = NORTH ? b0 - p * G : b0 + p * G;
#pragma unroll
            for (int t = 0; t < G; ++t)
                buf[p][t] = load_rec_gen<T, M>(fm + (size_t)set_of_ring<T, M, NORTH>(base + t, s, even, n_sets) * set_stride);
        }
        int q = 0;
        for (; q + P <= ng; q += P) {
            uint32_t blk[P * NCH * NB], prt[P * NCH * NB];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int base = NORTH ? b0 - (q + p) * G : b0 + (q + p) * G;
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        blk[(p * NCH + c) * NB + k] = (uint32_t)((base * M) >> 2) + (uint32_t)k;
                        prt[(p * NCH + c) * NB + k] = up0 + c;
                    }
            }
            PhiloxBlock wb[P * NCH * NB];
            philox4x32_10_n<P * NCH * NB>(blk, um, prt, k0, k1, wb);
            T nbs[P][NCH][4 * NB];
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        const PhiloxBlock& w = wb[(p * NCH + c) * NB + k];
                        BoxMuller<T>::pair(w.w[0], w.w[1], sc[c], nbs[p][c][4 * k], nbs[p][c][4 * k + 1]);
                        BoxMuller<T>::pair(w.w[2], w.w[3], sc[c], nbs[p][c][4 * k + 2], nbs[p][c][4 * k + 3]);
                    }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int base = NORTH ? b0 - (q + p) * G : b0 + (q + p) * G;
#pragma unroll
                for (int tt = 0; tt < G; ++tt) {
                    const int t = NORTH ? G - 1 - tt : tt;
                    step_ring_gen<T, M, NORTH, NCH>(buf[p][t], nbs[p], t, x);
                    if constexpr (STORE) store_gen<T, M, NCH>(g, (size_t)(base + t) * row, x);
                }
                const int nbase = NORTH ? base - P * G : base + P * G;
#pragma unroll
                for (int t = 0; t < G; ++t)
                    buf[p][t] = load_rec_gen<T, M>(fm + (size_t)set_of_ring<T, M, NORTH>(nbase + t, s, even, n_sets) *
                                                            set_stride);
            }
        }
        // fewer than P full groups left: their records are already in the slots
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (q + p < ng) {
                const int base = NORTH ? b0 - (q + p) * G : b0 + (q + p) * G;
                T nb[NCH][4 * NB];
                group_normals<T, M, NCH>(base, um, up0, k0, k1, sc, nb);
#pragma unroll
                for (int tt = 0; tt < G; ++tt) {
                    const int t = NORTH ? G - 1 - tt : tt;
                    step_ring_gen<T, M, NORTH, NCH>(buf[p][t], nb, t, x);
                    if constexpr (STORE) store_gen<T, M, NCH>(g, (size_t)(base + t) * row, x);
                }
            }
        }
    }
    if (NORTH) {
        const int end = b0 - ng * G + G - 1;   // highest ring not yet produced
        if (end >= r_last) {
            const int base = (end / G) * G;
            step_group_gen<T, M, true, STORE, NCH>(base, r_last, end, s, even, n_sets, um, up0, k0, k1, sc, fm,
                                                   set_stride, g, row, x);
        }
    } else {
        const int lo = b0 + ng * G;
        if (lo <= r_last)
            step_group_gen<T, M, false, STORE, NCH>(lo, lo, r_last, s, even, n_sets, um, up0, k0, k1, sc, fm,
                                                    set_stride, g, row, x);
    }
}

// The state the walk of an order M >= 3 chain starts from (as chain_start): the start draw
// at ring s with set 0 (eq. (state_initial); A = 0), stored by the northern chain; for the
// southern chain the crossing s -> s+1 (even n_theta, set 1, stored), then y = D x.
template <typename T, int M, int NCH>
__device__ __forceinline__ void chain_start_gen(int s, int even, int h, uint32_t um, uint32_t up0, uint32_t k0,
                                                uint32_t k1, const T (&sc)[NCH], const T* __restrict__ fm,
                                                size_t set_stride, T* __restrict__ g, size_t row, bool store,
                                                T (&x)[NCH][M])
{
    constexpr int G = GenGroup<M>::G;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int p = 0; p < M; ++p) x[c][p] = T(0);
    {
        const int bs = (s / G) * G;
        T nb[NCH][4 * GenGroup<M>::NB];
        group_normals<T, M, NCH>(bs, um, up0, k0, k1, sc, nb);
        const RecGen<T, M> R = load_rec_gen<T, M>(fm);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            T w[M];
            ring_normals<T, M, true>(nb[c], s - bs, w);
            chain_step_gen<T, M>(R, x[c], w);
        }
        if (store && h == 0) store_gen<T, M, NCH>(g, (size_t)s * row, x);
    }
    if (h == 1 && even) {
        const int r = s + 1;
        const int br = (r / G) * G;
        T nb[NCH][4 * GenGroup<M>::NB];
        group_normals<T, M, NCH>(br, um, up0, k0, k1, sc, nb);
        const RecGen<T, M> R = load_rec_gen<T, M>(fm + set_stride);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            T w[M];
            ring_normals<T, M, true>(nb[c], r - br, w);
            chain_step_gen<T, M>(R, x[c], w);
        }
        if (store) store_gen<T, M, NCH>(g, (size_t)r * row, x);
    }
    if (h == 1) {
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int p = 1; p < M; p += 2) x[c][p] = -x[c][p];   // y = D x
    }
}

// The NCH chains of one lane at order M >= 3 (layout and hemisphere roles as run_chain):
// the start draw at ring s, for the south the crossing step (even n_theta) and the switch
// to y = D x, then the walk to ring 0 or n-1.
template <typename T, int M, int NCH = 1>
__device__ __forceinline__ void run_chain_gen(int n, int s, int even, int n_sets, int h, int m, int up0, uint32_t k0,
                                              uint32_t k1, const T* __restrict__ fm, size_t set_stride,
                                              T* __restrict__ g, size_t row, size_t south_off = 0)
{
    constexpr int G = GenGroup<M>::G;
    const uint32_t um = (uint32_t)m, up = (uint32_t)up0;
    T sc[NCH];
    chain_scales<T, NCH>(m, up, sc);
    T x[NCH][M];
    chain_start_gen<T, M, NCH>(s, even, h, um, up, k0, k1, sc, fm, set_stride, g, row, true, x);
    constexpr int P = GenDepth<T, M, NCH>::value;
    if (h == 0) {
        if constexpr (P == 0) {
            for (int top = s - 1; top >= 0;) {
                const int base = (top / G) * G;
                step_group_gen<T, M, true, true, NCH>(base, base, top, s, even, n_sets, um, up, k0, k1, sc, fm,
                                                      set_stride, g, row, x);
                top = base - 1;
            }
        } else {
            walk_gen<T, M, P, true, true, NCH>(s, even, s - 1, 0, um, up, k0, k1, sc, fm, set_stride, n_sets, g, row,
                                               x);
        }
    } else {
        if constexpr (P == 0) {
            for (int lo = even ? s + 2 : s + 1; lo <= n - 1;) {
                const int base = (lo / G) * G;
                const int hi = base + G - 1 < n - 1 ? base + G - 1 : n - 1;
                step_group_gen<T, M, false, true, NCH>(base, lo, hi, s, even, n_sets, um, up, k0, k1, sc,
                                                       fm + south_off, set_stride, g, row, x);
                lo = base + G;
            }
        } else {
            walk_gen<T, M, P, false, true, NCH>(s, even, even ? s + 2 : s + 1, n - 1, um, up, k0, k1, sc,
                                                fm + south_off, set_stride, n_sets, g, row, x);
        }
    }
}

// ------------------------------------------------------------------ C2R FFT
// Per ring: X_m = g_m (m <= m_top, else 0; X_0 taken real; X_{N-m} = conj X_m), N = n_phi,
// H = N/2.
//   T_j = sum_m X_m e^{2 pi i m j / N}
// via one complex inverse FFT of length H: with w = e^{2 pi i / N},
//   Z_k = (X_k + conj X_{H-k}) + i w^k (X_k - conj X_{H-k}),  k < H  (X_H = 0),
//   z_j = sum_k Z_k e^{2 pi i k j / H},   T_{2j} = Re z_j,  T_{2j+1} = Im z_j.
// The ring is read from and written back to the same memory (the modes were stored in
// place by the recursion), staged through LDS; Stockham radix-8/4/2 passes, each pass
// reading all its inputs before a barrier and writing after it.

template <typename T>
struct Cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> mul_i(Cx<T> a) { return {-a.im, a.re}; }   // i a

// In-register inverse DFT of size R (kernel e^{+2 pi i r q / R}).
template <typename T, int R>
__device__ __forceinline__ void dft_inv(Cx<T>* v)
{
    if (R == 2) {
        const Cx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 4) {
        const Cx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const Cx<T> s13 = cadd(v[1], v[3]), d13 = mul_i(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else {   // R == 8: radix-2 over two size-4 DFTs of the even and odd samples
        Cx<T> e[4] = {v[0], v[2], v[4], v[6]};
        Cx<T> o[4] = {v[1], v[3], v[5], v[7]};
        dft_inv<T, 4>(e);
        dft_inv<T, 4>(o);
        const T h = T(0.70710678118654752440);
        const Cx<T> o1 = {h * (o[1].re - o[1].im), h * (o[1].re + o[1].im)};   // (1+i)/sqrt2
        const Cx<T> o2 = mul_i(o[2]);                                            // i
        const Cx<T> o3 = {-h * (o[3].re + o[3].im), h * (o[3].re - o[3].im)};   // (-1+i)/sqrt2
        v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
    }
}

// LDS slot of element i: one pad slot after every 16 elements, so that the strided
// Stockham writes (stride Ns R elements per thread) spread over the banks.
__device__ __forceinline__ int lds_slot(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_slots(int h) { return h + (h >> 4); }

// Twiddles w^r, r = 1..R-1, of one butterfly: w = tw[t] and w^4 = tw[4t] from the table
// (t < N/4 whenever R = 8, since k < Ns <= H/8), the rest by at most two products.
template <typename T, int R>
__device__ __forceinline__ void butterfly_twiddles(const Cx<T>* __restrict__ tw, int t, Cx<T>* w)
{
    w[1] = tw[t];
    if (R >= 4) {
        w[2] = cmul(w[1], w[1]);
        w[3] = cmul(w[2], w[1]);
    }
    if (R == 8) {
        w[4] = tw[4 * t];
        w[5] = cmul(w[4], w[1]);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
    }
}

// One Stockham pass of radix R over H points held in LDS buffer `buf`, current
// sub-transform length Ns = 2^LOG2NS.  Butterfly b: k = b mod Ns; inputs b + r H/R
// times e^{2 pi i k r / (Ns R)}; outputs to ((b / Ns) Ns R + k) + q Ns.  Twiddles come
// from the table tw[t] = e^{2 pi i t / N}, N = 2H.
template <typename T, int LOG2H, int R, int NT, int LOG2NS>
__device__ __forceinline__ void stockham_pass(Cx<T>* buf, const Cx<T>* __restrict__ tw)
{
    constexpr int Ns = 1 << LOG2NS;
    constexpr int H = 1 << LOG2H;
    constexpr int NB = H / R;
    constexpr int PER = (NB + NT - 1) / NT;
    Cx<T> v[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if (NB % NT == 0 || b < NB) {
            const int k = b & (Ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[lds_slot(b + r * NB)];
            if (Ns > 1) {
                // twiddle exponent k r / (Ns R) of a full turn = (k r N / (Ns R)) / N
                constexpr int shift = (LOG2H + 1) - (LOG2NS + (R == 8 ? 3 : (R == 4 ? 2 : 1)));
                Cx<T> w[R];
                butterfly_twiddles<T, R>(tw, k << shift, w);
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], w[r]);
            }
            dft_inv<T, R>(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if (NB % NT == 0 || b < NB) {
            const int k = b & (Ns - 1);
            const int o = (b - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[lds_slot(o + q * Ns)] = v[i][q];
        }
    }
    __syncthreads();
}

// Radix 8 while at least 3 bits remain, then one radix-4 or radix-2 pass.
template <typename T, int LOG2H, int NT, int DONE>
__device__ __forceinline__ void run_passes(Cx<T>* buf, const Cx<T>* __restrict__ tw)
{
    constexpr int REM = LOG2H - DONE;
    if constexpr (REM >= 3) {
        stockham_pass<T, LOG2H, 8, NT, DONE>(buf, tw);
        run_passes<T, LOG2H, NT, DONE + 3>(buf, tw);
    } else if constexpr (REM == 2) {
        stockham_pass<T, LOG2H, 4, NT, DONE>(buf, tw);
    } else if constexpr (REM == 1) {
        stockham_pass<T, LOG2H, 2, NT, DONE>(buf, tw);
    }
}

// The pre-processing works on mirror pairs (k, H-k), k = tid + i NT < H/2: both Z_k and
// Z_{H-k} come from the same two modes, with w^{H-k} = -conj(w^k).  Pair k = 0 (whose
// partner X_H is zero) also carries the self-paired k = H/2.  A thread holds PAIRS + 1
// pairs of modes (X_k, X_{H-k}); the last slot is X_{H/2} for thread 0.
template <int LOG2H, int NT>
struct PrepShape {
    static constexpr int H = 1 << LOG2H;
    static constexpr int HALF = H / 2;
    static constexpr int PAIRS = HALF > 0 ? (HALF + NT - 1) / NT : 0;
};

template <typename T, int LOG2H, int NT>
__device__ __forceinline__ void c2r_load(const Cx<T>* __restrict__ row, int m_top, Cx<T>* xa, Cx<T>* xb)
{
    using S = PrepShape<LOG2H, NT>;
    const int tid = threadIdx.x;
    const Cx<T> zero = {T(0), T(0)};
#pragma unroll
    for (int i = 0; i < S::PAIRS; ++i) {
        const int k = tid + i * NT;
        xa[i] = zero;
        xb[i] = zero;
        if (S::HALF % NT == 0 || k < S::HALF) {
            if (k <= m_top) xa[i] = row[k];
            if (k == 0) xa[i].im = T(0);                      // g_0 is real
            if (k > 0 && S::H - k <= m_top) xb[i] = row[S::H - k];
        }
    }
    xa[S::PAIRS] = zero;   // X_{H/2} (thread 0), or X_1 when H = 1... never: H >= 2
    if (tid == 0 && S::HALF <= m_top) xa[S::PAIRS] = row[S::HALF];
}

// Z_k = (X_k + conj X_{H-k}) + i w^k (X_k - conj X_{H-k}) for both members of each pair,
// written to LDS.
template <typename T, int LOG2H, int NT>
__device__ __forceinline__ void c2r_prep(const Cx<T>* __restrict__ tw, const Cx<T>* xa, const Cx<T>* xb,
                                         Cx<T>* buf)
{
    using S = PrepShape<LOG2H, NT>;
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < S::PAIRS; ++i) {
        const int k = tid + i * NT;
        if (S::HALF % NT == 0 || k < S::HALF) {
            const Cx<T> a = xa[i], b = xb[i];                 // X_k, X_{H-k}
            const Cx<T> ca = {a.re, -a.im}, cb = {b.re, -b.im};
            const Cx<T> w = tw[k];
            const Cx<T> wm = {-w.re, w.im};                   // w^{H-k} = -conj(w^k)
            buf[lds_slot(k)] = cadd(cadd(a, cb), mul_i(cmul(w, csub(a, cb))));
            if (k > 0) buf[lds_slot(S::H - k)] = cadd(cadd(b, ca), mul_i(cmul(wm, csub(b, ca))));
        }
    }
    if (tid == 0) {
        const Cx<T> a = xa[S::PAIRS];                         // X_{H/2}, its own partner
        const Cx<T> ca = {a.re, -a.im};
        const Cx<T> w = tw[S::HALF];
        buf[lds_slot(S::HALF)] = cadd(cadd(a, ca), mul_i(cmul(w, csub(a, ca))));
    }
}

// Pointwise map applied as the transformed row is stored: none, or the lognormal field
// exp(mu + sigma T) of a Gaussian field T (the application named at the end of Sec. 4).
// `on` is uniform over the launch.
template <typename T>
struct Epilogue {
    T mu, sigma;
    int on;
};

__device__ __forceinline__ float exp_t(float x) { return expf(x); }
__device__ __forceinline__ double exp_t(double x) { return exp(x); }

template <typename T>
__device__ __forceinline__ Cx<T> epilogue(const Epilogue<T>& ep, Cx<T> v)
{
    if (ep.on) {
        v.re = exp_t(fma(ep.sigma, v.re, ep.mu));
        v.im = exp_t(fma(ep.sigma, v.im, ep.mu));
    }
    return v;
}

// C2R of one ring row (2H reals, holding modes 0..H-1 as complex on entry), by NT threads
// with an LDS buffer of lds_slots(H) complex values.  Ends with the row written; the caller must
// barrier before reusing `buf`.
template <typename T, int LOG2H, int NT>
__device__ __forceinline__ void c2r_row(T* __restrict__ data_row, const T* __restrict__ twr, int m_top,
                                        Cx<T>* buf, const Epilogue<T>& ep)
{
    using S = PrepShape<LOG2H, NT>;
    constexpr int H = 1 << LOG2H;
    constexpr int PER = (H + NT - 1) / NT;
    const Cx<T>* tw = reinterpret_cast<const Cx<T>*>(twr);
    Cx<T>* __restrict__ row = reinterpret_cast<Cx<T>*>(data_row);
    // pre-processing pair by pair, straight from global memory into LDS
#pragma unroll
    for (int i = 0; i < S::PAIRS; ++i) {
        Cx<T> xa[2], xb[2];
        const int k = threadIdx.x + i * NT;
        const Cx<T> zero = {T(0), T(0)};
        xa[0] = xb[0] = xa[1] = zero;
        if (S::HALF % NT == 0 || k < S::HALF) {
            if (k <= m_top) xa[0] = row[k];
            if (k == 0) xa[0].im = T(0);                      // g_0 is real
            if (k > 0 && H - k <= m_top) xb[0] = row[H - k];
            const Cx<T> a = xa[0], b = xb[0];
            const Cx<T> ca = {a.re, -a.im}, cb = {b.re, -b.im};
            const Cx<T> w = tw[k];
            const Cx<T> wm = {-w.re, w.im};
            buf[lds_slot(k)] = cadd(cadd(a, cb), mul_i(cmul(w, csub(a, cb))));
            if (k > 0) buf[lds_slot(H - k)] = cadd(cadd(b, ca), mul_i(cmul(wm, csub(b, ca))));
        }
    }
    if (threadIdx.x == 0) {
        const Cx<T> zero = {T(0), T(0)};
        const Cx<T> a = (S::HALF <= m_top) ? row[S::HALF] : zero;
        const Cx<T> ca = {a.re, -a.im};
        buf[lds_slot(S::HALF)] = cadd(cadd(a, ca), mul_i(cmul(tw[S::HALF], csub(a, ca))));
    }
    __syncthreads();
    run_passes<T, LOG2H, NT, 0>(buf, tw);
    // T_{2j} + i T_{2j+1} = z_j: the complex result written as interleaved reals
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int k = threadIdx.x + i * NT;
        if (H % NT == 0 || k < H) row[k] = epilogue(ep, buf[lds_slot(k)]);
    }
}

// C2R of rows row0, row0 + stride, ... < rows by one workgroup.  With PREFETCH the next
// row's modes are loaded into registers right after the current row has been moved into
// LDS, so their global latency overlaps the current row's passes (a barrier waits on
// LDS traffic only); without it each row is loaded when its turn comes (fewer registers).
template <typename T, int LOG2H, int NT, bool PREFETCH>
__device__ __forceinline__ void c2r_rows(T* __restrict__ data, const T* __restrict__ twr, int m_top,
                                         Cx<T>* buf, int rows, int row0, int stride, const Epilogue<T>& ep)
{
    constexpr int H = 1 << LOG2H;
    constexpr int PER = (H + NT - 1) / NT;
    if constexpr (!PREFETCH) {
        for (int r = row0; r < rows; r += stride) {
            c2r_row<T, LOG2H, NT>(data + (size_t)r * (2 * H), twr, m_top, buf, ep);
            __syncthreads();
        }
        return;
    } else {
        const Cx<T>* tw = reinterpret_cast<const Cx<T>*>(twr);
        Cx<T> xa[PrepShape<LOG2H, NT>::PAIRS + 1], xb[PrepShape<LOG2H, NT>::PAIRS + 1];
        if (row0 < rows)
            c2r_load<T, LOG2H, NT>(reinterpret_cast<const Cx<T>*>(data + (size_t)row0 * (2 * H)), m_top, xa, xb);
        for (int r = row0; r < rows; r += stride) {
            c2r_prep<T, LOG2H, NT>(tw, xa, xb, buf);
            __syncthreads();
            const int rn = r + stride;
            if (rn < rows)
                c2r_load<T, LOG2H, NT>(reinterpret_cast<const Cx<T>*>(data + (size_t)rn * (2 * H)), m_top, xa, xb);
            run_passes<T, LOG2H, NT, 0>(buf, tw);
            Cx<T>* __restrict__ row = reinterpret_cast<Cx<T>*>(data + (size_t)r * (2 * H));
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int k = threadIdx.x + i * NT;
                if (H % NT == 0 || k < H) row[k] = epilogue(ep, buf[lds_slot(k)]);
            }
            __syncthreads();
        }
    }
}


// ------------------------------------------------------------------ radix-16 C2R rows
// The C2R of rows of n_phi = 8192 (H = 4096 = 16^3) as three radix-16 Stockham passes of
// 256 threads, one butterfly per thread and pass.  The first pass takes its inputs
// Z_{t + 256 r} straight from the pre-processing in registers (thread t loads its modes
// X_k, k = t + 256 r, and their mirror partners X_{H-k}, which thread 256 - t also loads, so
// the second read comes from the cache), and the last pass stores its outputs
// z_{t + 256 q} straight to the row: the row sits in LDS only between the passes, 128 KB of
// LDS traffic and four barriers per row against 320 KB and nine for radix-8 passes.

// Inverse DFT of 16 values (kernel e^{+2 pi i r q / 16}) as 4 x 4: inverse DFT4s over r1 of
// x_{4 r1 + r0}, twiddles w^{r0 q1} with w = e^{2 pi i / 16}, inverse DFT4s over r0; output
// q = q1 + 4 q2.
template <typename T>
__device__ __forceinline__ void dft_inv16(Cx<T>* v)
{
    Cx<T> a[4][4];   // a[r0][q1]
#pragma unroll
    for (int r0 = 0; r0 < 4; ++r0) {
        Cx<T> t[4] = {v[r0], v[4 + r0], v[8 + r0], v[12 + r0]};
        dft_inv<T, 4>(t);
#pragma unroll
        for (int q = 0; q < 4; ++q) a[r0][q] = t[q];
    }
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);   // cos, sin pi/8
    const T h = T(0.70710678118654752440);
    const Cx<T> w1 = {c1, s1}, w2 = {h, h}, w3 = {s1, c1}, w6 = {-h, h}, w9 = {-c1, -s1};
    a[1][1] = cmul(a[1][1], w1);
    a[1][2] = cmul(a[1][2], w2);
    a[1][3] = cmul(a[1][3], w3);
    a[2][1] = cmul(a[2][1], w2);
    a[2][2] = mul_i(a[2][2]);
    a[2][3] = cmul(a[2][3], w6);
    a[3][1] = cmul(a[3][1], w3);
    a[3][2] = cmul(a[3][2], w6);
    a[3][3] = cmul(a[3][3], w9);
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1) {
        Cx<T> t[4] = {a[0][q1], a[1][q1], a[2][q1], a[3][q1]};
        dft_inv<T, 4>(t);
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) v[q1 + 4 * q2] = t[q2];
    }
}

// v[r] *= w^r, r = 1..15, w = tw[e]: w, w^4, w^8 from the table (e, 4e, 8e < N), the rest
// by at most two products.
template <typename T>
__device__ __forceinline__ void twiddle16(Cx<T>* v, const Cx<T>* __restrict__ tw, int e)
{
    const Cx<T> w1 = tw[e], w4 = tw[4 * e], w8 = tw[8 * e];
    const Cx<T> w2 = cmul(w1, w1), w3 = cmul(w2, w1);
    Cx<T> w[8];
    w[0] = {T(1), T(0)};
    w[1] = w1;
    w[2] = w2;
    w[3] = w3;
    w[4] = w4;
    w[5] = cmul(w4, w1);
    w[6] = cmul(w4, w2);
    w[7] = cmul(w4, w3);
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], w[r]);
    v[8] = cmul(v[8], w8);
#pragma unroll
    for (int r = 1; r < 8; ++r) v[8 + r] = cmul(v[8 + r], cmul(w8, w[r]));
}

// Mirror partners of the pre-processing: 1 through LDS (one more barrier), 0 from global
// memory (each value is loaded by two threads).
#ifndef SMF_R16_XCHG
#define SMF_R16_XCHG 1
#endif

// One row of n_phi = 8192 by 256 threads; `buf` holds lds_slots(4096) values.  Ends after the
// row's last LDS read (a barrier), so the caller may start the next row at once.
template <typename T>
__device__ __forceinline__ void c2r_row_r16(T* __restrict__ data_row, const T* __restrict__ twr, int m_top,
                                            Cx<T>* buf, const Epilogue<T>& ep)
{
    constexpr int H = 4096;
    const int t = threadIdx.x;
    const Cx<T>* tw = reinterpret_cast<const Cx<T>*>(twr);
    Cx<T>* __restrict__ row = reinterpret_cast<Cx<T>*>(data_row);
    const Cx<T> zero = {T(0), T(0)};
    // pre-processing: Z_k = (X_k + conj X_{H-k}) + i w^k (X_k - conj X_{H-k}), k = t + 256 r,
    // X_k = 0 above m_top, Im X_0 = 0, X_H = 0; w^k = tw[t] tw[256 r]
    Cx<T> xa[16], xb[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int k = t + 256 * r;
        xa[r] = k <= m_top ? row[k] : zero;
    }
    if (t == 0) xa[0].im = T(0);
#if SMF_R16_XCHG
    // the mirror partners through LDS: every thread stores its modes, then reads X_{H-k}
#pragma unroll
    for (int r = 0; r < 16; ++r) buf[lds_slot(t + 256 * r)] = xa[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int k = t + 256 * r;
        xb[r] = k > 0 ? buf[lds_slot(H - k)] : zero;
    }
#else
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int k = t + 256 * r;
        xb[r] = (k > 0 && H - k <= m_top) ? row[H - k] : zero;
    }
#endif
    const Cx<T> wt = tw[t];
    Cx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const Cx<T> a = xa[r], cb = {xb[r].re, -xb[r].im};
        const Cx<T> w = r == 0 ? wt : cmul(wt, tw[256 * r]);
        v[r] = cadd(cadd(a, cb), mul_i(cmul(w, csub(a, cb))));
    }
#if SMF_R16_XCHG
    __syncthreads();   // every partner read before the first pass overwrites the buffer
#endif
    // pass 1 (Ns = 1): no twiddles; outputs 16 t + q
    dft_inv16<T>(v);
#pragma unroll
    for (int q = 0; q < 16; ++q) buf[lds_slot(16 * t + q)] = v[q];
    __syncthreads();
    // pass 2 (Ns = 16): k = t mod 16, twiddles e^{2 pi i k r / 256} = tw[32 k r]; outputs
    // (t - k) 16 + k + 16 q
    {
        const int k = t & 15;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = buf[lds_slot(t + 256 * r)];
        __syncthreads();
        twiddle16<T>(v, tw, 32 * k);
        dft_inv16<T>(v);
        const int o = (t - k) * 16 + k;
#pragma unroll
        for (int q = 0; q < 16; ++q) buf[lds_slot(o + 16 * q)] = v[q];
    }
    __syncthreads();
    // pass 3 (Ns = 256): k = t, twiddles e^{2 pi i t r / 4096} = tw[2 t r]; outputs t + 256 q,
    // the results z_j = T_{2j} + i T_{2j+1}, stored to the row
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = buf[lds_slot(t + 256 * r)];
    __syncthreads();
    twiddle16<T>(v, tw, 2 * t);
    dft_inv16<T>(v);
#pragma unroll
    for (int q = 0; q < 16; ++q) row[t + 256 * q] = epilogue(ep, v[q]);
}

}  // namespace smf
