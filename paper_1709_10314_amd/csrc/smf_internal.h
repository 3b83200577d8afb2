// Internal declarations shared by the HIP translation units of libsmf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smf.h"

namespace smf {

// Thresholds of the factorisation (equilibrated, thresholded Cholesky):
//   a block diagonal entry not above kTiny is exactly zero (its row/column is dropped);
//   after equilibration a pivot, or a conditional variance relative to the marginal one,
//   not above kTau is dropped.
constexpr double kTiny = 1e-290;
constexpr double kTau = 1e-12;

// Factor record per (set j, mode m), stored [set][m][E] with m stride n_phi/2:
// M = 1 -> {A00, B00}; M = 2 -> {A00, A01, A10, A11, B00, B10, B11, 0};
// M = 3, 4 -> A row-major, then B's lower triangle by rows, zero-padded to E = 16, 32.
__host__ __device__ constexpr int factor_stride(int order)
{
    return order == 1 ? 2 : (order == 2 ? 8 : (order == 3 ? 16 : 32));
}

// Position of B_pq (q <= p) in an M >= 3 record.
template <int M>
__host__ __device__ constexpr int b_index(int p, int q) { return M * M + p * (p + 1) / 2 + q; }

struct Geometry {
    int order;       // Markov order M
    int n_theta;
    int n_phi;
    int ell_max;
    int m_top;       // highest mode sampled
    int m_rows;      // chain rows per factor set: n_phi / 2 (ring plans: the 64-mode tiles up to
                     // m_top); rows above m_top hold zeros
    int n_sets;      // factor sets per mode
    int s;           // start ring
    int even;        // n_theta even (crossing step present)
};

inline Geometry make_geometry(int order, int n_theta, int n_phi, int ell_max)
{
    Geometry g;
    g.order = order;
    g.n_theta = n_theta;
    g.n_phi = n_phi;
    g.ell_max = ell_max;
    g.m_top = ell_max < n_phi / 2 - 1 ? ell_max : n_phi / 2 - 1;
    g.m_rows = n_phi / 2;
    g.even = (n_theta % 2 == 0);
    g.n_sets = g.even ? n_theta / 2 + 1 : (n_theta + 1) / 2;
    g.s = g.even ? n_theta / 2 - 1 : (n_theta - 1) / 2;
    return g;
}

// ---- setup (FP64) ----
hipError_t launch_spectrum(const double* kappa_dev, int n_kappa, const double* c_explicit_dev,
                           int ell_max, double* C_dev, int* bad_dev, hipStream_t st);
// z_dev: ring values of an explicit grid (device, n_theta doubles) or null for ring centres.
// south: the southern walk's own sets of a grid with no symmetry, stored mirrored.
// ubasis (order 2): the state basis (g, U g) of Sec. 3 in place of (g, dg/dz).
hipError_t launch_factors(const Geometry& g, const double* C_dev, const double* z_dev, int south, int ubasis,
                          double* f64, float* f32, hipStream_t st);
hipError_t launch_twiddles(int n_phi, double* tw64, float* tw32, hipStream_t st);
// Sec. 3 at order 1 (C_l = 1/(kappa + l(l+1)) for every l) and order 2 (two distinct kappa,
// basis (g, U g)): the hypergeometric factors H_m(z_i) into hp and H_m(-z_i) into hn, per kappa
// a table [n_theta][m_rows + 1] (m up to m_top + order - 1), the tables of the kappa one after
// the other; then the factor records from them.
hipError_t launch_green_tables(const Geometry& g, int n_kappa, const double* kappa, const double* z_dev, double* hp,
                               double* hn, hipStream_t st);
hipError_t launch_factors_green(const Geometry& g, const double* kappa, const double* z_dev, int south,
                                const double* hp, const double* hn, double* f64, float* f32, hipStream_t st);
// Largest n_kappa * n_theta * (n_phi / 2 + 1) of a Green's-function plan (its two setup tables
// of that many doubles each)
constexpr long long kGreenMaxTable = 1LL << 27;
// Phi per (fine ring block, m) for the affine scan, layout [block][m][M*M], m stride m_rows.
hipError_t launch_phi(const Geometry& g, const double* f64, int blocks, double* phi64, float* phi32,
                      hipStream_t st);

// ---- affine scan across rings ----
// Main-walk sets [j0, n_sets) of a hemisphere, j0 = 2 for even n_theta (set 1 is the
// crossing) else 1.  The plan cuts them into scan_fine fine blocks (a power of two <= 16,
// each of >= kScanMinSets sets, or 1 when the walk is too short); a scanned call uses
// `blocks` ring blocks of scan_fine / blocks fine blocks each.
constexpr int kScanMaxBlocks = 16;
constexpr int kScanMinSets = 8;
constexpr int kScanAutoMinSets = 32;   // the automatic choice keeps blocks this long
// a scanned call runs one wave per ring block in a workgroup: 16 (FP32) or 8 (FP64, whose
// walk needs up to 256 VGPRs) waves at most, and 8 at orders 3 and 4
inline int scan_max_blocks(int fp64, int order = 2) { return (fp64 || order > 2) ? 8 : 16; }
inline int scan_fine_blocks(const Geometry& g)
{
    const int walk = g.n_sets - (g.even ? 2 : 1);
    int b = 1;
    while (b < kScanMaxBlocks && walk / (2 * b) >= kScanMinSets) b *= 2;
    return b;
}

// ---- sampling ----
// nch: chains per lane, 1 (one part) or 2 (both parts of a mode; FP32 only).
// south_off: elements from the northern factor table to the southern walk's own table
// (0: the south mirrors the northern sets).
hipError_t launch_recursion(const Geometry& g, int fp64, const void* fac, size_t south_off, uint64_t seed,
                            int count, void* out, int nch, hipStream_t st);
// exp(mu + sigma T) applied by the FFT as it stores T (the sample type's precision).
struct LognormalMap {
    double mu, sigma;
};
hipError_t launch_c2r(const Geometry& g, int fp64, const void* tw, int count, void* data,
                      const LognormalMap* ln, hipStream_t st);
// The chains of launch_recursion as an affine scan over `blocks` ring blocks per chain
// (blocks >= 2 dividing fine_blocks; phi holds the plan's fine-block transitions).
// south_off, phi_south_off: elements to the southern walk's own factor and transition
// tables (0: mirrored).
hipError_t launch_scan(const Geometry& g, int fp64, const void* fac, size_t south_off, const void* phi,
                       size_t phi_south_off, int fine_blocks, int blocks, uint64_t seed, int count, void* out,
                       int nch, hipStream_t st);

// Ring synthesis of a ring plan: the modes g ([count][n_theta][g_row] complex, m <= m_top)
// to the pixels of rings with n_ring[i] pixels (even) starting at longitude phi0[i], ring i
// of field f at out + f * total + off[i].  Device arrays list, n_ring, phi0, off; list holds
// the n_direct rings whose odd prime passes are all direct, then the n_chirp rings whose
// largest odd prime P (of n_ring / 2) takes the chirp-z pass, L = the power of two >= 2P - 1.
// ln (may be null): the lognormal map applied as the pixels are stored.
constexpr int kRingMaxEll = 8191;        // modes of the chains: n_phi <= 16384
constexpr int kRingMaxPixels32 = 8192;   // largest ring: two buffers + small tables in LDS
constexpr int kRingMaxPixels64 = 4096;
constexpr int kRingMaxCount = 65535;     // fields of one call (grid y)
// Smallest prime that takes the chirp-z pass (measured on HEALPix nside 1024 x 8 fields with the
// radix-4 chirp-z FFTs: 0.806 ms from 383, 0.834 from 251, 0.927 from 127)
#ifndef SMF_RING_CHIRP_MIN
#define SMF_RING_CHIRP_MIN 383
#endif
// Weight of a Bluestein ring transform of length L, per L log2 L, against the estimated work of
// the general kernel's odd-prime passes, for the choice of its class.  Not a count of operations:
// the general kernel's launch is the last to finish when the classes overlap, so moving rings
// out of it pays beyond their own work (measured on HEALPix nside 1024 x 8 fields with the
// Bluestein tables computed at setup and the classes balanced over the streams: synthesis
// 0.449 ms at 8, 0.436 at 6, 0.426 at 3.5, 0.422 at 2.5, 0.419 at 1.5, 0.418 at 0)
#ifndef SMF_RING_BLUE_COST
#define SMF_RING_BLUE_COST 1.5
#endif
// Smallest Bluestein length (log2)
#ifndef SMF_RING_BLUE_MIN_LOG2
#define SMF_RING_BLUE_MIN_LOG2 10
#endif
constexpr int kRingChirpMaxL32 = 4096;   // largest chirp-z length (LDS)
constexpr int kRingChirpMaxL64 = 2048;
// Rings whose half-length h is a power of two L, or whose whole length-h DFT goes through
// Bluestein's convolution of power-of-two length L >= 2h - 1, with 2^kRingFftMinLog2 <= L <=
// 2^kRingFftMaxLog2, take a launch per class and L (rings_fft.hip) ahead of the two above.
constexpr int kRingFftMinLog2 = 10;
constexpr int kRingFftMaxLog2 = 12;
constexpr int kRingFftClasses = kRingFftMaxLog2 - kRingFftMinLog2 + 1;
struct RingSplit {
    int n_direct, n_chirp;            // rings of each launch
    int n_max_direct, n_max_chirp;    // largest ring of each
    int l_max;                        // largest chirp-z length
    int n_blue[kRingFftClasses];      // Bluestein rings by L = 2^(kRingFftMinLog2 + c)
    int n_pow2[kRingFftClasses];      // rings with h = L
};
// Ring list order: Bluestein rings (largest L first), power-of-two rings (largest first),
// then the n_direct and n_chirp rings of launch_ring_c2r.
int ring_fft_count(const RingSplit& rs);
int ring_tw_entries();                                     // complex entries of the tables
size_t ring_fft_lds_bytes(int log2l, int m_top, bool fp64);
hipError_t launch_ring_tw(double* tw64, float* tw32, hipStream_t st);
// hs_dev[w]: half-lengths h whose Bluestein length is 2^log2l; the transform of each one's
// kernel goes to out (plan type) at offs_dev[w] values
hipError_t launch_ring_spectra(int log2l, int lengths, const int* hs_dev, const int64_t* offs_dev,
                               const double* tw64, bool fp64, void* out, hipStream_t st);
// One launch of the class (Bluestein or power-of-two) of length 2^log2l: `rings` rings from list.
hipError_t launch_ring_fft_class(bool blue, int log2l, int rings, int n_theta, int m_top, int g_row, int64_t total,
                                 bool fp64, int count, const void* g, const int* list, const int* n_ring,
                                 const double* phi0, const int64_t* off, const void* tw, const void* spec,
                                 const int64_t* spec_off, void* out, const LognormalMap* ln, hipStream_t st);
// Streams besides the caller's that a ring plan's synthesis spreads its launches over (forked
// from and joined back to the caller's stream by events).  Two, so that the caller's stream,
// these and the queue the runtime keeps once a cooperative launch (the persistent batch form)
// has run fit the four hardware queues a process gets: with three, a plan made after such a
// launch shared a queue between two of its streams and its classes ran one after the other
// (HEALPix nside 1024 x 8: 0.478 against 0.418 ms; two streams: 0.418 either way)
constexpr int kRingAuxStreams = 2;
#ifndef SMF_RING_FORK
#define SMF_RING_FORK 1
#endif
size_t ring_lds_bytes(int n_max, int m_top, bool fp64, int l_max = 0);
int ring_largest_odd_prime(int h);    // 1 when h is a power of two
hipError_t launch_ring_c2r(int n_theta, int m_top, int g_row, int64_t total, const RingSplit& rs, bool fp64,
                           int count, const void* g, const int* list, const int* n_ring, const double* phi0,
                           const int64_t* off, void* out, const LognormalMap* ln, hipStream_t st);

}  // namespace smf

namespace smf {
struct BatchState;
}

struct smf_plan {
    smf::Geometry g;
    int flags;           // SMF_FP64 or SMF_FP32
    double* C;           // [ell_max + 1]
    double* f64;         // FP64 factors
    float* f32;          // FP32 factors (SMF_FP32 plans)
    double* tw64;        // e^{+2 pi i t / n_phi}, t < n_phi
    float* tw32;
    int device;
    smf::BatchState* batch;   // non-null for a batch plan (see smf_setup_batch)
    int scan_fine;            // fine ring blocks with a stored transition (1: no scan)
    int scan_req;             // ring blocks asked for: 0 automatic, 1 never, else that many
    double* phi64;            // [scan_fine][m_rows][M*M] block transitions (twice for asym)
    float* phi32;
    int asym;                 // 1: a grid with no symmetry, the south walks its own sets
    size_t south_off;         // elements from the northern to the southern factor table
    size_t phi_south_off;     // the same for the block transitions
    double* zgrid;            // host copy of an explicit grid (null: ring centres)
    // rings with their own pixel counts (smf_setup_rings); n_ring_dev null otherwise
    int* n_ring_dev;          // [n_theta] pixels per ring
    double* phi0_dev;         // [n_theta] longitude of each ring's first pixel
    int64_t* ring_off_dev;    // [n_theta + 1] start of each ring in a field
    int64_t* ring_off;        // host copy
    int n_ring_max;           // largest ring
    int* ring_list_dev;       // [n_theta] rings by launch (see RingSplit)
    smf::RingSplit ring_split;
    double* ring_tw64;        // power-of-two transform tables (ring_tw_entries complex values)
    float* ring_tw32;         // the same rounded to FP32 (FP32 plans)
    void* ring_spec_dev;      // Bluestein tables per half-length (2 L values: the kernel's transform, chirp, chirp x twiddle), plan type
    int64_t* ring_spec_off_dev;   // [n_theta] each ring's transform (in complex values)
    hipStream_t ring_aux[smf::kRingAuxStreams];   // null when the synthesis is a single launch
    hipEvent_t ring_fork;
    hipEvent_t ring_join[smf::kRingAuxStreams];
};
