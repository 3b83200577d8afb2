/*
 * smf.h -- C ABI of the MI355X (gfx950) sampler of isotropic Gaussian random fields
 * on the sphere by latitude-ring Gauss-Markov recursions and an FFT along phi
 * (Creasey & Lang, "Fast generation of isotropic Gaussian random fields on the
 * sphere", arXiv:1709.10314).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: SMF_OK (0) on success, a negative SMF_E* code on error.  On error no
 *    output buffer is written and no plan is created; smf_error_string() names the code.
 *  - Device pointers are HIP device memory (e.g. torch.cuda tensors); host pointers are
 *    ordinary CPU memory.  The caller owns every buffer it passes; the plan owns its own
 *    device buffers (factors, spectrum, twiddles) and frees them in smf_destroy().
 *  - Streams are hipStream_t passed as void* (NULL = the null stream).  Sampling calls
 *    are asynchronous on that stream; setup synchronises its stream before returning.
 *  - The sampling calls only read a plan, so one plan may be used from several streams at
 *    once (each call needs its own output buffer); the calls that change a plan
 *    (smf_set_ring_blocks, smf_set_factors, smf_autotune_batch, smf_batch_set_shape) must
 *    not overlap them.
 *
 * Grid: n_theta iso-latitude rings at ring centres theta_i = pi (i + 1/2) / n_theta
 * (ring 0 nearest the north pole, z_i = cos theta_i) and n_phi equispaced longitudes
 * phi_j = 2 pi j / n_phi (Sec. 4, grid and Alg. 2).  Modes m = 0..m_top with
 * m_top = min(ell_max, n_phi/2 - 1).
 */
#ifndef SMF_H
#define SMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smf_plan smf_plan;

/* Angular power spectrum, eq. (Cl): C_l = prod_{i<n_kappa} (kappa_i + l(l+1))^-1 for
 * l = 0..ell_max, and C_l = 0 above ell_max.  If c_ell is non-NULL it is used instead
 * (ell_max + 1 values, host memory).  `order` is the Markov order M, i.e. the state
 * dimension (value and first M-1 z-derivatives, Sec. 2 Markov property); M in {1, 2, 3, 4}.
 * For the rational form M is normally n_kappa. */
typedef struct {
    int order;
    int n_kappa;
    const double* kappa;   /* host, n_kappa values */
    const double* c_ell;   /* host, ell_max + 1 values, or NULL */
    int ell_max;
} smf_spectrum;

enum {
    SMF_OK = 0,
    SMF_EINVAL = -1,     /* bad argument (shape, order, NULL pointer, count < 0, ...) */
    SMF_ENOMEM = -2,     /* device allocation failed */
    SMF_EHIP = -3,       /* a HIP runtime call or kernel launch failed */
    SMF_ENUMERIC = -4    /* spectrum has a C_l that is not finite and positive */
};

enum {
    SMF_FP64 = 1,        /* sample in FP64 (recursion, normals, FFT) */
    SMF_FP32 = 2,        /* sample in FP32 (factors rounded from the FP64 setup) */
    SMF_NO_MIRROR = 4,   /* or'ed with one of the above: store the southern walk's own factor
                            sets, (s+j-1) -> (s+j) in true coordinates, instead of reusing the
                            northern ones through the mirror D A D, D B D of the symmetry remark
                            after Alg. 1 (twice the factor memory).  On a grid symmetric about
                            the equator the two tables agree to the bit and so do the samples;
                            a grid with no symmetry always stores both. */
    SMF_FUSED = 8,       /* reserved for a single-kernel recursion + FFT; smf_setup returns
                            SMF_EINVAL for it (the two launches of smf_sample are the path) */
    SMF_GREEN = 32,      /* or'ed with SMF_FP64 or SMF_FP32: the setup of Sec. 3 at order 1 or 2.
                            The spectrum is eq. (Cl) with n_kappa = order distinct real kappa_i in
                            [1e-5, 1e4] (c_ell NULL; the Green's functions grow like exp(pi sqrt kappa)
                            and are formed in FP64, and lose digits as kappa -> 0; at order 2 |kappa_2 - kappa_1| >= 1e-3 max kappa,
                            as the partial fractions cancel log10(kappa / |kappa_2 - kappa_1|)
                            digits) for every l >= 0, not truncated (ell_max is ignored and
                            every mode up to n_phi/2 - 1 is sampled), and J^m comes from the Green's
                            functions of the mode's operator, eq. (Jmatrix_efficient) with the
                            partial fractions of eq. (C_ell_efficient), and P^m_lambda of complex
                            degree (kappa_i = -lambda_i(lambda_i+1)) from its hypergeometric series,
                            eq. (Legendre_hypergeometric), instead of sums over l: the chain is then
                            exactly Markov.  At order 2 the state is (g, U_m g), the basis of
                            SMF_UBASIS.  Needs order * n_theta * (n_phi / 2 + 1) <= 2^27 (two setup
                            tables of that many doubles). */
    SMF_KAPPA_PAIR = 64, /* with SMF_GREEN at order 2: kappa = {alpha, beta} names the complex-
                            conjugate pair kappa = alpha +- i beta (alpha >= -50, 0 < beta <= 1000, 1e-5 <= |kappa| <= 1e4:
                            outside, the series of the Green's functions cancels), the spectrum
                            C_l = 1/((l(l+1) + alpha)^2 + beta^2) (the Sec. 5 example is alpha = 0,
                            beta = sqrt(10)); the two terms of the partial fractions are complex
                            conjugates and the Green's functions have complex degree and complex
                            kappa.  SMF_EINVAL without SMF_GREEN at order 2. */
    SMF_UBASIS = 16      /* order 2 only, or'ed with one of the above: the chain state is
                            (g, U_m g) with the operator U_m of Sec. 3 (eq. (Jmatrix_more_efficient):
                            U_m maps P^m to P^{m+1}, so the setup sums L_{l,m+1} instead of
                            z-derivatives) in place of (g, dg/dz).  The field has the same law;
                            its realisations for given normals differ. */
};

/* Alg. 1 (pre-computation of covariance matrices), run on the GPU in FP64: for every
 * mode m <= m_top, the start factor B_eq (eq. (state_initial)) at the start ring, and for
 * each ring step the transition A = J(b,a) J(a,a)^+ (eq. (trans_matrix)) and the lower
 * Cholesky factor B of S = J(b,b) - A J(a,b) (eq. (innov_matrix)), with J the
 * cross-covariance blocks of Lemma 2.1 summed over l <= ell_max.  Only the northern half
 * is stored; the southern steps are the mirror D A D, D B D (symmetry remark after Alg. 1).
 *   spec      host; copied, not retained.
 *   n_theta   >= 2 rings.     n_phi  power of two in [4, 16384].
 *   flags     exactly one of SMF_FP64, SMF_FP32, optionally or'ed with SMF_NO_MIRROR,
 *             SMF_UBASIS (order 2) or SMF_GREEN (orders 1 and 2; with SMF_KAPPA_PAIR at order 2).
 *   out       receives the new plan (host pointer to a pointer).
 * Orders 3 and 4 take the second and third z-derivatives of L_lm from the associated
 * Legendre equation; their records hold A row-major and B's lower triangle (16 and 32
 * values per record with padding).
 * Errors: SMF_EINVAL (shapes, order not in 1..4, ell_max < 0, n_kappa < 0, NULL
 * pointers, flags), SMF_ENUMERIC (a C_l not finite and > 0), SMF_ENOMEM, SMF_EHIP. */
int smf_setup(const smf_spectrum* spec, int n_theta, int n_phi, int flags, void* hip_stream,
              smf_plan** out);

/* Alg. 1 on an explicit grid: its signature takes the ring values z as an input.  z_host
 * (host, n_theta doubles, copied) lists the rings from north to south: strictly
 * decreasing and inside (-1, 1); sin(theta_i) is taken as sqrt((1 - z_i)(1 + z_i)).  The
 * start ring (s = n_theta/2 - 1 or (n_theta-1)/2) and the crossing step are those of
 * smf_setup.  A grid symmetric to the bit, z[n_theta-1-i] == -z[i], stores only the
 * northern steps and mirrors them for the south (the remark after Alg. 1); any other grid
 * also stores the southern walk's own steps (s+j-1) -> (s+j), twice the factor memory.  The
 * phi grid, the sampling calls and their output are unchanged.  Examples: the ring-centre
 * grid itself (for odd n_theta it is the paper's symmetric example grid, read as
 * z_j = sin(pi j / n_theta)), Gauss-Legendre nodes, HEALPix ring latitudes, shifted ring
 * centres.
 * Errors: as smf_setup, plus SMF_EINVAL for a NULL z_host or a grid that is not strictly
 * decreasing in (-1, 1). */
int smf_setup_grid(const smf_spectrum* spec, int n_theta, const double* z_host, int n_phi, int flags,
                   void* hip_stream, smf_plan** out);

/* Alg. 2 (Gaussian random field generation): `count` fields, field f drawn with the
 * Philox4x32-10 key seed + f.  Writes out_dev, device memory of count*n_theta*n_phi
 * float (SMF_FP32 plan) or double (SMF_FP64 plan), layout [field][ring][phi], ring 0
 * nearest the north pole.  count = 0 is a no-op.  Uses no memory beyond out_dev: the
 * modes g_m are written into out_dev and transformed in place.
 * Errors: SMF_EINVAL (NULL plan/out with count > 0, count < 0, count * n_theta > 2^31 - 1),
 * SMF_EHIP. */
int smf_sample(const smf_plan* plan, uint64_t seed, int count, void* out_dev, void* hip_stream);

/* A lognormal field (the application named at the end of Sec. 4): smf_sample with the
 * pointwise map out = exp(mu + sigma T) applied as the FFT stores T, in the plan's
 * precision (FP32: expf of fmaf(sigma, T, mu)).  Same layout, size and keys as smf_sample.
 * Errors: as smf_sample, plus SMF_EINVAL for a mu or sigma that is not finite. */
int smf_sample_lognormal(const smf_plan* plan, uint64_t seed, int count, double mu, double sigma, void* out_dev,
                         void* hip_stream);

/* The chains of Alg. 2 only (eqs. (state_initial) and (state_space)), without the FFT:
 * writes g_m(z_i) for field f, ring i, mode m as interleaved (Re, Im) pairs at
 * g_dev[((f*n_theta + i)*(n_phi/2) + m)*2 + {0,1}], element type as in smf_sample; the
 * entries for m > m_top are zero.  Same size and errors as smf_sample. */
int smf_sample_modes(const smf_plan* plan, uint64_t seed, int count, void* g_dev, void* hip_stream);

/* The last step of Alg. 2 on its own: the unnormalised complex-to-real inverse DFT along
 * phi of every ring, T(z_i, phi_j) = g_0 + 2 sum_{m=1}^{m_top} Re(g_m e^{i m phi_j}), in
 * place.  data_dev holds count fields of modes in the layout smf_sample_modes writes
 * (entries m > m_top and the imaginary part of g_0 are ignored) and receives the fields in
 * the layout smf_sample writes.  smf_sample = smf_sample_modes then smf_transform.
 * Errors: SMF_EINVAL (NULL plan/data with count > 0, count < 0, count * n_theta > 2^31 - 1,
 * batch plan), SMF_EHIP. */
int smf_transform(const smf_plan* plan, int count, void* data_dev, void* hip_stream);

/* Ring blocks of the affine scan (single-field plans).  The recursion of eq. (state_space)
 * is affine in the state, so a chain cut into ring blocks can run its blocks in parallel:
 * each block's end state from zero start, then the true block starts by composing the
 * blocks' transitions (products of the step matrices A, built at setup) with those end
 * states, then each block again from its true start.  Used when a call's chains alone
 * cannot fill the GPU; it doubles the arithmetic and changes results only by rounding.
 *   blocks  0: automatic: with w = count * 2 * ceil(n_phi / 64) (the wavefronts of the plain
 *              recursion with one chain per lane), no scan from w >= 1024; below that FP32
 *              scans with 8 blocks (w >= 512) or 16 blocks, FP64 with the fewest blocks
 *              giving >= 4096 wavefronts; every block keeps >= 32 ring steps or the
 *              count of blocks halves (no scan below 2);
 *           1: never;
 *           2, 4, 8 or 16: always, with that many blocks, capped at the plan's maximum (the
 *              largest power of two <= 16 leaving >= 8 ring steps per block, 1 when the
 *              walk has fewer than 16 steps) and at 8 for SMF_FP64 plans.
 * Plans of order 3 or 4 run one part per lane and scan with at most 8 blocks; their
 * automatic choice is the fewest blocks giving >= 4096 wavefronts, as for SMF_FP64.
 * The plan stores one transition per (fine block, m): 16 * (n_phi/2) * M*M values in FP64
 * (and FP32 for SMF_FP32 plans).
 * Errors: SMF_EINVAL (NULL, batch plan, blocks not 0, 1 or a power of two <= 16). */
int smf_set_ring_blocks(smf_plan* plan, int blocks);

/* The ring blocks a call of smf_sample or smf_sample_modes with `count` fields would use
 * (1 = plain recursion).  Errors: SMF_EINVAL (NULL, batch plan, count < 0). */
int smf_get_ring_blocks(const smf_plan* plan, int count, int* blocks);

/* Plan geometry (single-field plans): dims[0..7] = {order, n_theta, n_phi, ell_max, m_top, n_sets, start_ring,
 * precision flag}.  n_sets = number of factor sets per mode (start, crossing for even
 * n_theta, then one per northern step).  Errors: SMF_EINVAL on NULL. */
int smf_plan_dims(const smf_plan* plan, int* dims);

/* Copies the FP64 factors to host arrays A_host and B_host, each of n_sets*(m_top+1)*M*M
 * doubles, layout [set][m][p][q] row-major (B lower triangular; set 0 holds A = 0 and
 * B = B_eq).  Set j >= 1 is the step between the ring pair it covers: for even n_theta
 * (start ring s = n_theta/2 - 1) set 1 is the crossing s -> s+1 and set j >= 2 the step
 * s-j+2 -> s-j+1; for odd n_theta (s = (n_theta-1)/2) set j >= 1 is s-j+1 -> s-j.
 * A plan on a grid with no symmetry (smf_plan_grid) holds 2*n_sets sets: the northern ones,
 * then the southern walk's, whose set j >= j0 (2 for even n_theta, else 1) is the step
 * s+j-1 -> s+j in true coordinates (sets below j0 repeat the northern ones).
 * Synchronous.  Errors: SMF_EINVAL on NULL, SMF_EHIP. */
int smf_get_factors(const smf_plan* plan, double* A_host, double* B_host);

/* The plan's ring grid: z_host (may be NULL) receives the n_theta ring values the setup
 * used (for smf_setup plans the ring centres, recomputed on the host to rounding), and
 * *symmetric (may be NULL) 1 when the south mirrors the northern factor sets, 0 when it
 * has its own (a grid with no symmetry).  Errors: SMF_EINVAL (NULL or batch plan). */
int smf_plan_grid(const smf_plan* plan, double* z_host, int* symmetric);

/* Alg. 2 takes the factors (A, B, B_eq) as its input: replaces the plan's factors with
 * caller-given FP64 ones in the layout of smf_get_factors (2*n_sets sets for a grid with no
 * symmetry; set 0: A ignored, B = B_eq; the upper triangle of each B is ignored), e.g. factors from another setup, then rounds the
 * FP32 copy (SMF_FP32 plans) and rebuilds the scan's block transitions.  Synchronous on
 * hip_stream; must not overlap sampling calls on the plan.
 * Errors: SMF_EINVAL (NULL, batch plan, a value that is not finite), SMF_EHIP. */
int smf_set_factors(smf_plan* plan, const double* A_host, const double* B_host, void* hip_stream);

/* ---- batched form: many fields of uneven shape, spectrum and order per call ---- */

/* One FP32 plan per field (Alg. 1 for each, as smf_setup with SMF_FP32) plus flat work
 * lists: chain items (field, group of m-tiles), longest chains first, and one FFT item
 * per ring of every field.  specs, n_theta, n_phi: host arrays of n entries (n in
 * [1, 65535]); n_phi[i] a power of two in [4, 4096]; flags must be SMF_FP32.
 * Errors: as smf_setup, per field. */
int smf_setup_batch(int n, const smf_spectrum* specs, const int* n_theta, const int* n_phi,
                    int flags, void* hip_stream, smf_plan** out);

/* Packed output layout of a batch plan: offsets[0..n] (host, n+1 int64) in elements;
 * field i occupies [offsets[i], offsets[i+1]) as [ring][phi].  Errors: SMF_EINVAL. */
int smf_batch_layout(const smf_plan* plan, int64_t* offsets);

/* Samples every field of a batch plan (Alg. 2 for each) into the caller's buffers: one
 * launch over all chain items, then one over all rings.
 *   seeds_host  host array of n Philox keys, field i drawn with seeds_host[i].
 *   outs_dev    host array of n device pointers; field i is written to outs_dev[i] as
 *               n_theta[i] * n_phi[i] floats, layout [ring][phi] (8-byte aligned).
 * Both arrays are read before the call returns.  The keys and pointers are staged
 * through one of four plan-owned slots (pinned host memory and a device table); a slot
 * is reused only once the call that last used it has completed on the GPU, so calls may
 * overlap on different streams.  Not for stream capture: the table is uploaded per call
 * (SMF_EINVAL while the stream is capturing); smf_sample_batch_packed is the capturable
 * form.  Errors: SMF_EINVAL (NULL plan or array, not a batch plan, a NULL or misaligned
 * buffer, a capturing stream), SMF_EHIP. */
int smf_sample_batch(const smf_plan* plan, const uint64_t* seeds_host, void* const* outs_dev, void* hip_stream);

/* The same fields into one packed buffer (layout of smf_batch_layout), field i drawn with
 * Philox key seed + i.  No memset, no allocation and no host synchronisation, so the
 * call can be captured in a HIP graph; it only reads the plan, so calls may overlap on
 * different streams.  out_dev: device float array of offsets[n] elements.
 * Errors: SMF_EINVAL (NULL, not a batch plan), SMF_EHIP. */
int smf_sample_batch_packed(const smf_plan* plan, uint64_t seed, void* out_dev, void* hip_stream);

/* Autotuner of the launch shape: times smf_sample_batch_packed with 1, 2 and 4 m-tiles per
 * chain item (2, 4 and 8 waves per workgroup), each in both forms of smf_batch_set_shape
 * (writing out_dev, seed as in smf_sample_batch_packed), keeps the fastest in the plan and
 * returns its m-tile count in *tiles_out (may be NULL; smf_batch_get_shape gives the form).
 * Synchronous; not to be called while the plan is in use.
 * Errors: SMF_EINVAL, SMF_EHIP. */
int smf_autotune_batch(smf_plan* plan, uint64_t seed, void* out_dev, void* hip_stream, int* tiles_out);

/* The batch plan's launch shape: tiles m-tiles per chain item (1, 2 or 4) and the form, 0 for
 * two launches (every chain item, then every ring), 1 for one cooperative launch of as many
 * workgroups as the device holds at once, which run the chain items, meet at a grid barrier
 * and run the ring items (the persistent form).  Results agree to FP32 rounding across shapes
 * (the ring transforms of the persistent form run 128 * tiles threads per row, and are
 * compiled separately for each count).
 * smf_autotune_batch times all six shapes and keeps the fastest.  Errors: SMF_EINVAL. */
int smf_batch_set_shape(smf_plan* plan, int tiles, int persistent);
int smf_batch_get_shape(const smf_plan* plan, int* tiles, int* persistent);

/* Rings with their own pixel counts (iso-latitude grids such as HEALPix, named in Sec. 1):
 * ring i (latitude z_host[i], or the ring centres if z_host is NULL, same rules as
 * smf_setup_grid) holds n_phi_ring[i] pixels at longitudes phi0[i] + 2 pi j / n_phi_ring[i],
 * j < n_phi_ring[i].  The plan is that of smf_setup_grid on n_phi = the smallest power of
 * two >= 2 (ell_max + 1), so m_top = ell_max and every mode is sampled (smf_plan_dims
 * reports that n_phi; every call of a plan works on it), plus the ring table.  Host arrays
 * of n_theta entries, copied.  With SMF_GREEN (and SMF_KAPPA_PAIR) the factors are those of
 * Sec. 3 for the modes up to ell_max, the band the rings are synthesised from (the spectrum
 * itself has no band limit, so the chains are exactly Markov).
 * Errors: as smf_setup_grid, plus SMF_EINVAL for a NULL n_phi_ring or phi0, an odd
 * n_phi_ring[i] or one outside [2, 8192] (SMF_FP32) or [2, 4096] (SMF_FP64), a phi0 that is
 * not finite, or ell_max > 8191. */
int smf_setup_rings(const smf_spectrum* spec, int n_theta, const double* z_host, const int* n_phi_ring,
                    const double* phi0, int flags, void* hip_stream, smf_plan** out);

/* (A ring plan runs chains only for the 64-mode tiles that hold m <= ell_max: its
 * smf_sample_modes leaves the entries above those tiles unwritten, which neither the ring
 * synthesis nor smf_transform reads.) */

/* Layout of a ring plan's fields: offsets[0..n_theta], ring i of a field at
 * [offsets[i], offsets[i+1]); a field holds offsets[n_theta] values.
 * Errors: SMF_EINVAL (NULL, not a ring plan). */
int smf_ring_layout(const smf_plan* plan, int64_t* offsets);

/* Alg. 2's last step on a ring plan's rings: with c_m = g_m e^{i m phi0[i]} and
 * c_{-m} = conj(c_m), T(z_i, phi0[i] + 2 pi j / n) = sum_{|m| <= m_top} c_m e^{2 pi i m j / n},
 * n = n_phi_ring[i]; modes above n / 2 alias onto the ring's pixels, none is dropped.
 * g_dev: `count` fields of modes in the smf_sample_modes layout of the plan (read only);
 * out_dev: count * offsets[n_theta] values of the plan's type, field f at
 * f * offsets[n_theta].  The buffers must not overlap.  count = 0 is a no-op.
 * Errors: SMF_EINVAL (NULL, not a ring plan, count < 0 or > 65535), SMF_EHIP. */
int smf_synthesize_rings(const smf_plan* plan, int count, const void* g_dev, void* out_dev, void* hip_stream);

/* smf_sample_modes into the caller's work buffer g_work (count * n_theta * n_phi values of
 * the plan's type, n_phi as smf_plan_dims reports), then smf_synthesize_rings into out_dev.
 * Field f uses Philox key seed + f.  Errors: as the two calls, plus SMF_EINVAL when g_work
 * and out_dev are the same pointer. */
int smf_sample_rings(const smf_plan* plan, uint64_t seed, int count, void* g_work, void* out_dev,
                     void* hip_stream);

/* smf_sample_rings for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): no work buffer is passed and none
 * is allocated; the modes go to a file-scope device array of the library, 64 MiB on each
 * device the library runs on (held until the process ends), so count * n_theta * n_phi values
 * of the plan's type (n_phi as smf_plan_dims reports) must fit in 64 MiB.  Every call on a
 * device shares that device's array: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.  Same results as smf_sample_rings.
 * Errors: as smf_sample_rings, plus SMF_EINVAL when the modes exceed 64 MiB; SMF_EHIP if the
 * array's device address cannot be obtained. */
int smf_sample_rings_noalloc(const smf_plan* plan, uint64_t seed, int count, void* out_dev, void* hip_stream);

/* smf_sample_rings with the lognormal map of smf_sample_lognormal, exp(mu + sigma T), applied
 * as the pixels are stored (the application named at the end of Sec. 4, on a ring plan).
 * Errors: as smf_sample_rings, plus SMF_EINVAL for a mu or sigma that is not finite. */
int smf_sample_rings_lognormal(const smf_plan* plan, uint64_t seed, int count, double mu, double sigma,
                               void* g_work, void* out_dev, void* hip_stream);

/* ---- throughput references for the roofline of the chain kernels (measured, not modelled) ---- */

/* The sampler's white noise alone: `workgroups` workgroups of 256 lanes, each lane making
 * stages * 8 Philox4x32-10 blocks (eight in lockstep per stage, as a lane of the order-2
 * recursion does) and turning every block into four FP32 Box-Muller normals, with none of
 * the recursion's loads, stores or chain steps; each lane writes the sum of its normals to
 * out_dev[lane] (workgroups * 256 floats, device).  Normals made: workgroups * 256 * stages
 * * 32.  Asynchronous on hip_stream; the caller times it.  Errors: SMF_EINVAL, SMF_EHIP. */
int smf_measure_normals(uint64_t seed, int workgroups, int stages, void* out_dev, void* hip_stream);

/* Unpacked FP32 fused multiply-adds: each of workgroups * 256 lanes runs 8 independent
 * chains of iters * 16 FMAs and writes their sum to out_dev[lane].  Lane-FMAs made:
 * workgroups * 256 * iters * 128.  Errors: SMF_EINVAL, SMF_EHIP. */
int smf_measure_fma(int workgroups, int iters, void* out_dev, void* hip_stream);

/* Test hook for the allocation-failure paths: after n more successful device (or pinned
 * host) allocations made by the library, the next one fails as if the device were out of
 * memory, and the call that made it returns SMF_ENOMEM having freed what it allocated;
 * n = -1 turns the injection off (the default).  Process-wide; not for concurrent use.
 * Errors: SMF_EINVAL (n < -1). */
int smf_debug_fail_alloc(int n);

/* Diagnostics on stderr, one line per event prefixed "[smf] ": level 0 none, 1 each plan's setup
 * (geometry, layout and transform-class choices, sizes) and the reason for each argument a
 * setup rejects, 2 also each sampling call's launch shape.  The level starts from the environment
 * variable SMF_LOG (0 when unset) and this call replaces it for the process.  Returns the
 * previous level; SMF_EINVAL for a negative level. */
int smf_set_log_level(int level);

/* Frees the plan and its device memory (synchronises the device first).  NULL is a
 * no-op. */
int smf_destroy(smf_plan* plan);

/* Static string for an SMF_* code. */
const char* smf_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* SMF_H */
