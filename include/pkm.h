/*
 * pkm.h - C ABI of libpkm: FFT-based power-spectrum multipoles with a local line of sight
 * (Hand, Li, Slepian & Seljak 2017, arXiv:1704.02357) on AMD Instinct MI355X (gfx950).
 *
 * What is computed.
 *   The FKP field F = w [n - alpha n_s] / I^(1/2) (Sec. 2.1, eq. FKP-density) is painted on
 *   an N^3 mesh (Sec. 2.3: NGP/CIC/TSC, optional interlacing and window compensation).  For
 *   every even l <= ell_max the multipole
 *       P_l(k) = (2l+1)/I  < F_0(k) F_l(-k) >_shell  - delta_l0 S            (eq. Pell-ours)
 *       F_l(k) = 4 pi/(2l+1) sum_m Y_lm(khat) FT[F Y_lm(rhat)](k)           (eq. Fell)
 *   is evaluated with 2l+1 transforms per l > 0 and the real harmonics of eq. real-Ylm.
 *   Wedges P(k, mu) follow from eq. wedge-est with the wedge means of eq. Lbar (Sec. 2.2).
 *
 * Conventions (readings of points the paper leaves open):
 *   - Node c of the mesh sits at box_origin + c L/N; painted taps wrap periodically.
 *   - Mesh coordinate u = (x - o) * (N/L) in FP64.  NGP/TSC centre node floor(u + 1/2),
 *     CIC base node floor(u).  The interlaced mesh is painted at u + 1/2 on every axis and
 *     the two transforms are averaged with phase exp(+i pi (n_x+n_y+n_z)/N).
 *   - Compensation: interlaced -> prod sinc^p(pi n_a/N); otherwise the alias-sum form
 *     prod sqrt(A_p(sin^2(pi n_a/N))) (p = 1, 2, 3 for NGP, CIC, TSC), applied once to the
 *     combined field before it is transformed back and harmonically weighted.
 *   - Every mode with a component equal to -N/2 is zero and belongs to no bin; k = 0 belongs
 *     to no bin.  Bin i holds the modes with T_i <= |n|^2 < T_{i+1},
 *     T_i = ceil(((k_i * L) / (2 pi))^2) computed in FP64.
 *   - alpha = N_data/N_randoms, I = alpha sum_r w^2 nbar, S = (sum_d w^2 + alpha^2 sum_r w^2)/I;
 *     without randoms (periodic box) nbar = N_data/L^3, I = nbar sum_d w^2, S = sum_d w^2/I.
 *
 * Memory and ownership.
 *   Every pointer argument is owned by the caller.  Host pointers are read (or written)
 *   only during the call.  Catalog arrays with on_device = 1 are device pointers on the
 *   plan's device, read on the plan's stream before the call returns.  A plan owns its
 *   device meshes; the painted field stays resident from pkm_paint until the next
 *   pkm_paint or pkm_plan_destroy, so several pkm_compute_multipoles calls may follow one
 *   paint.  Calls are synchronous with respect to the host.  A plan is not thread safe;
 *   distinct plans are independent.
 *
 * Errors.  Every function returns a pkm_status; nothing aborts or throws across the ABI.
 *   On error the outputs are untouched and pkm_plan_last_error() holds a message;
 *   pkm_plan_last_error(NULL) gives why the calling thread's last plan creation failed.
 *   PKM_EINVAL leaves the plan unchanged, except for the normalisation check of painting
 *   (pkm_paint, pkm_finish), which leaves it unpainted.  After PKM_EDEVICE the plan must be
 *   destroyed.
 */
#ifndef PKM_H
#define PKM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PKM_ABI_VERSION 4

typedef enum {
  PKM_OK = 0,
  PKM_EINVAL = 1,     /* invalid argument (plan unchanged) */
  PKM_EORDER = 2,     /* compute before paint */
  PKM_ENOMEM = 3,     /* device allocation failed or footprint above the budget */
  PKM_EDEVICE = 4,    /* HIP runtime error; destroy the plan */
  PKM_EBUSY = 5,      /* server queue full / request not finished */
  PKM_ECANCELLED = 6  /* request cancelled */
} pkm_status;

enum { PKM_NGP = 1, PKM_CIC = 2, PKM_TSC = 3 };
enum { PKM_FP32 = 0, PKM_FP64 = 1 };
enum { PKM_LOS_LOCAL = 0, PKM_LOS_GLOBAL = 1 };

/* Mesh and estimator parameters (Sec. 2.1, Sec. 2.3).
 *   nmesh        N: 2^a 3^b with a >= 2, 16 <= N <= 1024.
 *   box_len      L > 0 (cubic box [o, o + L)^3).
 *   box_origin   o.
 *   observer     position of the observer (local line of sight from it to each node).
 *   los_mode/los PKM_LOS_GLOBAL uses the unit vector `los` in pkm_kmu_global only.
 *   window       PKM_NGP | PKM_CIC | PKM_TSC.
 *   interlaced   0/1: second mesh at +1/2 cell, averaged in Fourier space.
 *   compensated  0/1: divide the combined field by the assignment window.
 *   precision    PKM_FP32 (FP32 meshes/transforms, FP64 index math and sums) or PKM_FP64.
 *   ell_max_hint largest ell_max later requested (sizes the field buffers); 0 means 4.
 *   max_group    upper bound on weighted fields kept in HBM at once; 0 = automatic.
 *   deterministic 0/1: bitwise-repeatable estimates.  Painting then rounds every tap to a
 *                multiple of 1/s of one fixed-point scale s shared by all tiles (chosen per
 *                paint so that no node's sum can exceed 2^60 / s) and sums the integers in
 *                LDS and in 64-bit accumulators (8 N^3 bytes per mesh, allocated with the
 *                plan), so no floating-point addition depends on scheduling; the post-pass
 *                keeps one histogram per wavefront (PKM_ENOMEM when that does not fit LDS).
 *                Slower; the environment variable PKM_DETERMINISTIC=1 turns it on for
 *                every plan.  pkm_kmu_global is not covered.                              */
typedef struct {
  int32_t nmesh;
  double box_len;
  double box_origin[3];
  double observer[3];
  int32_t los_mode;
  double los[3];
  int32_t window;
  int32_t interlaced;
  int32_t compensated;
  int32_t precision;
  int32_t ell_max_hint;
  int32_t max_group;
  int32_t deterministic;
} pkm_params;

/* A catalog: n objects, positions pos[3*i + a] (FP64, absolute coordinates), optional
 * weights w[i] (NULL -> 1) and number densities nbar[i] (required for randoms).
 * on_device = 1: the three pointers are device pointers on the plan's device.
 * One estimate takes at most PKM_MAX_PARTICLES data + random objects (2^31 - 2^16): the
 * painting sort keeps per-tile counts, offsets and ranks in 32-bit integers.  Larger
 * catalogs are rejected with PKM_EINVAL before anything is allocated or copied.            */
#define PKM_MAX_PARTICLES ((int64_t)2147418112)
typedef struct {
  const double* pos;
  const double* w;
  const double* nbar;
  int64_t n;
  int32_t on_device;
} pkm_catalog;

/* Result of pkm_compute_multipoles.  The caller allocates:
 *   poles   (ell_max/2 + 1) x (n_edges - 1) doubles, row l/2 holds P_l;
 *   k_mean  n_edges - 1 doubles (mean |k| of the bin's modes, NaN if empty);
 *   n_modes n_edges - 1 counts (full-sphere modes).
 * Any of the three may be NULL.  The scalars are filled by the call.                      */
typedef struct {
  double* poles;
  double* k_mean;
  int64_t* n_modes;
  double alpha;
  double norm_I;
  double shot_noise;
  int32_t n_transforms;
} pkm_result;

/* Device, stream and optional allocator.  hip_stream is a hipStream_t (NULL = default
 * stream).  alloc/free may route device allocations through a caller's allocator (e.g. a
 * framework's caching allocator); NULL selects hipMalloc/hipFree.                          */
typedef struct {
  int32_t device_id;
  void* hip_stream;
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, void* stream, void* ctx);
  void* alloc_ctx;
} pkm_device;

/* Kernel stages reported by pkm_stats (stage_ms / stage_launches index). */
enum {
  PKM_STAGE_SUMS = 0,      /* catalog reductions */
  PKM_STAGE_FILL = 1,      /* mesh zeroing */
  PKM_STAGE_PAINT = 2,     /* mass assignment */
  PKM_STAGE_ZFWD = 3,      /* forward z of the painted meshes */
  PKM_STAGE_YCOL = 4,      /* forward y column passes (painted meshes and weighted fields) */
  PKM_STAGE_XCOMBINE = 5,  /* x pass + interlace combine + compensation + inverse x */
  PKM_STAGE_IYCOL = 6,     /* inverse y pass of the combined field */
  PKM_STAGE_ZPRE = 7,      /* inverse z to D_c + Y_lm(xhat) weighting + forward z per field */
  PKM_STAGE_XPOST = 8,     /* forward x per field + sum_m Y_lm(khat) B + product with C + binning */
  PKM_STAGE_REDUCE = 9,    /* fixed-order reduction of the bin partial sums */
  PKM_NSTAGES = 10
};

/* Per-plan counters.  stage_ms / stage_launches accumulate (since the last pkm_reset_stats)
 * only while stage timing is enabled (pkm_set_stage_timing), from HIP events recorded on
 * the plan's stream around every launch. */
typedef struct {
  int64_t device_bytes;      /* device memory held by the plan */
  int32_t n_transforms;      /* transforms of the last paint + compute */
  int32_t n_groups;          /* field groups of the last compute */
  double ms_paint;           /* device time of the last pkm_paint */
  double ms_compute;         /* device time of the last pkm_compute_multipoles */
  double model_bytes_paint;  /* algorithmic HBM bytes of the last paint */
  double model_bytes_compute;/* algorithmic HBM bytes of the last compute */
  double stage_ms[10];
  int64_t stage_launches[10];
} pkm_stats_t;

typedef struct pkm_plan pkm_plan;

/* Launch shape of the passes.  A zero field keeps the built-in choice for the mesh size and
 * precision.  e_col / e_z / e_post are elements per thread of the length-N column passes,
 * the length-N/2 z passes and the post-pass (4, 6, 8, 12 or 16 with a radix schedule for
 * the length); tile is columns per block of the column passes; tile_post is y lines (one per
 * kz) per post-pass tile; zlines is z lines per block (a divisor of N); paint_tile is the
 * painting tile side (4, 8, 16); post_axis names the last transform axis of the weighted
 * fields, the axis + 1: the fields are stored kz-major ([kz][x][y]) and finish along y, so
 * only 0 (default) and 2 are accepted.  A shape that breaks a kernel limit (threads per
 * block, LDS bytes, divisibility) is rejected with PKM_EINVAL.                             */
typedef struct {
  int32_t e_col, tile, e_z, zlines, e_post, tile_post, paint_tile, post_axis;
} pkm_shape;

int pkm_abi_version(void);
const char* pkm_status_str(pkm_status s);

/* Host-only check of a data / randoms pair as pkm_paint, pkm_enqueue and pkm_batch_add take
 * it (Sec. 2.1 eq. FKP-density: data non-empty; randoms NULL for a periodic box, else
 * non-empty with n-bar; n >= 0; positions present; at most PKM_MAX_PARTICLES objects in
 * all).  Reads only the structs, never the arrays; no device access.  PKM_OK or
 * PKM_EINVAL.                                                                               */
pkm_status pkm_check_catalogs(const pkm_catalog* data, const pkm_catalog* randoms);

/* Validate the parameters, build twiddle / harmonic / compensation tables and allocate the
 * plan's device buffers.  *out is set only on success.                                     */
pkm_status pkm_plan_create(const pkm_params* p, const pkm_device* dev, pkm_plan** out);

/* pkm_plan_create with a launch shape (NULL = built-in); pkm_plan_shape reports the shape a
 * plan runs with (every field filled in).                                                   */
pkm_status pkm_plan_create_shaped(const pkm_params* p, const pkm_device* dev, const pkm_shape* shape,
                                  pkm_plan** out);
pkm_status pkm_plan_shape(const pkm_plan* plan, pkm_shape* out);

/* Device bytes a plan with these parameters would hold for one estimate of ell_max over
 * n_edges k edges with n_particles objects (meshes, weighted fields, particle sort buffers,
 * partial sums; an upper estimate, the figure the serving loop admits requests by).  Host
 * only; -1 when the parameters are invalid.                                                 */
int64_t pkm_plan_footprint(const pkm_params* p, int32_t ell_max, int32_t n_edges, int64_t n_particles);

/* Autotuner: times candidate launch shapes on a seeded synthetic catalog of n_particles
 * objects (1/21 data, 20/21 randoms, uniform in the box) for estimates up to ell_max, one
 * group of passes at a time (painting tile, z passes, column passes, post-pass and its
 * axis), each candidate `reps` times after one warm-up, keeping the fastest per group.
 * Writes the chosen shape, the device time of one estimate with it and with the built-in
 * shape (ms; either pointer may be NULL).  Synchronous; creates and frees its own plans.   */
pkm_status pkm_autotune(const pkm_params* p, const pkm_device* dev, int32_t ell_max, int64_t n_particles,
                        int32_t reps, pkm_shape* best, double* best_ms, double* default_ms);

/* Sec. 2.1 (eq. FKP-density) and Sec. 2.3: catalog scalars, painting of data minus
 * alpha x randoms (randoms NULL -> periodic box), forward transforms, interlace combine,
 * compensation, and the inverse transform of the combined field.  Replaces any previous
 * paint of this plan.  The estimate divides by the normalisation I = alpha sum_r n-bar w^2
 * (n-bar sum_d w^2 in a periodic box): when I is not positive (every random weight or n-bar
 * zero, or every data weight in a periodic box), PKM_EINVAL and the plan is left unpainted
 * (PKM_EORDER until the next successful paint).                                            */
pkm_status pkm_paint(pkm_plan* plan, const pkm_catalog* data, const pkm_catalog* randoms);

/* Sec. 2.1 eq. Pell-ours / eq. Fell, binned as in Sec. 2.2 (uniform or arbitrary increasing
 * k edges, n_edges >= 2, edges >= 0): every even l <= ell_max (ell_max even, 0..16).
 * Requires a prior pkm_paint (else PKM_EORDER).                                           */
pkm_status pkm_compute_multipoles(pkm_plan* plan, int32_t ell_max, const double* k_edges, int32_t n_edges,
                                  pkm_result* out);

/* The same multipoles through either decomposition of L_l(khat . xhat) named in Sec. 2.1:
 *   PKM_BASIS_SPHERICAL  the addition theorem (eq. add-theorem, eq. Fell): 2l+1 transforms
 *                        per l; identical to pkm_compute_multipoles.
 *   PKM_BASIS_CARTESIAN  the Cartesian decomposition the paper compares against: L_l is
 *                        expanded in powers (khat . xhat)^p and each power into monomials,
 *                        (p+1)(p+2)/2 transforms per even degree p >= 2, shared by every l
 *                        (22 transforms in all for l <= 4, 525 for l <= 16, against 15 and
 *                        153).  The degree sums are combined with the Legendre coefficients
 *                        on the host in FP64; the cancellation among those coefficients
 *                        (their absolute sum is 8.5 at l = 4 and 1.7e5 at l = 16)
 *                        multiplies the rounding error of the FP32 form by as much.
 * Arguments, outputs and errors as pkm_compute_multipoles; other basis values: PKM_EINVAL.
 * out->n_transforms counts the transforms of the chosen basis.                              */
#define PKM_BASIS_SPHERICAL 0
#define PKM_BASIS_CARTESIAN 1
pkm_status pkm_compute_multipoles_basis(pkm_plan* plan, int32_t ell_max, const double* k_edges, int32_t n_edges,
                                        int32_t basis, pkm_result* out);

/* Every multipole l = 0 .. ell_max (ell_max 0..16), odd l included, through the spherical-
 * harmonic decomposition of eq. Fell: 2l+1 transforms per l > 0, (ell_max+1)^2 - 1 in all.
 * The paper treats even l only (odd ones vanish under a single line of sight, Sec. 1); with
 * the local line of sight of eq. Pell-ours the odd shell averages do not vanish but are purely
 * imaginary: a mode and its mirror contribute with L_l(-x) = -L_l(x), and their real parts
 * cancel.  out->poles has (ell_max + 1) x (n_edges - 1) doubles, row l:
 *   even l: P_l as pkm_compute_multipoles (shot noise subtracted at l = 0);
 *   odd l:  R_l = Im P_l of eq. Pell-ours with the paper's exponent exp(+i k.r) in eq. Fell,
 *           i.e. (2l+1)/(I N_i) sum_bin Im[C conj A_l] with the forward transforms exp(-i k.x)
 *           used here; no shot-noise term.  (Eq. Pell-yama, whose second integral is
 *           conj F_l(k) rather than F_l(-k), equals eq. Pell-ours for even l and is -i R_l for
 *           odd l.)
 * k_mean, n_modes, the scalars and errors as pkm_compute_multipoles; out->n_transforms counts
 * the odd fields too.  Synchronous only (the asynchronous, batch and serving paths take even
 * l).                                                                                       */
pkm_status pkm_compute_multipoles_all(pkm_plan* plan, int32_t ell_max, const double* k_edges, int32_t n_edges,
                                      pkm_result* out);

/* Fixed line of sight (the plan's `los`): P(k_i, mu_j) = sum |C|^2 / (I N_ij) - S over the
 * modes with mu = |khat . los| in [mu_j, mu_{j+1}) (mu = 1 in the last bin).  Outputs are
 * (n_k_edges-1) x (n_mu_edges-1), row-major by k; either may be NULL.                      */
pkm_status pkm_kmu_global(pkm_plan* plan, const double* k_edges, int32_t n_k_edges, const double* mu_edges,
                          int32_t n_mu_edges, double* pkmu_out, int64_t* nmodes_out);

/* pkm_kmu_global for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same (k, mu) cells,
 * arguments, outputs and errors, but no device or pinned allocation and no free.  Its
 * thresholds, mu edges, per-block partial sums and results live in one fixed device array
 * of 12.7 MB per device (each device the library runs on holds it until the process ends).
 * At most 3072 (k, mu) cells, as for pkm_kmu_global; more is PKM_EINVAL.  Every call on one
 * device shares that array: calls that overlap on one device (from several threads, or on
 * plans with different streams) race and must be serialised by the caller.  The cells' sums
 * are accumulated over 256 blocks instead of pkm_kmu_global's 1024, so the two agree to
 * FP64 rounding (counts exactly).  Synchronous, like pkm_kmu_global.                      */
pkm_status pkm_kmu_global_noalloc(pkm_plan* plan, const double* k_edges, int32_t n_k_edges, const double* mu_edges,
                                  int32_t n_mu_edges, double* pkmu_out, int64_t* nmodes_out);

/* Sec. 2.2 eq. wedge-est with eq. Lbar, host only, FP64:
 *   wedges_out[i*(n_mu_edges-1) + j] = sum_{even l <= ell_max} poles[(l/2)*n_k + i] Lbar_l(mu_j, mu_{j+1}).
 * mu edges strictly increasing in [0, 1].                                                   */
pkm_status pkm_wedges(const double* poles, int32_t ell_max, int32_t n_k, const double* mu_edges, int32_t n_mu_edges,
                      double* wedges_out);

/* Sec. 3.1 eq. nonuniform-bins: the ell_max/2 + 2 edges (mu_0 = 0, last = 1) for which
 * every bin but the first integrates L_{ell_max+1}(mu)/mu to zero.  Host only.             */
pkm_status pkm_nonuniform_mu_edges(int32_t ell_max, double* edges_out);

/* Sec. 4.1 eq. gamma: the angular part of the Gaussian covariance of wedges reconstructed
 * from the even multipoles l <= ell_max of a linear Kaiser spectrum (1 + beta mu^2)^2 P(k),
 *   gamma_out[m*(n_mu_edges-1) + n] = sum_{l,l'} (2l+1)(2l'+1) Lbar_l(mu_m) Lbar_l'(mu_n)
 *                                     int_{-1}^{1} (dmu/2) L_l L_l' (1 + beta mu^2)^4,
 * so that cov[P(k_i, mu_m), P(k_i, mu_n)] = 2 gamma_mn P^2 / N_k (eq. trunc-Cmn), and the
 * wedge correlation matrix is gamma normalised by its diagonal.  Host only, FP64; the mu
 * integral is done by an exact Gauss rule.  mu edges strictly increasing in [0, 1],
 * ell_max even 0..64, beta finite; otherwise PKM_EINVAL.                                    */
pkm_status pkm_kaiser_wedge_gamma(int32_t ell_max, const double* mu_edges, int32_t n_mu_edges, double beta,
                                  double* gamma_out);

pkm_status pkm_stats(const pkm_plan* plan, pkm_stats_t* out);
/* Enable (1) or disable (0) per-launch event timing; pkm_reset_stats clears the sums. */
pkm_status pkm_set_stage_timing(pkm_plan* plan, int32_t enable);
pkm_status pkm_reset_stats(pkm_plan* plan);
const char* pkm_plan_last_error(const pkm_plan* plan);
void pkm_plan_destroy(pkm_plan* plan);

/* 3D transforms of the plan's size and precision on caller device buffers (the same passes
 * the estimator runs).  Forward: real N^3 mesh (x, y, z; z contiguous) -> half spectrum
 * N x N x N/2 complex (kz = 0..N/2-1; the kz = N/2 plane is not produced).  Inverse: half
 * spectrum (kz = N/2 taken as zero) -> real mesh, normalised by 1/N^3.  `in` is not modified
 * by the forward transform; the inverse overwrites `in`.                                   */
pkm_status pkm_fft3d_forward(pkm_plan* plan, const void* in_real_dev, void* out_half_dev);
pkm_status pkm_fft3d_inverse(pkm_plan* plan, void* in_half_dev, void* out_real_dev);

/* Copy a resident plan buffer to host memory (test hook):
 *   which = 0: painted mesh D1 (real N^3), 1: interlaced mesh D2 (real N^3),
 *           2: combined field C (half spectrum N x N x N/2 complex),
 *           3: D_c, the field that is harmonically weighted (real N^3).
 * bytes must equal the buffer size (N^3 or N^3 complex/2 elements of the plan precision). */
pkm_status pkm_plan_read_buffer(pkm_plan* plan, int32_t which, void* host_dst, size_t bytes);

/* ---------------------------------------------------------------------------------------
 * Asynchronous estimates.  The same computation as pkm_paint + pkm_compute_multipoles
 * (Sec. 2.1 eq. FKP-density, eq. Pell-ours, eq. Fell; Sec. 2.3), split so that the device
 * work can overlap with other plans' work or be recorded into a HIP graph.
 *
 * pkm_prepare     builds the request's host tables (k thresholds, field groups, reduce maps)
 *                 and reserves device and pinned-host buffers for up to max_particles data +
 *                 random objects.  Synchronous; may allocate.  Re-preparing with another
 *                 ell_max or other edges replaces the tables.
 * pkm_enqueue     enqueues one whole estimate (paint, transforms, multipoles, and the copy
 *                 of the bin sums to the plan's pinned staging) on the plan's stream and
 *                 returns without waiting.  Catalogs must be device-resident (on_device = 1)
 *                 and stay valid and unmodified until pkm_finish returns.  Allocates no device
 *                 memory and issues no synchronous HIP call: the enqueue may be captured into a
 *                 graph (with stage timing off; with it on, the plan's per-launch timing events
 *                 are recorded too, the first enqueues may create them, and pkm_finish adds the
 *                 times to pkm_stats).
 *                 PKM_EBUSY if a previous enqueue has not been finished; PKM_EORDER if the
 *                 plan is not prepared, or if a synchronous pkm_compute_multipoles(_basis)
 *                 with another ell_max, other edges or the Cartesian basis has replaced the
 *                 prepared request since (prepare again); PKM_EINVAL above the reserved
 *                 particle count.
 * pkm_query       PKM_OK when the enqueued estimate has completed, PKM_EBUSY while it runs.
 * pkm_finish      waits for it and normalises (FP64, host) into `out` as pkm_compute_multipoles
 *                 does for the prepared ell_max and edges.  Afterwards the plan holds the
 *                 painted field as after pkm_paint.  PKM_EINVAL (plan unpainted, `out`
 *                 untouched) when the normalisation I is not positive, as for pkm_paint.
 * pkm_paint / pkm_compute_multipoles return PKM_EBUSY between pkm_enqueue and pkm_finish.
 * ------------------------------------------------------------------------------------- */
pkm_status pkm_prepare(pkm_plan* plan, int32_t ell_max, const double* k_edges, int32_t n_edges,
                       int64_t max_particles);
pkm_status pkm_enqueue(pkm_plan* plan, const pkm_catalog* data, const pkm_catalog* randoms);
pkm_status pkm_query(pkm_plan* plan);
pkm_status pkm_finish(pkm_plan* plan, pkm_result* out);

/* ---------------------------------------------------------------------------------------
 * Batches: many estimates (e.g. a set of covariance mocks of uneven mesh size, Sec. 4.1's
 * motivation) issued as one unit.  Each item is (prepared plan, device catalogs).  Items on
 * distinct plans run concurrently on the plans' streams (each plan needs its own non-null
 * stream); items sharing a plan run in the order added.  With use_graph = 1 the first run
 * captures the whole issue sequence into a HIP graph (fork/join over the plans' streams) and
 * later runs replay it with one launch; adding an item drops the graph.  The catalogs'
 * device pointers and counts are recorded: their contents may change between runs, their
 * addresses and sizes may not.  Plans in a batch must not be re-prepared or used directly
 * while the batch holds them: a run checks every item's plan first and, if the plan's
 * buffers or request tables changed since the item was added, drops the graph, issues
 * nothing and returns PKM_EORDER (add the items again).
 *   pkm_batch_run    issues (or replays) every item, waits, and reports the device time
 *                    from the fork to the join in *ms_out (may be NULL).
 *   pkm_batch_result normalises item `index` of the last run into `out` (FP64, host);
 *                    PKM_EINVAL, `out` untouched, when the item's normalisation I is not
 *                    positive (as for pkm_paint).
 * ------------------------------------------------------------------------------------- */
typedef struct pkm_batch pkm_batch;
pkm_status pkm_batch_create(int32_t device_id, pkm_batch** out);
pkm_status pkm_batch_add(pkm_batch* batch, pkm_plan* plan, const pkm_catalog* data, const pkm_catalog* randoms,
                         int32_t* index_out);
pkm_status pkm_batch_run(pkm_batch* batch, int32_t use_graph, double* ms_out);
pkm_status pkm_batch_result(pkm_batch* batch, int32_t index, pkm_result* out);
int32_t pkm_batch_size(const pkm_batch* batch);
const char* pkm_batch_last_error(const pkm_batch* batch);
void pkm_batch_destroy(pkm_batch* batch);

/* ---------------------------------------------------------------------------------------
 * Serving: a request loop on one device.  A request names mesh parameters, ell_max, k edges
 * and its catalogs: host arrays copied at submit, or a catalog registered with the server
 * (device copies that stay resident until unregistered).  Requests are admitted from the first
 * 8 queued ones in arrival order: the first whose footprint fits hbm_budget_bytes (idle plans
 * evicted least recently used first) while fewer than max_inflight estimates run, so a request
 * blocked on memory does not hold back smaller ones behind it; once the oldest request has been
 * passed 16 times, nothing else is admitted before it.  Admission also keeps the device's own
 * free memory, after the request, at 2 GiB or 1% of the device (the larger) for the runtime's
 * kernel scratch, evicting idle plans and releasing the pool's kept blocks first, else waiting.
 * A request that cannot fit even with no plan resident fails with PKM_ENOMEM.  Admitted requests run on separate streams and overlap
 * on the device; plans (meshes, tables, staging) stay resident and are reused by later requests
 * with the same mesh, box, observer, window, precision and max_group.  A plan keeps the painted
 * field of the registered catalog it served last: a later request for that catalog on that plan
 * skips the paint and the catalog copy and computes the multipoles of the field it holds (Sec.
 * 2.1: every F_l is built from the one painted field by 2l+1 transforms).  Results are computed exactly as by
 * pkm_paint + pkm_compute_multipoles.  Plan memory comes from the device's stream-ordered pool
 * (hipMallocAsync/hipFreeAsync on the plan's stream).
 *   pkm_server_register_catalog   copies data (and randoms, NULL for none) to the device and
 *                      returns an id > 0 (PKM_EINVAL as pkm_check_catalogs; PKM_ENOMEM when
 *                      it does not fit the budget next to the running plans).  Its bytes
 *                      count in resident_bytes until it is unregistered.
 *   pkm_server_unregister_catalog frees it; PKM_EBUSY while queued or running requests name
 *                      it, PKM_EINVAL for an unknown id.  Ids are never reused.
 *   pkm_server_submit  queues a request and returns its ticket (PKM_EINVAL on bad input).
 *   pkm_server_poll    PKM_EBUSY until the request has finished, then copies the result
 *                      into `out` (arrays sized as for pkm_compute_multipoles) once.  A
 *                      request whose normalisation I is not positive fails with PKM_EINVAL.
 *   pkm_server_wait    blocks until then.
 *   pkm_server_stats   completed / failed / queued / in-flight counts, resident and peak
 *                      device bytes, the largest number of concurrent estimates seen,
 *                      latency percentiles (submit to completion, ms) over all requests and
 *                      per precision, throughput, requests served from a held painted field,
 *                      registered catalogs and their bytes.
 *   pkm_server_reset_stats  starts the statistics afresh (counts, latencies, the largest
 *                      concurrency, the peak bytes and the throughput window); requests
 *                      in flight when it is called count when they finish.
 *   pkm_server_destroy finishes the requests in flight, cancels queued ones, frees all
 *                      (registered catalogs included).
 * The server functions are thread safe.
 * ------------------------------------------------------------------------------------- */
typedef struct {
  int32_t device_id;
  int64_t hbm_budget_bytes;  /* admission budget; <= 0 selects 80% of the free memory */
  int32_t max_inflight;      /* concurrent estimates, 1..32 */
  /* Device allocations of plans and catalog buffers (not of registered catalogs), as in
   * pkm_device, called on the worker thread with the plan's stream.  Both NULL selects the
   * stream-ordered pool; a NULL return fails that request alone with PKM_ENOMEM. */
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, void* stream, void* ctx);
  void* alloc_ctx;
  /* > 0: requests that leave max_group at 0 get max_group = field_group and ell_max_hint = 16,
   * so one plan per mesh configuration serves every ell_max (a request with more fields than
   * field_group runs its groups one after another) and plans stop being re-created as ell_max
   * changes.  0: plans follow each request's own max_group and ell_max_hint.  At most 256. */
  int32_t field_group;
} pkm_server_config;

typedef struct {
  pkm_params params;         /* ell_max_hint and max_group are taken from here */
  int32_t ell_max;           /* even, 0..16 */
  const double* k_edges;
  int32_t n_edges;
  pkm_catalog data;          /* host arrays (on_device = 0); ignored when catalog_id != 0 */
  pkm_catalog randoms;       /* host arrays, used when has_randoms = 1 (nbar required) */
  int32_t has_randoms;       /* ignored when catalog_id != 0 */
  uint64_t catalog_id;       /* a registered catalog, or 0 for the host catalogs above */
} pkm_request;

typedef struct {
  int64_t completed, failed, queued, inflight;
  int64_t resident_plans, resident_bytes, peak_bytes;
  int32_t max_concurrent;
  double latency_p50_ms, latency_p99_ms, latency_mean_ms;
  double throughput_per_s;   /* completed requests / (last completion - first submit) */
  int64_t completed_fp32, completed_fp64;
  double latency_p50_ms_fp32, latency_p99_ms_fp32, latency_p50_ms_fp64, latency_p99_ms_fp64;
  int64_t mesh_reuses;       /* requests served from a painted field their plan held */
  int64_t registered_catalogs, registered_bytes;
} pkm_server_stats_t;

typedef struct pkm_server pkm_server;
pkm_status pkm_server_create(const pkm_server_config* cfg, pkm_server** out);
pkm_status pkm_server_register_catalog(pkm_server* server, const pkm_catalog* data, const pkm_catalog* randoms,
                                       uint64_t* catalog_id);
pkm_status pkm_server_unregister_catalog(pkm_server* server, uint64_t catalog_id);
pkm_status pkm_server_submit(pkm_server* server, const pkm_request* request, int64_t* ticket);
pkm_status pkm_server_poll(pkm_server* server, int64_t ticket, pkm_result* out);
pkm_status pkm_server_wait(pkm_server* server, int64_t ticket, pkm_result* out);
pkm_status pkm_server_stats(pkm_server* server, pkm_server_stats_t* out);
pkm_status pkm_server_reset_stats(pkm_server* server);
const char* pkm_server_last_error(const pkm_server* server);
void pkm_server_destroy(pkm_server* server);

#ifdef __cplusplus
}
#endif

#endif /* PKM_H */
