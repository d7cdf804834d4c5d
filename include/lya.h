/*
 * lya.h -- C ABI of the MI355X Lyman-alpha pair-accumulation library.
 *
 * The library computes, on one AMD Instinct MI355X (gfx950):
 *   - the weighted pixel-pair sums behind the two-point estimator
 *       xi_A = sum_A delta_i w_i delta_j w_j / sum_A w_i w_j
 *     over every pair of pixels (i, j) from different forests whose
 *     separation (r_par, r_perp) lies in the rectangular bin A
 *     (arXiv:2507.00129, Sec. 2.1, eq. estimator_two);
 *   - the distortion matrix D_AB = w_A^-1 sum_{ij in A} w_i w_j
 *       sum_{i'j' in B} eta_ii' eta_jj'
 *     with eta the per-forest continuum projection built from w and
 *     Lambda = log(lambda) (Sec. 2.2, eq. distortion and the eta definition);
 *   - the gradient of xi with respect to delta and w for a caller-supplied
 *     dL/dxi, also through the continuum projection;
 *   - the pair sums split by subsample and the subsample covariance of xi,
 *     and the weighted bin-mean r_par, r_perp and z of each bin;
 *   - the triplet sums of the anisotropic three-point function
 *     xi3_A = sum_A w_i d_i w_j d_j w_k d_k / sum_A w_i w_j w_k over pixels of
 *     three distinct forests (Sec. 2.3, eq. estimator_three), also split by
 *     subsample;
 *   - optionally (lya_options.deterministic), xi sums that are bitwise
 *     reproducible and identical for a realisation alone or batched.
 *
 * Geometry.  Forest f has a sky direction n_f (from ra, dec).  With
 * s = |n_f - n_g| / 2 = sin(theta/2) and c = sqrt(1 - s^2), a pixel pair at
 * comoving distances D_i, D_j has r_par = |D_i - D_j| c and
 * r_perp = (D_i + D_j) s.  Bins are half-open, [e_k, e_{k+1}) on both axes;
 * a pair is in the grid iff both axes are.  The flat bin index is
 * A = k_par * n_perp + k_perp.  Pairs are unordered: each pixel pair from two
 * different forests of the same realisation is counted once.
 *
 * Memory.  Every pointer in lya_forests and every output pointer is a DEVICE
 * pointer on the device the context was created for; the grid edges are HOST
 * pointers.  All memory is owned by the caller; the library never frees
 * caller memory and keeps no caller pointer after the call returns.  Work is
 * enqueued on the caller's stream (a hipStream_t passed as void*, NULL = the
 * default stream); each call synchronises that stream a few times to size
 * its work lists, and returns once all of its work has been enqueued.
 * Outputs are fully overwritten (the library zeroes them first).
 *
 * Errors.  Every call returns a status; nothing aborts and nothing throws.
 * Arguments are checked before any work is enqueued; with
 * lya_options.validate set, array contents are checked on the device too
 * (offsets, finiteness, signs, realisation ids).  lya_last_error() returns a
 * human-readable message for the last failure on a context.
 *
 * Threading.  A context may be used by one host thread at a time.  Two
 * contexts may run concurrently.  The calls of one context share its device
 * workspace: a call enqueued on another stream than the previous one must
 * not run before the previous call's work has finished.
 */
#ifndef LYA_H
#define LYA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LYA_OK = 0,
  LYA_E_INVALID = 1,     /* bad argument or bad array contents */
  LYA_E_NOMEM = 2,       /* device workspace allocation failed */
  LYA_E_DEVICE = 3,      /* a HIP call failed */
  LYA_E_UNSUPPORTED = 4  /* valid input this build cannot handle (see message) */
} lya_status;

typedef enum {
  /* Pair geometry and products in FP32 (distances re-centred so that
     FP32 keeps ~1e-4 Mpc/h); pairs within rounding of a bin edge are re-binned
     in FP64, so binning equals the FP64 decision.  xi: runs of at most 32
     same-bin FP32 products are summed in FP32 registers and the run sums are
     accumulated in FP64 (LDS, then global) -- FP64 accumulation, not a
     compensated FP32 sum.  D: the row histograms and the row contraction are
     FP32, accumulated in FP32 over a run of forest pairs and then added to
     FP64 totals.  Per-forest projection sums and the final normalisation
     are FP64. */
  LYA_FP32_COMP = 0,
  /* Everything in FP64. */
  LYA_FP64 = 1
} lya_precision;

typedef enum {
  LYA_ETA_IDENTITY = 0,   /* eta = I */
  LYA_ETA_MEAN = 1,       /* eta_ii' = delta_ii' - w_i'/W_f */
  LYA_ETA_MEAN_SLOPE = 2  /* ... - (L_i - Lbar) w_i' (L_i' - Lbar) / S_f   (Sec. 2.2) */
} lya_eta;

/* Forests in CSR layout (Sec. 3.1: one sky position and a variable-length
   table of delta, w and lambda per forest).  Pixels of forest f are
   offsets[f] .. offsets[f+1]-1. */
typedef struct {
  int64_t n_forests;          /* >= 0 */
  int64_t n_pix;              /* == offsets[n_forests] (checked when validating) */
  const int64_t *offsets;     /* [n_forests + 1], offsets[0] == 0, non-decreasing */
  const double *ra;           /* [n_forests] right ascension, radians */
  const double *dec;          /* [n_forests] declination, radians */
  const double *dist;         /* [n_pix] comoving distance, Mpc/h, > 0 */
  const double *delta;        /* [n_pix] flux fluctuation */
  const double *weight;       /* [n_pix] >= 0; w = 0 masks a pixel out */
  const double *loglam;       /* [n_pix] log(lambda), any base (eta only) */
  const int32_t *realisation; /* [n_forests] in [0, n_realisations), or NULL (all 0) */
  int32_t n_realisations;     /* >= 1; outputs are stacked per realisation */
} lya_forests;

/* Bin edges (HOST pointers), strictly increasing, finite, edges[0] >= 0;
   bins are half-open, [e_k, e_k+1) (Sec. 2.1).  Edges uniformly spaced on both
   axes (to 1e-9 of a bin) are binned from floor((r - e_0) / dr) with an FP64
   edge guard; any other edges are binned by searching the FP64 edge arrays
   for every pair in range (same results, slower).  n_par * n_perp <= 4096. */
typedef struct {
  int32_t n_par;
  int32_t n_perp;
  const double *edges_par;   /* [n_par + 1] */
  const double *edges_perp;  /* [n_perp + 1] */
} lya_grid;

typedef struct {
  int32_t precision;          /* lya_precision */
  int32_t eta;                /* lya_eta: projection used by lya_dmat and project_deltas */
  int32_t project_deltas;     /* lya_xi: replace delta by eta delta per forest first */
  int32_t autotune;           /* pick kernel variants by timing them on this input */
  int32_t validate;           /* check array contents on the device (one extra sync) */
  int32_t timing;             /* record per-stage device times (see lya_stats) */
  int32_t variant;            /* >= 0 forces that kernel variant; -1 lets the
                                 autotuner (or the default) choose */
  int32_t counters;           /* lya_dmat: count the work done (in-grid pairs,
                                 outer-product FMAs, out-of-window pairs; see
                                 lya_stats); adds a little work to the kernel */
  double dmat_keep_fraction;  /* lya_dmat: keep forest pair (f<g) iff
                                 splitmix64(seed ^ (f<<32 | g)) < floor(p * 2^64);
                                 p in (0, 1], p = 1 keeps all (Sec. 2.2: D on a
                                 subset of forest pairs) */
  uint64_t seed;
  int32_t deterministic;      /* lya_xi: bitwise-reproducible sums, independent of
                                 the order the GPU adds pairs in, and identical
                                 for a realisation run alone or batched with
                                 others.  Runs of at most 32 same-bin products
                                 w d w d (and w w) of one pixel against
                                 consecutive pixels of the other forest are
                                 summed in a fixed order in the precision's
                                 arithmetic, scaled by 2^s_r and rounded to an
                                 integer q, |q| <= 2^55, with s_r per
                                 realisation from the largest |w d| and w of
                                 its pixels; the integers are summed exactly
                                 (two 64-bit words) and N, W converted to FP64
                                 at the end.  The rounding adds at most
                                 2^-49 max|w d|^2 (max w^2) per run.  Needs
                                 fewer than 2^36 pairs per bin and realisation
                                 (LYA_E_UNSUPPORTED otherwise); one fixed kernel
                                 variant.  The other calls return
                                 LYA_E_UNSUPPORTED when it is set. */
} lya_options;

/* What the last call on a context did. */
typedef struct {
  int64_t forest_pairs;       /* unordered forest pairs in the work list */
  int64_t work_items;         /* persistent-kernel work items */
  int64_t candidate_pairs;    /* pixel pairs of the listed forest pairs (sum n_f n_g) */
  int32_t variant;            /* kernel variant index used for the main kernel */
  int32_t grid_blocks;        /* persistent workgroups launched */
  /* device milliseconds per stage, filled when options.timing != 0 */
  float ms_precompute, ms_worklist, ms_main, ms_finalize;
  /* lya_dmat with options.counters != 0: pixel pairs inside the grid over the
     kept forest pairs, and multiply-adds spent on the row outer products and
     on the H (x) Q term (the algorithmic work of the factorised form) */
  int64_t ingrid_pairs;
  int64_t outer_fmas;
  /* lya_dmat with options.counters != 0: in-grid pixel pairs that fell outside
     their forest pair's precomputed r_perp window (a consistency check: 0) */
  int64_t lost_pairs;
} lya_stats;

typedef struct lya_context lya_context;

/* Fills *opts with defaults: FP32_COMP, MEAN_SLOPE, no projection,
   autotune on, validate on, timing off, variant -1, keep fraction 1, seed 0,
   deterministic off. */
void lya_options_default(lya_options *opts);

/* Creates a context bound to HIP device `device`.  The context owns a
   grow-only device workspace and the autotuner's cache. */
lya_status lya_create(lya_context **ctx, int device);
void lya_destroy(lya_context *ctx);
/* Message of the last failure on ctx; with ctx == NULL, the message of the
   last lya_create that failed on the calling thread ("NULL context" if
   none). */
const char *lya_last_error(const lya_context *ctx);
lya_status lya_last_stats(const lya_context *ctx, lya_stats *out);

/* Pair sums and xi (Sec. 2.1, eq. estimator_two).  Outputs, each
   [n_realisations * n_bins] row-major by realisation, device:
     num[A]    = sum_A w_i delta_i w_j delta_j
     wsum[A]   = sum_A w_i w_j
     npairs[A] = number of pixel pairs in A (any weight)
     xi[A]     = num[A] / wsum[A], 0 where wsum[A] == 0   (may be NULL)
   With project_deltas, delta is first replaced per forest by eta delta
   (eta of options.eta). */
lya_status lya_xi(lya_context *ctx, const lya_forests *forests, const lya_grid *grid,
                  const lya_options *opts, void *stream,
                  double *num, double *wsum, int64_t *npairs, double *xi);

/* Size of the device array that lya_xi_noalloc works in (64 MiB per GPU). */
#define LYA_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* lya_xi for callers that cannot allocate device memory: code that must not
   call hipMalloc (inside a stream capture, a tight serving loop, a harness
   that forbids allocation).  Same arguments, outputs, options and errors as
   lya_xi.  The work space (per-forest sums, packed pixel records, sky index,
   neighbour lists, work items, sort buffers) is taken from a fixed device
   array of LYA_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it
   runs on until the process ends (its address is looked up once per device,
   in lya_create); the call allocates no device or pinned memory.  An input
   whose work space does not fit returns LYA_E_UNSUPPORTED with the size in
   the message (the outputs are then unspecified); as a guide, ~1e6 pixels
   with ~8e6 forest pairs fit.  The autotuner is not run: options.variant >= 0
   forces a variant, otherwise a variant the context has already tuned for
   this shape, else the default.  All calls on one GPU share that GPU's array
   and everything they need in it is rewritten by each call: calls that
   overlap on one GPU (two threads, two contexts, or two streams with no
   ordering between the calls) race and give wrong results. */
lya_status lya_xi_noalloc(lya_context *ctx, const lya_forests *forests, const lya_grid *grid,
                          const lya_options *opts, void *stream,
                          double *num, double *wsum, int64_t *npairs, double *xi);

/* lya_xi plus the weighted bin-mean coordinates of the pairs, the r_par,
   r_perp and z columns that the paper's output carries next to xi for the
   model fit (Sec. 3.1: the PICCA-format output read by Vega).  Extra outputs,
   each [n_realisations * n_bins], device:
     rpar[A]  = sum_A w_i w_j r_par / wsum[A]
     rperp[A] = sum_A w_i w_j r_perp / wsum[A]
     z[A]     = sum_A w_i w_j (z_i + z_j) / 2 / wsum[A]
   (0 where wsum[A] == 0), with the pixel redshift z_i = lambda_i / 1215.67 - 1
   and lambda_i = exp(loglam_i) Angstrom: for z, loglam must be the NATURAL
   log of the wavelength in Angstrom (the other outputs accept any base).
   In the FP32 form the coordinates come from the FP32 bin coordinates that
   the binning computes, so their error is that of the separations (about
   1e-4 Mpc/h), not of the FP64 form. */
lya_status lya_xi_means(lya_context *ctx, const lya_forests *forests, const lya_grid *grid,
                        const lya_options *opts, void *stream,
                        double *num, double *wsum, int64_t *npairs, double *xi,
                        double *rpar, double *rperp, double *z);

/* Pair sums split by subsample, for the subsampling covariance of xi (the
   paper estimates the errors from subsamples of the forests in sky pixels,
   Sec. 2.1 and the 3PCF figure).  subsample[f] in [0, n_sub) (device,
   [n_forests], e.g. the sky pixel of forest f); each unordered pixel pair of
   forests f, g is credited to the subsample of the one with the smaller input
   index.  Outputs as lya_xi, each [n_realisations * n_sub * n_bins] row-major
   (realisation, subsample, bin); summing over subsamples gives lya_xi's sums.
   An id outside [0, n_sub) returns LYA_E_INVALID before anything is written
   beyond the zeroed outputs. */
lya_status lya_xi_subsamples(lya_context *ctx, const lya_forests *forests, const lya_grid *grid,
                             const lya_options *opts, void *stream,
                             const int32_t *subsample, int32_t n_sub,
                             double *num, double *wsum, int64_t *npairs, double *xi);

/* Subsample covariance of xi from one realisation's [n_sub * n_bins] sums
   (device, as written by lya_xi_subsamples):
     xi[A]     = N_A / W_A with N_A, W_A summed over subsamples (0 if W_A == 0)
     cov[A][B] = sum_s W_sA W_sB (xi_sA - xi_A)(xi_sB - xi_B) / (W_A W_B)
               = sum_s (N_sA - W_sA xi_A)(N_sB - W_sB xi_B) / (W_A W_B),
   0 where W_A W_B == 0.  Outputs device, xi [n_bins], cov [n_bins * n_bins]. */
lya_status lya_xi_covariance(lya_context *ctx, const double *num, const double *wsum,
                             int64_t n_sub, int64_t n_bins, void *stream,
                             double *xi, double *cov);

/* Bins of the anisotropic three-point function (HOST pointers).  A triangle
   is seen from a main vertex i by its sides r1 = x_j - x_i, r2 = x_k - x_i
   (x = D n): side lengths on r_edges (uniform, r_edges[0] >= 0, half-open,
   r >= r_max outside), the angles theta1, theta2 of the sides to the line of
   sight of the vertex's quasar on theta_edges (strictly increasing within
   [0, pi], any spacing), and the cosine of the inner angle on cos_edges
   (uniform within [-1, 1], n_cos <= 256); theta and cos bins are half-open
   with the last one closed.  Flat index
     A = (((k_r1 n_r + k_r2) n_cos + k_cos) n_theta + k_theta1) n_theta + k_theta2
   (the order of the paper's 3PCF figure), n_bins = n_r^2 n_cos n_theta^2 <= 2^30. */
typedef struct {
  int32_t n_r;
  int32_t n_theta;
  int32_t n_cos;
  const double *r_edges;      /* [n_r + 1] */
  const double *theta_edges;  /* [n_theta + 1], radians */
  const double *cos_edges;    /* [n_cos + 1] */
} lya_grid3;

/* Triplet sums of the anisotropic 3PCF (Sec. 2.3, eq. estimator_three) over
   triplets of pixels from three distinct forests of one realisation, every
   vertex and both side orders entered (six entries per unordered triplet; a
   side of zero length is left out).  Always FP64 (options.precision is
   ignored); project_deltas / eta as for lya_xi.  Outputs, each
   [n_realisations * n_bins], device:
     num[A]   = sum_A w_i d_i w_j d_j w_k d_k
     wsum[A]  = sum_A w_i w_j w_k
     ntrip[A] = number of entries in A (any weight)
     xi[A]    = num[A] / wsum[A], 0 where wsum[A] == 0   (may be NULL)
   Three kernels: variant 0 sums each vertex pixel's entries in LDS per (r,
   theta) cell of the first side before adding them to the global sums
   (grids with n_r n_theta <= 1024 and n_cos n_theta <= 2048, up to 2048
   partner pixels per vertex); variant 2 does the same with the partner list
   in a device scratch (up to 32768 partners); variant 1 adds every entry to
   the global sums (up to 3072 partners, any grid).  options.variant = -1
   takes variant 0 where the grid allows, else 1, and re-runs the call with
   variant 2 when a pixel has more partners than variant 0 holds; variants 0
   and 2 forced on a larger grid, and variant 0 forced on a pixel with more
   than 2048 partners, return LYA_E_UNSUPPORTED.  Returns LYA_E_UNSUPPORTED
   if a pixel has more partner pixels with a side in the r grid than the
   kernel that runs holds (the outputs are then incomplete). */
lya_status lya_xi3(lya_context *ctx, const lya_forests *forests, const lya_grid3 *grid,
                   const lya_options *opts, void *stream,
                   double *num, double *wsum, int64_t *ntrip, double *xi);

/* lya_xi3's sums split by subsample, for the dispersion of the 3PCF (the
   paper's 3PCF figure takes it from subsamples of the forests in sky
   pixels).  subsample[f] in [0, n_sub) (device, [n_forests]); every entry is
   credited to the subsample of its main vertex's forest (the vertex the
   triangle is binned from).  Outputs as lya_xi3, each
   [n_realisations * n_sub * n_bins] row-major (realisation, subsample, bin);
   summing over subsamples gives lya_xi3's sums.  An id outside [0, n_sub)
   returns LYA_E_INVALID before anything is written beyond the zeroed
   outputs. */
lya_status lya_xi3_subsamples(lya_context *ctx, const lya_forests *forests, const lya_grid3 *grid,
                              const lya_options *opts, void *stream,
                              const int32_t *subsample, int32_t n_sub,
                              double *num, double *wsum, int64_t *ntrip, double *xi);

/* Distortion matrix (Sec. 2.2, eq. distortion) over the forest pairs kept by
   options.dmat_keep_fraction / seed, with eta of options.eta.  Outputs,
   device:
     dmat[r][A][B] = D_AB of realisation r, [n_realisations * n_bins * n_bins]
     wsum_d[r][A]  = w_A over the kept pairs, [n_realisations * n_bins]
   Rows with wsum_d == 0 are zero.  delta is not read.  Besides the work
   lists, the context's workspace holds the pair histograms that the
   large-tile kernels keep between passes: ~0.7 GB (FP32 form) or ~0.5 GB
   (FP64 form) on a 256-CU device, whatever the input size. */
lya_status lya_dmat(lya_context *ctx, const lya_forests *forests, const lya_grid *grid,
                    const lya_options *opts, void *stream,
                    double *dmat, double *wsum_d);

/* Gradient of a scalar L(xi) with respect to delta and w: the derivative of
   the estimator of Sec. 2.1 (eq. estimator_two), xi_A = N_A / W_A, through
   N_A and W_A for fixed bins (positions get no gradient: the binning is
   piecewise constant).  Inputs
   grad_xi = dL/dxi, xi and wsum as produced by lya_xi with the same options,
   each [n_realisations * n_bins], device.  Outputs [n_pix], device.
   Without project_deltas:
     grad_delta[i]  = w_i sum_j gamma_{A(i,j)} w_j delta_j
     grad_weight[i] = sum_j gamma_{A(i,j)} w_j (delta_i delta_j - xi_{A(i,j)})
   with gamma_A = grad_xi[A] / wsum[A] (0 where wsum[A] == 0) and j over every
   pixel of every other forest of the same realisation.
   With project_deltas (xi built from delta' = eta delta, eta of options.eta,
   Sec. 2.2): the same sums with delta' give g' = dL/d delta' and h' = dL/dw
   at fixed delta'; eta depends on w through W, the weighted mean of Lambda
   and S, and the chain rule through it gives, per forest,
     grad_delta[k]  = g'_k - w_k c_k,   grad_weight[k] = h'_k - delta'_k c_k,
     c_k = sum_i g'_i / W + (L_k - Lbar) sum_i (L_i - Lbar) g'_i / S
   (the slope part only where the slope term is in use; c = 0 where eta = I).
   These are gradients with respect to the raw delta and w. */
lya_status lya_xi_backward(lya_context *ctx, const lya_forests *forests, const lya_grid *grid,
                           const lya_options *opts, void *stream,
                           const double *grad_xi, const double *xi, const double *wsum,
                           double *grad_delta, double *grad_weight);

/* Short name of a main-kernel variant (the index lya_stats.variant reports):
   kernel 0 = the xi pair kernel, 1 = the distortion-matrix kernel.  Returns a
   static string, or NULL for an index out of range. */
const char *lya_variant_name(int32_t kernel, int32_t variant);

/* Measured peak rates of the context's GPU, the denominators of the pair
   kernels' roofline fractions: out[LYA_N_PEAKS] (HOST) gets lane-operations per second
   over the whole chip from microbenchmark kernels (many waves per SIMD, long
   runs of independent operations, timed with events on `stream`):
     out[0] FP32 VALU fused multiply-add (non-packed)
     out[1] FP64 VALU fused multiply-add
     out[2] LDS atomic add, FP32 (64 lanes on 64 consecutive words)
     out[3] LDS atomic add, FP64 (64 consecutive doubles)
     out[4] LDS atomic add, u32 (64 consecutive words)
     out[5] LDS atomic add, FP32, four lanes on each address
     out[6] LDS store, 32 bits (64 consecutive words)
     out[7] FP32 VALU add
     out[8] u32 VALU add
   Takes a few hundred milliseconds and synchronises the stream. */
#define LYA_N_PEAKS 9
lya_status lya_measure_peaks(lya_context *ctx, void *stream, double *out);

#ifdef __cplusplus
}
#endif

#endif /* LYA_H */
