// Internal definitions shared by the HIP kernels and the host runtime of the
// MI355X Lyman-alpha pair library.  Not part of the public ABI (see lya.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lya.h"

namespace lya {

constexpr int kMaxBins = 4096;     // n_par * n_perp limit (LDS histograms)
constexpr int kMaxStrips = 4096;   // declination strips of the sky index
constexpr int kMaxRealisations = 1 << 20;
constexpr int kChunkMax = 64;      // neighbour forests per xi / backward work item

// Per-forest geometry and layout, FP64 (64 bytes).
struct ForestInfo {
  double nx, ny, nz;   // unit vector (cos dec cos ra, cos dec sin ra, sin dec)
  double dmin, dmax;   // extent along the line of sight (+inf/-inf when empty)
  int64_t pix0;        // first pixel
  int32_t npix;
  int32_t real;        // realisation id
};

// Per-forest eta sums (Sec. 2.2), FP64.
struct EtaInfo {
  double W;      // sum w
  double lbar;   // sum w L / W
  double S;      // sum w (L - lbar)^2
  int32_t slope;   // slope term kept
  int32_t active;  // W > 0 and the projection applies (eta mode not identity)
};

// Device-side scalars produced by the precompute stage.
struct Globals {
  unsigned long long dmin_bits;  // atomics on the bit patterns of positive doubles
  unsigned long long dmax_bits;
  double dc;        // re-centring distance (exactly representable in FP32)
  double m;         // max |D - dc|
  float tau_par;    // FP32 edge-guard half width, in bins
  float tau_perp;
  int32_t flag;     // validation error bits
  int32_t pad;
};

// Pixel records for the xi and backward kernels.
struct __align__(16) Rec32 { float d, wd, w, del; };   // d = D - dc
struct __align__(32) Rec64 { double d, wd, w, del; };  // d = D

// Pixel records for the distortion kernel: D, w and the eta factors
// p = (1, a), q = (u, b) with a = L - lbar, u = w / W, b = w a / S.
// DRec32 also keeps the FP64 distance D for the FP32 edge guard.
struct __align__(16) DRec32 { float d, w, a, u; float b, pad; double D; };
struct __align__(16) DRec64 { double d, w, a, u, b, pad; };

// One persistent-kernel work item: forest at sorted position p against the
// neighbour list entries [nb_begin, nb_begin + nb_count).
struct Item {
  int64_t nb_begin;
  int32_t p;
  int32_t nb_count;
};

// Uniform grid description passed by value to the pair kernels.
struct GridDev {
  int32_t n_par, n_perp;
  double e0_par, e0_perp;       // first edges
  double inv_par, inv_perp;     // 1 / bin width
  double emax_par, emax_perp;   // last edges
  int32_t zero_lo_par, zero_lo_perp;  // first edge is exactly 0
  // 0: uniformly spaced edges on both axes (bin = floor of the coordinate,
  // edge guard only near integers); 1: other edges -- the coordinates use the
  // mean bin width and every pair is binned by searching the FP64 edge arrays
  int32_t exact_all;
};

// Validation error bits (Globals::flag).
enum : int32_t {
  kBadOffsets = 1, kBadFinite = 2, kBadWeight = 4, kBadDist = 8, kBadReal = 16, kBadNpix = 32,
  kBadSub = 64, kBadCap3 = 128, kBadCapC = 256, kBadDet = 512, kBadCapW = 1024
};

// ---------------------------------------------------------------- geometry
// s = |n_f - n_g| / 2 and c = sqrt(1 - s^2) (chord form of the half angle).
// Written with explicit operation order and no contraction so that every
// kernel gets bit-identical values.
__device__ __forceinline__ void pair_sc(const ForestInfo& a, const ForestInfo& b, double& s,
                                        double& c) {
  const double dx = a.nx - b.nx, dy = a.ny - b.ny, dz = a.nz - b.nz;
  const double q = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  s = __dmul_rn(0.5, __dsqrt_rn(q));
  c = __dsqrt_rn(__dsub_rn(1.0, __dmul_rn(s, s)));
}

// Conservative forest-pair cut: false only if no pixel pair can be in the
// grid.  r_perp >= (Dmin_f + Dmin_g) s and r_par >= gap c, with the same
// rounded operations as the separations, so monotone rounding keeps it exact.
__device__ __forceinline__ bool pair_may_bin(const ForestInfo& a, const ForestInfo& b,
                                             double eperp_max, double epar_max) {
  double s, c;
  pair_sc(a, b, s, c);
  const double rperp_min = __dmul_rn(__dadd_rn(a.dmin, b.dmin), s);
  const double gap = fmax(0.0, fmax(__dsub_rn(b.dmin, a.dmax), __dsub_rn(a.dmin, b.dmax)));
  const double rpar_min = __dmul_rn(gap, c);
  return rperp_min < eperp_max && rpar_min < epar_max;
}

// Exact bin of r against FP64 edges[0..n]: the k with edges[k] <= r <
// edges[k + 1], or -1 outside [edges[0], edges[n]).  k0 is a guess: on a
// uniform grid it is right or one bin off; otherwise the remaining range is
// bisected.
__device__ __forceinline__ int bin_exact(double r, const double* __restrict__ edges, int n, int k0) {
  if (!(r >= edges[0]) || !(r < edges[n])) return -1;
  const int k = k0 < 0 ? 0 : (k0 > n - 1 ? n - 1 : k0);
  int lo, hi;  // invariant: edges[lo] <= r < edges[hi]
  if (r < edges[k]) {  // k >= 1 here, since r >= edges[0]
    if (r >= edges[k - 1]) return k - 1;
    lo = 0;
    hi = k - 1;
  } else if (r >= edges[k + 1]) {  // k + 1 < n here, since r < edges[n]
    if (r < edges[k + 2]) return k + 1;
    lo = k + 2;
    hi = n;
  } else {
    return k;
  }
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (r < edges[m]) hi = m;
    else lo = m;
  }
  return lo;
}

// SplitMix64 output function (Steele, Lea & Flood 2014): mix(x + golden gamma).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------- host launchers
// All launchers enqueue on `stream` and return hipSuccess or the launch error.

struct PrecomputeArgs {
  const lya_forests* F;
  int eta_mode;
  int project;
  int want_xi32, want_xi64, want_d32, want_d64;
  int pack_z;           // xi records carry the pixel redshift in their fourth slot
  ForestInfo* finfo;
  EtaInfo* einfo;
  double* delta_proj;   // [n_pix] when project
  Rec32* rec32;
  Rec64* rec64;
  DRec32* drec32;
  DRec64* drec64;
  Globals* glob;
  double eperp_max, epar_max, e0_par, e0_perp, inv_par, inv_perp;
};
hipError_t launch_validate(const lya_forests* F, Globals* glob, hipStream_t st);
// flag bit kBadSub when a subsample id lies outside [0, n_sub)
hipError_t launch_validate_sub(const int32_t* sub, int64_t n_forests, int32_t n_sub, Globals* glob,
                               hipStream_t st);
// subsample covariance: totals N_A, W_A, xi_A and cov_AB from [n_sub][nb] sums
hipError_t launch_covariance(const double* num, const double* wsum, int64_t n_sub, int64_t nb, double* x,
                             double* tot_w, double* xi, double* cov, hipStream_t st);
hipError_t launch_forest_stats(const PrecomputeArgs& a, hipStream_t st);
hipError_t launch_globals(const PrecomputeArgs& a, hipStream_t st);
hipError_t launch_pack(const PrecomputeArgs& a, hipStream_t st);

struct WorklistArgs {
  int64_t n_forests;
  int32_t n_real;
  const ForestInfo* finfo;
  const double* ra;
  const double* dec;
  int n_strips;
  double strip_h;
  double theta;           // largest angle at which a pixel pair can be in the grid (<= strip_h)
  double eperp_max, epar_max;
  int symmetric;          // neighbours on both sides (backward)
  int own_by_index;       // each unordered pair listed under the forest with the smaller input index
  int use_keep;           // distortion subset
  uint64_t keep_thr, seed;
  // outputs / scratch
  uint64_t* keys;
  uint64_t* keys_sorted;
  int32_t* ids;
  int32_t* sorted;        // sorted position -> forest
  int32_t* cell_begin;    // [n_real * n_strips]
  int32_t* cell_end;
  int64_t* cnt;           // [n_forests]
  int64_t* nb_off;        // [n_forests]
  int32_t* nbr;           // neighbour sorted positions
  int32_t* pair_p;        // optional: sorted position of the first forest per entry
  unsigned long long* cand;  // total candidate pixel pairs (sum n_f n_g), accumulated by the count pass
  int64_t* item_cnt;      // [n_forests]
  int64_t* item_off;
  Item* items;
  int chunk;
  void* cub_tmp;
  size_t cub_bytes;
};
size_t worklist_cub_bytes(int64_t n);
hipError_t launch_sort_forests(WorklistArgs& a, hipStream_t st);
hipError_t launch_count_neighbours(const WorklistArgs& a, hipStream_t st);
hipError_t launch_scan(const int64_t* in, int64_t* out, int64_t n, void* tmp, size_t bytes,
                       hipStream_t st);
hipError_t launch_fill_neighbours(const WorklistArgs& a, hipStream_t st);
hipError_t launch_count_items(const WorklistArgs& a, hipStream_t st);
hipError_t launch_fill_items(const WorklistArgs& a, hipStream_t st);

struct XiArgs {
  const ForestInfo* finfo;
  const int32_t* sorted;
  const int32_t* nbr;
  const Item* items;
  int64_t n_items;
  unsigned int* counter;
  const Rec32* rec32;
  const Rec64* rec64;
  const double* dist;
  const double* edges_par;
  const double* edges_perp;
  const Globals* glob;
  GridDev g;
  double* num;
  double* wsum;
  unsigned long long* npairs;
  // optional subsample of each forest (input index): a pair is added to the
  // output slab realisation * n_sub + sub[f] of its owning forest f
  const int32_t* sub;
  int32_t n_sub;
  // bin means (MEANS form): msum[c * n_out + A], c = sum w w x_par,
  // sum w w x_perp (bin units), sum w w (z_i + z_j)
  double* msum;
  int64_t n_out;
  // deterministic form: det_max[2 r], det_max[2 r + 1] = bit patterns of the
  // largest |w d| and w of realisation r; det_acc[4 A + c] = exact integer sums
  // (N low, N high, W low, W high words)
  const unsigned long long* det_max;
  unsigned long long* det_acc;
  // a workgroup flushes its LDS histograms before the candidate pairs added
  // since its last flush could exceed this (u32 counts hold < 2^32)
  double flush_pairs;
};
// default of XiArgs::flush_pairs
constexpr double kXiFlushPairs = 4.0e9;
int xi_num_variants();
const char* xi_variant_name(int v);
hipError_t launch_xi(int variant, int precision, const XiArgs& a, int blocks, hipStream_t st);
// deterministic form (fixed-point integer sums, one variant)
hipError_t launch_xi_det(int precision, const XiArgs& a, int blocks, hipStream_t st);
int xi_det_blocks_per_cu(int precision, int n_bins);
// det_max[2 r], [2 r + 1] = largest |w delta| and w of realisation r (as bits)
hipError_t launch_det_max(const lya_forests* F, const ForestInfo* finfo, const double* delta,
                          unsigned long long* det_max, hipStream_t st);
// num, wsum from the integer sums; flags kBadDet where a bin has 2^36 pairs or more
hipError_t launch_finalize_det(const unsigned long long* det_acc, const unsigned long long* det_max,
                               const unsigned long long* npairs, int64_t n_out, int n_bins, double* num,
                               double* wsum, Globals* glob, hipStream_t st);
int xi_blocks_per_cu(int variant, int precision, int n_bins);

struct DmatArgs {
  const ForestInfo* finfo;
  const EtaInfo* einfo;    // per-forest eta sums (scales of the q vectors)
  const int32_t* sorted;
  const int32_t* nbr;      // second forest (sorted position) of each kept pair
  const int32_t* pair_p;   // first forest (sorted position) of each kept pair
  int64_t n_pairs;
  // pairs ordered by their r_perp window (realisation, first k_perp, span)
  const uint64_t* wkeys;   // sorted window keys
  const int32_t* worder;   // pair index of each sorted key
  int64_t n_items;         // chunks of `chunk` consecutive sorted pairs
  int32_t chunk;
  int32_t item_stride;     // item i is chunk i * item_stride (1; more for the autotuner's sample)
  unsigned int* counter;
  const DRec32* drec32;
  const DRec64* drec64;
  const double* edges_par;
  const double* edges_perp;
  const Globals* glob;
  GridDev g;
  double* dnum;    // [R][nb][nb] numerator of D
  double* wd;      // [R][nb] sum w_i w_j over the kept pairs
  unsigned long long* counters;  // optional [3]: in-grid pixel pairs, outer-product FMAs, out-of-window pairs
  // optional (nullptr: off): the pair histograms of windows of two segments,
  // kept between passes, hsave_run pairs per wave (dmat_hsave_bytes_per_block)
  void* hsave;
  int32_t hsave_run;
};
constexpr int kDmatHsaveRun = 64;
// window key of every kept pair (dmat_window_key below); pairs with no
// possible in-grid pixel pair get ~0
hipError_t launch_dmat_keys(const DmatArgs& a, uint64_t* keys, int32_t* idx, hipStream_t st);
// Window key of a kept forest pair: (span of k_perp rows, descending;
// realisation; first k_perp row), so that the sorted list groups pairs by
// window width, widest (costliest) first, which keeps the end of a launch
// short; ~0 (last) for a pair with no r_perp inside the grid.
__host__ __device__ constexpr uint64_t dmat_window_key(int span, int real, int kt0) {
  return ((uint64_t)(0xFFFF - span) << 48) | ((uint64_t)real << 24) | (uint64_t)kt0;
}
__device__ __forceinline__ int dmat_key_span(uint64_t k) { return 0xFFFF - (int)(k >> 48); }
__device__ __forceinline__ int dmat_key_real(uint64_t k) { return (int)((k >> 24) & 0xFFFFFF); }
__device__ __forceinline__ int dmat_key_kt0(uint64_t k) { return (int)(k & 0xFFFFFF); }
// first position of the sorted keys whose window span is at most max_span
// (one thread; writes the count of wider pairs to *out)
hipError_t launch_dmat_span_split(const uint64_t* keys, int64_t n, int max_span, int64_t* out, hipStream_t st);
hipError_t launch_sort_keys(uint64_t* keys_in, uint64_t* keys_out, int32_t* v_in, int32_t* v_out,
                            int64_t n, void* tmp, size_t bytes, hipStream_t st);
size_t sort_keys_bytes(int64_t n);
// microbenchmarks of the LDS atomic / store and VALU FMA rates (k_peaks.hip)
hipError_t launch_lds_rate(int kind, int blocks, int iters, unsigned long long* sink, hipStream_t st);
hipError_t launch_valu_rate(int kind, int blocks, int iters, void* out, hipStream_t st);  // 0 FP32 FMA, 1 FP64 FMA, 2 FP32 add, 3 u32 add
int peak_block();
int peak_unroll_lds();
int peak_unroll_valu();

// the symmetric-tile D kernels of one or two waves (two tile shapes per form)
int dmat_wave_num_variants();
int dmat_wave_tile_blocks(int v, int precision);  // tile blocks per side of a symmetric-tile variant
// bytes of the kept pair histograms per workgroup of a variant (0: it keeps none)
size_t dmat_wave_hsave_bytes_per_block(int v, int precision, int run);
size_t dmat_hsave_bytes_per_block(int variant, int precision, int run);
const char* dmat_wave_variant_name(int v);
hipError_t launch_dmat_wave(int variant, int precision, const DmatArgs& a, int blocks, hipStream_t st);
int dmat_wave_blocks_per_cu(int variant, int precision);
int dmat_num_variants();
const char* dmat_variant_name(int v);
hipError_t launch_dmat(int variant, int precision, const DmatArgs& a, int blocks, hipStream_t st);
int dmat_blocks_per_cu(int variant, int precision);
hipError_t launch_finalize_dmat(double* d, const double* wd, int64_t n_rows, int nb, hipStream_t st);

struct BwdArgs {
  const ForestInfo* finfo;
  const int32_t* sorted;
  const int32_t* nbr;
  const Item* items;       // one item per forest, all its neighbours (symmetric list)
  int64_t n_items;
  unsigned int* counter;
  const Rec32* rec32;
  const Rec64* rec64;
  const double* dist;
  const double* weight;
  const double* delta;
  const double* edges_par;
  const double* edges_perp;
  const Globals* glob;
  GridDev g;
  const double2* gtab;     // [R][nb] (gamma, gamma * xi) in local bin order
  double* grad_delta;
  double* grad_weight;
};
hipError_t launch_gamma(const double* grad_xi, const double* xi, const double* wsum, double2* out,
                        int64_t n, int NP, int NT, hipStream_t st);
hipError_t launch_xi_bwd(int precision, const BwdArgs& a, int blocks, hipStream_t st);
hipError_t launch_xi_means(int precision, const XiArgs& a, int blocks, hipStream_t st);

// Three-point function (FP64): pixel positions and products, and the kernel.
struct Point3 { double x, y, z, wd, w, pad; };
struct Xi3Args {
  const ForestInfo* finfo;
  const int32_t* sorted;
  const int32_t* nbr;
  const Item* items;
  int64_t n_items;
  unsigned int* counter;
  const Point3* pts;
  Globals* glob;
  int32_t n_r, n_t, n_c;
  int64_t n_bins;
  const double* r_edges;          // [n_r + 1]
  const double* cos_theta_edges;  // [n_t + 1] cosines of the theta edges (decreasing)
  const double* cos_edges;        // [n_c + 1]
  double r_e0, r_inv, c_e0, c_inv;
  double* num;            // n_copies copies of [R][n_bins], copy c at c * copy_stride
  double* wsum;
  unsigned long long* ntrip;
  int32_t n_copies;
  int64_t copy_stride;
  // optional subsample of each forest (input index): entries go to slab
  // realisation * n_sub + sub[f] of their main vertex's forest f
  const int32_t* sub;
  int32_t n_sub;
  // wide kernel: per workgroup two partner lists of w_cap entries (5 doubles,
  // 2 ints each) at blockIdx.x * 10 w_cap in w_dbl, blockIdx.x * 4 w_cap in w_int
  double* w_dbl;
  int32_t* w_int;
  int32_t w_cap;
};
hipError_t launch_xi3_reduce(const double* num_c, const double* wsum_c, const unsigned long long* cnt_c,
                             int n_copies, int64_t stride, int64_t n, double* num, double* wsum, int64_t* ntrip,
                             hipStream_t st);
hipError_t launch_xi3_points(const lya_forests* F, const ForestInfo* finfo, const double* delta, Point3* pts,
                             hipStream_t st);
// kernel 0: sums each vertex's entries in LDS before the global atomics (grids
// with xi3_can_combine; flags kBadCapC when a vertex has more partners than it
// holds); 1: global atomics per entry; 2: as 0 with the partner list in global
// scratch (flags kBadCapW beyond w_cap)
hipError_t launch_xi3(const Xi3Args& a, int kernel, int blocks, hipStream_t st);
int xi3_blocks_per_cu(int kernel);
bool xi3_can_combine(int n_r, int n_t, int n_c);
int xi3_combine_capacity();
int xi3_max_cos_bins();
int xi3_partner_capacity();
int xi_means_blocks_per_cu(int precision, int n_bins);
hipError_t launch_finalize_means(const double* wsum, const double* msum, int64_t n, const GridDev& g,
                                 double* rpar, double* rperp, double* z, hipStream_t st);
hipError_t launch_project_adjoint(const lya_forests* F, const EtaInfo* einfo, const double* delta_proj,
                                  double* grad_delta, double* grad_weight, hipStream_t st);
int xi_bwd_blocks_per_cu(int precision, int n_bins);

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_finalize_xi(const double* num, const double* wsum, double* xi, int64_t n,
                              hipStream_t st);

}  // namespace lya
