// Host runtime of the C ABI declared in lya.h: argument checks, the
// grow-only device workspace, stage orchestration on the caller's stream,
// and the autotuner that picks kernel variants by timing them on the input.
#include <math.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lya_common.h"

using namespace lya;

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct lya_context {
  int device = 0;
  int n_cu = 1;
  std::string err;
  lya_stats stats{};
  std::map<std::string, Buf> bufs;
  std::map<std::string, int> tuned;
  hipEvent_t ev[8]{};
  void* pinned = nullptr;  // small pinned host staging area
  // candidate pairs after which an xi workgroup flushes its LDS histograms;
  // the environment variable LYA_XI_FLUSH_PAIRS lowers it (a test hook that
  // exercises the flush on small inputs)
  double xi_flush_pairs = kXiFlushPairs;
  // the no-allocation entry point carves its workspace from `scratch_base`
  // (this device's copy of the library's fixed scratch array) while `noalloc`
  // is set, bumping `scratch_off`
  unsigned char* scratch_base = nullptr;
  hipError_t scratch_status = hipSuccess;
  bool noalloc = false;
  size_t scratch_off = 0;
};

// Fixed device scratch of lya_xi_noalloc.  Every GPU the library runs on holds
// its own copy until the process ends.  In host code this name is only a
// stand-in for the symbol: the device address of a GPU's copy comes from
// hipGetSymbolAddress, taken once per device (scratch_of) and kept.
static __device__ __align__(256) unsigned char scratch[LYA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr double kPi = 3.141592653589793;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_addr[kMaxDevices] = {};

// Device address of the scratch array on `device`, which must be current;
// looked up once per device.
hipError_t scratch_of(int device, unsigned char** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = (unsigned char*)p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

constexpr int kDmatChunk = 1024;  // kept forest pairs per distortion work item

lya_status fail(lya_context* ctx, lya_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
lya_status fail(lya_context* ctx, lya_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return s;
}

// Message of the last lya_create that failed on this thread (no context to
// hold it); lya_last_error(NULL) returns it.
thread_local char g_create_err[256] = "";

lya_status create_failed(lya_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
lya_status create_failed(lya_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_create_err, sizeof g_create_err, fmt, ap);
  va_end(ap);
  return s;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, LYA_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

#define LYA_TRY(expr)               \
  do {                              \
    lya_status s_ = (expr);         \
    if (s_ != LYA_OK) return s_;    \
  } while (0)

// Grow-only named workspace buffer (256-byte aligned by hipMalloc); in the
// no-allocation mode a 256-byte aligned slice of the device scratch array.
lya_status ws(lya_context* ctx, const char* name, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  if (ctx->noalloc) {
    const size_t at = (ctx->scratch_off + 255) & ~(size_t)255;
    if (at > LYA_NOALLOC_SCRATCH_BYTES || bytes > LYA_NOALLOC_SCRATCH_BYTES - at)
      return fail(ctx, LYA_E_UNSUPPORTED,
                  "input too large for the no-allocation scratch: %s needs %zu bytes at offset %zu of %llu",
                  name, bytes, at, (unsigned long long)LYA_NOALLOC_SCRATCH_BYTES);
    *out = ctx->scratch_base + at;
    ctx->scratch_off = at + bytes;
    return LYA_OK;
  }
  Buf& b = ctx->bufs[name];
  if (b.bytes < bytes) {
    if (b.p) {
      hipDeviceSynchronize();
      hipFree(b.p);
      b.p = nullptr;
      b.bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&b.p, want) != hipSuccess) {
      hipGetLastError();
      b.p = nullptr;
      return fail(ctx, LYA_E_NOMEM, "device allocation of %zu bytes for %s failed", want, name);
    }
    b.bytes = want;
  }
  *out = b.p;
  return LYA_OK;
}

template <typename T>
lya_status wst(lya_context* ctx, const char* name, size_t count, T** out) {
  void* p = nullptr;
  lya_status s = ws(ctx, name, count * sizeof(T), &p);
  *out = (T*)p;
  return s;
}

lya_status check_axis(lya_context* ctx, const double* e, int n, const char* axis, double& e0,
                      double& inv, double& emax, bool& uniform) {
  if (!e) return fail(ctx, LYA_E_INVALID, "edges_%s is NULL", axis);
  if (n < 1) return fail(ctx, LYA_E_INVALID, "n_%s = %d must be >= 1", axis, n);
  for (int k = 0; k <= n; ++k)
    if (!isfinite(e[k])) return fail(ctx, LYA_E_INVALID, "edges_%s[%d] is not finite", axis, k);
  if (e[0] < 0.0) return fail(ctx, LYA_E_INVALID, "edges_%s[0] = %g is negative", axis, e[0]);
  for (int k = 0; k < n; ++k)
    if (!(e[k + 1] > e[k]))
      return fail(ctx, LYA_E_INVALID, "edges_%s not strictly increasing at %d", axis, k);
  // uniform to 1e-9 of a bin: binned from floor(x) with the edge guard;
  // otherwise every pair searches the edge array (GridDev::exact_all)
  const double d = (e[n] - e[0]) / n;
  uniform = true;
  for (int k = 0; k <= n; ++k)
    if (fabs(e[k] - (e[0] + k * d)) > 1e-9 * d) uniform = false;
  e0 = e[0];
  inv = 1.0 / d;
  emax = e[n];
  return LYA_OK;
}

lya_status check_common(lya_context* ctx, const lya_forests* F, const lya_grid* G,
                        const lya_options* o, GridDev& gd) {
  if (!ctx) return LYA_E_INVALID;
  if (!F || !G || !o) return fail(ctx, LYA_E_INVALID, "NULL forests, grid or options");
  if (F->n_forests < 0 || F->n_pix < 0) return fail(ctx, LYA_E_INVALID, "negative n_forests or n_pix");
  if (F->n_forests > INT32_MAX - 1 || F->n_pix > ((int64_t)1 << 40))
    return fail(ctx, LYA_E_UNSUPPORTED, "too many forests or pixels");
  if (F->n_realisations < 1 || F->n_realisations > kMaxRealisations)
    return fail(ctx, LYA_E_INVALID, "n_realisations = %d out of range", F->n_realisations);
  if (F->n_forests > 0 && (!F->offsets || !F->ra || !F->dec))
    return fail(ctx, LYA_E_INVALID, "NULL offsets, ra or dec");
  if (F->n_pix > 0 && (!F->dist || !F->delta || !F->weight || !F->loglam))
    return fail(ctx, LYA_E_INVALID, "NULL dist, delta, weight or loglam");
  if (o->precision != LYA_FP32_COMP && o->precision != LYA_FP64)
    return fail(ctx, LYA_E_INVALID, "unknown precision %d", o->precision);
  if (o->eta < LYA_ETA_IDENTITY || o->eta > LYA_ETA_MEAN_SLOPE)
    return fail(ctx, LYA_E_INVALID, "unknown eta mode %d", o->eta);
  if (!(o->dmat_keep_fraction > 0.0 && o->dmat_keep_fraction <= 1.0))
    return fail(ctx, LYA_E_INVALID, "dmat_keep_fraction = %g outside (0, 1]", o->dmat_keep_fraction);
  if ((int64_t)G->n_par * G->n_perp > kMaxBins)
    return fail(ctx, LYA_E_UNSUPPORTED, "n_par * n_perp = %lld exceeds %d bins",
                (long long)G->n_par * G->n_perp, kMaxBins);
  double e0p, ip, ep, e0t, it, et;
  bool up, ut;
  LYA_TRY(check_axis(ctx, G->edges_par, G->n_par, "par", e0p, ip, ep, up));
  LYA_TRY(check_axis(ctx, G->edges_perp, G->n_perp, "perp", e0t, it, et, ut));
  gd.n_par = G->n_par;
  gd.n_perp = G->n_perp;
  gd.e0_par = e0p;
  gd.e0_perp = e0t;
  gd.inv_par = ip;
  gd.inv_perp = it;
  gd.emax_par = ep;
  gd.emax_perp = et;
  gd.zero_lo_par = e0p == 0.0;
  gd.zero_lo_perp = e0t == 0.0;
  gd.exact_all = (up && ut) ? 0 : 1;
  return LYA_OK;
}

__global__ void init_globals_kernel(Globals* g) {
  g->dmin_bits = 0x7FF0000000000000ull;  // +inf
  g->dmax_bits = 0ull;
  g->dc = 0.0;
  g->m = 0.0;
  g->tau_par = 0.f;
  g->tau_perp = 0.f;
  g->flag = 0;
  g->pad = 0;
}

struct Prepared {
  Globals* glob = nullptr;
  ForestInfo* finfo = nullptr;
  Rec32* rec32 = nullptr;
  Rec64* rec64 = nullptr;
  DRec32* drec32 = nullptr;
  DRec64* drec64 = nullptr;
  double* edges_par = nullptr;
  double* edges_perp = nullptr;
  EtaInfo* einfo = nullptr;
  double* delta_proj = nullptr;  // eta delta per forest (project only), FP64
  Globals host{};
};

// Validation, per-forest sums and record packing.
lya_status prepare(lya_context* ctx, const lya_forests* F, const lya_grid* G, const GridDev& gd,
                   const lya_options* o, hipStream_t st, bool xi_rec, bool d_rec, bool project,
                   Prepared& P, bool pack_z = false) {
  const int64_t N = F->n_forests, npix = F->n_pix;
  LYA_TRY(wst(ctx, "globals", 1, &P.glob));
  LYA_TRY(wst(ctx, "finfo", (size_t)N, &P.finfo));
  EtaInfo* einfo;
  LYA_TRY(wst(ctx, "einfo", (size_t)N, &einfo));
  LYA_TRY(wst(ctx, "edges_par", (size_t)gd.n_par + 1, &P.edges_par));
  LYA_TRY(wst(ctx, "edges_perp", (size_t)gd.n_perp + 1, &P.edges_perp));
  HIP_TRY(hipMemcpyAsync(P.edges_par, G->edges_par, sizeof(double) * (gd.n_par + 1), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P.edges_perp, G->edges_perp, sizeof(double) * (gd.n_perp + 1), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(init_globals_kernel, dim3(1), dim3(1), 0, st, P.glob);
  HIP_TRY(hipGetLastError());
  if (o->validate) {
    HIP_TRY(launch_validate(F, P.glob, st));
    HIP_TRY(hipMemcpyAsync(ctx->pinned, &P.glob->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int32_t flag = *(int32_t*)ctx->pinned;
    if (flag) {
      return fail(ctx, LYA_E_INVALID, "invalid forest arrays:%s%s%s%s%s%s",
                  flag & kBadOffsets ? " offsets not non-decreasing from 0" : "",
                  flag & kBadNpix ? " offsets[n_forests] != n_pix" : "",
                  flag & kBadFinite ? " non-finite values" : "",
                  flag & kBadWeight ? " negative weights" : "",
                  flag & kBadDist ? " non-positive distances" : "",
                  flag & kBadReal ? " realisation id out of range" : "");
    }
  }
  PrecomputeArgs a{};
  a.F = F;
  a.eta_mode = o->eta;
  a.project = project;
  a.want_xi32 = xi_rec && o->precision == LYA_FP32_COMP;
  a.want_xi64 = xi_rec && o->precision == LYA_FP64;
  a.want_d32 = d_rec && o->precision == LYA_FP32_COMP;
  a.want_d64 = d_rec && o->precision == LYA_FP64;
  a.pack_z = pack_z;
  a.finfo = P.finfo;
  a.einfo = einfo;
  a.glob = P.glob;
  a.eperp_max = gd.emax_perp;
  a.epar_max = gd.emax_par;
  a.e0_par = gd.e0_par;
  a.e0_perp = gd.e0_perp;
  a.inv_par = gd.inv_par;
  a.inv_perp = gd.inv_perp;
  if (project) LYA_TRY(wst(ctx, "delta_proj", (size_t)npix, &a.delta_proj));
  if (a.want_xi32) LYA_TRY(wst(ctx, "rec32", (size_t)npix, &a.rec32));
  if (a.want_xi64) LYA_TRY(wst(ctx, "rec64", (size_t)npix, &a.rec64));
  if (a.want_d32) LYA_TRY(wst(ctx, "drec32", (size_t)npix, &a.drec32));
  if (a.want_d64) LYA_TRY(wst(ctx, "drec64", (size_t)npix, &a.drec64));
  HIP_TRY(launch_forest_stats(a, st));
  HIP_TRY(launch_globals(a, st));
  HIP_TRY(launch_pack(a, st));
  HIP_TRY(hipMemcpyAsync(ctx->pinned, P.glob, sizeof(Globals), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  memcpy(&P.host, ctx->pinned, sizeof(Globals));
  P.einfo = einfo;
  P.delta_proj = a.delta_proj;
  P.rec32 = a.rec32;
  P.rec64 = a.rec64;
  P.drec32 = a.drec32;
  P.drec64 = a.drec64;
  return LYA_OK;
}

struct Worklist {
  int32_t* sorted = nullptr;
  int32_t* nbr = nullptr;
  int32_t* pair_p = nullptr;
  Item* items = nullptr;
  int64_t n_pairs = 0;
  int64_t n_items = 0;
  int64_t candidates = 0;
};

lya_status read_i64(lya_context* ctx, const int64_t* dev, int64_t* host, int count, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(ctx->pinned, dev, sizeof(int64_t) * count, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  memcpy(host, ctx->pinned, sizeof(int64_t) * count);
  return LYA_OK;
}

// Sky index, neighbour lists and work items (Sec. 2.1 pre-ordering).
lya_status build_worklist(lya_context* ctx, const lya_forests* F, const GridDev& gd,
                          const Prepared& P, hipStream_t st, bool symmetric, bool use_keep,
                          uint64_t keep_thr, uint64_t seed, bool want_pairs, int chunk,
                          const char* tag, Worklist& W, bool own_by_index = false) {
  const int64_t N = F->n_forests;
  const int R = F->n_realisations;
  const double dmin = __builtin_bit_cast(double, P.host.dmin_bits);
  double arg = (dmin > 0.0 && isfinite(dmin)) ? gd.emax_perp / (2.0 * dmin) : 2.0;
  double theta = arg >= 1.0 ? kPi : 2.0 * asin(arg);
  theta = theta * (1.0 + 1e-9) + 1e-12;
  int n_strips = (int)floor(kPi / theta);
  if (n_strips < 1) n_strips = 1;
  if (n_strips > kMaxStrips) n_strips = kMaxStrips;
  const int max_by_real = (int)((1u << 12) - 1);
  if (n_strips > max_by_real) n_strips = max_by_real;

  WorklistArgs a{};
  a.n_forests = N;
  a.n_real = R;
  a.finfo = P.finfo;
  a.ra = F->ra;
  a.dec = F->dec;
  a.n_strips = n_strips;
  a.strip_h = kPi / n_strips;
  a.theta = theta;
  a.eperp_max = gd.emax_perp;
  a.epar_max = gd.emax_par;
  a.symmetric = symmetric || own_by_index;
  a.own_by_index = own_by_index;
  a.use_keep = use_keep;
  a.keep_thr = keep_thr;
  a.seed = seed;
  a.chunk = chunk;
  std::string t(tag);
  LYA_TRY(wst(ctx, "wl_keys", (size_t)N, &a.keys));
  LYA_TRY(wst(ctx, "wl_keys_sorted", (size_t)N, &a.keys_sorted));
  LYA_TRY(wst(ctx, "wl_ids", (size_t)N, &a.ids));
  LYA_TRY(wst(ctx, (t + "_sorted").c_str(), (size_t)N, &a.sorted));
  LYA_TRY(wst(ctx, "wl_cell_begin", (size_t)R * n_strips, &a.cell_begin));
  LYA_TRY(wst(ctx, "wl_cell_end", (size_t)R * n_strips, &a.cell_end));
  LYA_TRY(wst(ctx, "wl_cnt", (size_t)N, &a.cnt));
  LYA_TRY(wst(ctx, "wl_nb_off", (size_t)N, &a.nb_off));
  LYA_TRY(wst(ctx, "wl_item_cnt", (size_t)N, &a.item_cnt));
  LYA_TRY(wst(ctx, "wl_item_off", (size_t)N, &a.item_off));
  a.cub_bytes = worklist_cub_bytes(N);
  LYA_TRY(ws(ctx, "wl_cub", a.cub_bytes, &a.cub_tmp));

  LYA_TRY(wst(ctx, "wl_cand", 1, &a.cand));
  HIP_TRY(launch_zero(a.cand, sizeof(unsigned long long), st));
  HIP_TRY(launch_sort_forests(a, st));
  HIP_TRY(launch_count_neighbours(a, st));
  HIP_TRY(launch_scan(a.cnt, a.nb_off, N, a.cub_tmp, a.cub_bytes, st));
  int64_t last[3];
  HIP_TRY(hipMemcpyAsync((char*)ctx->pinned, a.cnt + (N - 1), 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync((char*)ctx->pinned + 8, a.nb_off + (N - 1), 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync((char*)ctx->pinned + 16, a.cand, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  memcpy(last, ctx->pinned, 24);
  const int64_t total = last[0] + last[1];
  W.candidates = last[2];
  LYA_TRY(wst(ctx, (t + "_nbr").c_str(), (size_t)total, &a.nbr));
  if (want_pairs) LYA_TRY(wst(ctx, (t + "_pair_p").c_str(), (size_t)total, &a.pair_p));
  HIP_TRY(launch_fill_neighbours(a, st));
  W.sorted = a.sorted;
  W.nbr = a.nbr;
  W.pair_p = a.pair_p;
  W.n_pairs = total;
  if (chunk > 0) {
    HIP_TRY(launch_count_items(a, st));
    HIP_TRY(launch_scan(a.item_cnt, a.item_off, N, a.cub_tmp, a.cub_bytes, st));
    HIP_TRY(hipMemcpyAsync((char*)ctx->pinned, a.item_cnt + (N - 1), 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync((char*)ctx->pinned + 8, a.item_off + (N - 1), 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    memcpy(last, ctx->pinned, 16);
    W.n_items = last[0] + last[1];
    LYA_TRY(wst(ctx, (t + "_items").c_str(), (size_t)W.n_items, &a.items));
    HIP_TRY(launch_fill_items(a, st));
    W.items = a.items;
  }
  return LYA_OK;
}

int xi_chunk(const lya_forests* F, int target_stream) {
  const double mean = F->n_forests ? (double)F->n_pix / (double)F->n_forests : 1.0;
  int c = (int)llround(target_stream / (mean > 1.0 ? mean : 1.0));
  if (c < 1) c = 1;
  if (c > kChunkMax) c = kChunkMax;
  return c;
}

// Optional per-stage device timing: events 0..5 bracket the stages.
struct Timer {
  lya_context* ctx;
  hipStream_t st;
  bool on;
  void at(int i) {
    if (on) hipEventRecord(ctx->ev[i], st);
  }
  float ms(int a, int b) {
    float t = 0.f;
    if (on) hipEventElapsedTime(&t, ctx->ev[a], ctx->ev[b]);
    return t;
  }
  lya_status finish(lya_context* c) {
    if (!on) return LYA_OK;
    if (hipEventSynchronize(c->ev[5]) != hipSuccess) return fail(c, LYA_E_DEVICE, "event sync failed");
    c->stats.ms_precompute = ms(0, 1);
    c->stats.ms_worklist = ms(1, 2);
    c->stats.ms_main = ms(3, 4);
    c->stats.ms_finalize = ms(4, 5);
    return LYA_OK;
  }
};

}  // namespace

extern "C" {

void lya_options_default(lya_options* o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->precision = LYA_FP32_COMP;
  o->eta = LYA_ETA_MEAN_SLOPE;
  o->project_deltas = 0;
  o->autotune = 1;
  o->validate = 1;
  o->timing = 0;
  o->variant = -1;
  o->counters = 0;
  o->dmat_keep_fraction = 1.0;
  o->seed = 0;
  o->deterministic = 0;
}

lya_status lya_create(lya_context** out, int device) {
  if (!out) return LYA_E_INVALID;
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || device < 0 || device >= n) {
    hipGetLastError();
    return create_failed(LYA_E_DEVICE, "hipGetDeviceCount: %s (%d devices, device %d requested)",
                         hipGetErrorString(e), n, device);
  }
  lya_context* ctx = new lya_context();
  ctx->device = device;
  if ((e = hipSetDevice(device)) != hipSuccess) {
    delete ctx;
    return create_failed(LYA_E_DEVICE, "hipSetDevice(%d): %s", device, hipGetErrorString(e));
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->n_cu = prop.multiProcessorCount;
  for (auto& ev : ctx->ev)
    if ((e = hipEventCreate(&ev)) != hipSuccess) {
      delete ctx;
      return create_failed(LYA_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
  if ((e = hipHostMalloc(&ctx->pinned, 4096)) != hipSuccess) {
    delete ctx;
    return create_failed(LYA_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
  }
  // the no-allocation entry point reports a failed lookup; the others never need it
  ctx->scratch_status = scratch_of(device, &ctx->scratch_base);
  if (ctx->scratch_status != hipSuccess) hipGetLastError();
  ctx->err.reserve(512);  // error messages then need no allocation
  if (const char* fp = getenv("LYA_XI_FLUSH_PAIRS")) {
    const double v = atof(fp);
    if (v >= 1.0 && v < kXiFlushPairs) ctx->xi_flush_pairs = v;
  }
  *out = ctx;
  return LYA_OK;
}

void lya_destroy(lya_context* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto& kv : ctx->bufs)
    if (kv.second.p) hipFree(kv.second.p);
  for (auto& e : ctx->ev)
    if (e) hipEventDestroy(e);
  if (ctx->pinned) hipHostFree(ctx->pinned);
  delete ctx;
}

const char* lya_last_error(const lya_context* ctx) {
  if (ctx) return ctx->err.c_str();
  return g_create_err[0] ? g_create_err : "NULL context";
}

lya_status lya_last_stats(const lya_context* ctx, lya_stats* out) {
  if (!ctx || !out) return LYA_E_INVALID;
  *out = ctx->stats;
  return LYA_OK;
}

namespace {

// xi sums, optionally split by the subsample of each pair's owning forest
// (sub != nullptr: outputs [R][n_sub][n_bins], each unordered pair owned by
// the forest with the smaller input index).
lya_status xi_impl(lya_context* ctx, const lya_forests* F, const lya_grid* G, const lya_options* o,
                   void* stream, const int32_t* sub, int32_t n_sub, double* num, double* wsum,
                   int64_t* npairs, double* xi, double* const* means = nullptr) {
  GridDev gd{};
  LYA_TRY(check_common(ctx, F, G, o, gd));
  if (!num || !wsum || !npairs) return fail(ctx, LYA_E_INVALID, "NULL output num, wsum or npairs");
  if (sub && n_sub < 1) return fail(ctx, LYA_E_INVALID, "n_sub must be >= 1");
  if (o->deterministic && (sub || means))
    return fail(ctx, LYA_E_UNSUPPORTED, "options.deterministic is honoured by lya_xi only");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  ctx->err.clear();
  ctx->stats = lya_stats{};
  const int nb = gd.n_par * gd.n_perp;
  const int64_t nout = (int64_t)F->n_realisations * (sub ? n_sub : 1) * nb;
  Timer tm{ctx, st, o->timing != 0};
  tm.at(0);
  HIP_TRY(launch_zero(num, nout * sizeof(double), st));
  HIP_TRY(launch_zero(wsum, nout * sizeof(double), st));
  HIP_TRY(launch_zero(npairs, nout * sizeof(int64_t), st));
  double* msum = nullptr;
  if (means) {
    LYA_TRY(wst(ctx, "xi_msum", (size_t)(3 * nout), &msum));
    HIP_TRY(launch_zero(msum, 3 * nout * sizeof(double), st));
  }
  if (F->n_forests > 0 && F->n_pix > 0) {
    Prepared P;
    LYA_TRY(prepare(ctx, F, G, gd, o, st, true, false, o->project_deltas != 0, P, means != nullptr));
    if (sub) {
      HIP_TRY(launch_validate_sub(sub, F->n_forests, n_sub, P.glob, st));
      HIP_TRY(hipMemcpyAsync(ctx->pinned, &P.glob->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (*(int32_t*)ctx->pinned & kBadSub) return fail(ctx, LYA_E_INVALID, "subsample id outside [0, n_sub)");
    }
    tm.at(1);
    Worklist W;
    const int chunk = xi_chunk(F, 4096);
    // subsample sums and the deterministic form list each unordered pair under
    // the forest with the smaller input index: the owner (and with it which
    // forest's pixels form the run sums) then does not depend on the sky
    // index, whose strip height follows the smallest distance of the whole
    // batch
    LYA_TRY(build_worklist(ctx, F, gd, P, st, false, false, 0, 0, false, chunk, "xi", W,
                           sub != nullptr || o->deterministic != 0));
    tm.at(2);
    ctx->stats.forest_pairs = W.n_pairs;
    ctx->stats.work_items = W.n_items;
    ctx->stats.candidate_pairs = W.candidates;
    unsigned int* counter;
    LYA_TRY(wst(ctx, "xi_counter", 1, &counter));
    XiArgs a{};
    a.finfo = P.finfo;
    a.sorted = W.sorted;
    a.nbr = W.nbr;
    a.items = W.items;
    a.n_items = W.n_items;
    a.counter = counter;
    a.rec32 = P.rec32;
    a.rec64 = P.rec64;
    a.dist = F->dist;
    a.edges_par = P.edges_par;
    a.edges_perp = P.edges_perp;
    a.glob = P.glob;
    a.g = gd;
    a.num = num;
    a.wsum = wsum;
    a.npairs = (unsigned long long*)npairs;
    a.sub = sub;
    a.n_sub = sub ? n_sub : 1;
    a.msum = msum;
    a.n_out = nout;
    a.flush_pairs = ctx->xi_flush_pairs;

    if (o->deterministic) {
      // fixed-point integer sums with a scale per realisation; one variant
      unsigned long long *det_max, *det_acc;
      LYA_TRY(wst(ctx, "xi_det_max", (size_t)(2 * F->n_realisations), &det_max));
      LYA_TRY(wst(ctx, "xi_det_acc", (size_t)(4 * nout), &det_acc));
      HIP_TRY(launch_zero(det_max, (size_t)(2 * F->n_realisations) * sizeof(unsigned long long), st));
      HIP_TRY(launch_zero(det_acc, (size_t)(4 * nout) * sizeof(unsigned long long), st));
      HIP_TRY(launch_det_max(F, P.finfo, o->project_deltas ? P.delta_proj : F->delta, det_max, st));
      a.det_max = det_max;
      a.det_acc = det_acc;
      const int blocks = xi_det_blocks_per_cu(o->precision, nb) * ctx->n_cu;
      ctx->stats.variant = -1;
      ctx->stats.grid_blocks = blocks;
      HIP_TRY(launch_zero(counter, 4, st));
      tm.at(3);
      HIP_TRY(launch_xi_det(o->precision, a, blocks, st));
      HIP_TRY(launch_finalize_det(det_acc, det_max, a.npairs, nout, nb, num, wsum, P.glob, st));
      tm.at(4);
      HIP_TRY(hipMemcpyAsync(ctx->pinned, &P.glob->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (*(int32_t*)ctx->pinned & kBadDet)
        return fail(ctx, LYA_E_UNSUPPORTED, "a bin holds 2^36 pairs or more (deterministic sums)");
      HIP_TRY(launch_finalize_xi(num, wsum, xi, nout, st));
      tm.at(5);
      return tm.finish(ctx);
    }

    if (means) {
      // one run-length form with the coordinate sums; no variant choice
      const int blocks = xi_means_blocks_per_cu(o->precision, nb) * ctx->n_cu;
      ctx->stats.variant = -1;
      ctx->stats.grid_blocks = blocks;
      HIP_TRY(launch_zero(counter, 4, st));
      tm.at(3);
      HIP_TRY(launch_xi_means(o->precision, a, blocks, st));
      tm.at(4);
      HIP_TRY(launch_finalize_xi(num, wsum, xi, nout, st));
      HIP_TRY(launch_finalize_means(wsum, msum, nout, gd, means[0], means[1], means[2], st));
      tm.at(5);
      return tm.finish(ctx);
    }

    // autotune: time each variant on a prefix of the work list, into scratch outputs
    char key[128];
    snprintf(key, sizeof key, "xi/%d/%d/%d", o->precision, nb,
             (int)(F->n_pix / (F->n_forests ? F->n_forests : 1) / 64));
    int variant = 0;
    auto found = ctx->tuned.find(key);
    if (o->variant >= 0) {
      if (o->variant >= xi_num_variants())
        return fail(ctx, LYA_E_INVALID, "variant %d out of range (xi has %d)", o->variant, xi_num_variants());
      variant = o->variant;
    } else if (found != ctx->tuned.end()) {
      variant = found->second;
    } else if (o->autotune && W.n_items > 0 && !ctx->noalloc) {
      double* sn;
      double* sw;
      unsigned long long* sc;
      LYA_TRY(wst(ctx, "tune_num", (size_t)nout, &sn));
      LYA_TRY(wst(ctx, "tune_wsum", (size_t)nout, &sw));
      LYA_TRY(wst(ctx, "tune_cnt", (size_t)nout, &sc));
      XiArgs t = a;
      t.num = sn;
      t.wsum = sw;
      t.npairs = sc;
      int64_t sample = W.n_items / 8;
      if (sample < 4 * ctx->n_cu) sample = W.n_items < 4 * ctx->n_cu ? W.n_items : 4 * ctx->n_cu;
      t.n_items = sample;
      float best = 1e30f;
      for (int v = 0; v < xi_num_variants(); ++v) {
        const int blocks = xi_blocks_per_cu(v, o->precision, nb) * ctx->n_cu;
        float ms_v = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
          HIP_TRY(launch_zero(counter, 4, st));
          HIP_TRY(hipEventRecord(ctx->ev[6], st));
          HIP_TRY(launch_xi(v, o->precision, t, blocks, st));
          HIP_TRY(hipEventRecord(ctx->ev[7], st));
          HIP_TRY(hipEventSynchronize(ctx->ev[7]));
          HIP_TRY(hipEventElapsedTime(&ms_v, ctx->ev[6], ctx->ev[7]));
        }
        if (ms_v < best) {
          best = ms_v;
          variant = v;
        }
      }
      ctx->tuned[key] = variant;
    }
    const int blocks = xi_blocks_per_cu(variant, o->precision, nb) * ctx->n_cu;
    ctx->stats.variant = variant;
    ctx->stats.grid_blocks = blocks;
    HIP_TRY(launch_zero(counter, 4, st));
    tm.at(3);
    HIP_TRY(launch_xi(variant, o->precision, a, blocks, st));
    tm.at(4);
  } else {
    tm.at(1);
    tm.at(2);
    tm.at(3);
    tm.at(4);
  }
  HIP_TRY(launch_finalize_xi(num, wsum, xi, nout, st));
  if (means) HIP_TRY(launch_finalize_means(wsum, msum, nout, gd, means[0], means[1], means[2], st));
  tm.at(5);
  return tm.finish(ctx);
}

}  // namespace

lya_status lya_xi(lya_context* ctx, const lya_forests* F, const lya_grid* G, const lya_options* o,
                  void* stream, double* num, double* wsum, int64_t* npairs, double* xi) {
  return xi_impl(ctx, F, G, o, stream, nullptr, 1, num, wsum, npairs, xi);
}

lya_status lya_xi_noalloc(lya_context* ctx, const lya_forests* F, const lya_grid* G,
                          const lya_options* o, void* stream, double* num, double* wsum, int64_t* npairs,
                          double* xi) {
  if (!ctx) return LYA_E_INVALID;
  if (!ctx->scratch_base)
    return fail(ctx, LYA_E_DEVICE, "address of the device scratch array unavailable: %s",
                hipGetErrorString(ctx->scratch_status));
  ctx->noalloc = true;
  ctx->scratch_off = 0;
  const lya_status s = xi_impl(ctx, F, G, o, stream, nullptr, 1, num, wsum, npairs, xi);
  ctx->noalloc = false;
  return s;
}

const char* lya_variant_name(int32_t kernel, int32_t variant) {
  if (kernel == 0) return (variant >= 0 && variant < xi_num_variants()) ? xi_variant_name(variant) : nullptr;
  if (kernel == 1) {
    if (variant == dmat_num_variants()) return "hybrid: sym-small for one-tile windows, sym-big for wider ones";
    return (variant >= 0 && variant < dmat_num_variants()) ? dmat_variant_name(variant) : nullptr;
  }
  return nullptr;
}

lya_status lya_measure_peaks(lya_context* ctx, void* stream, double* out) {
  if (!ctx) return LYA_E_INVALID;
  if (!out) return fail(ctx, LYA_E_INVALID, "NULL output");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  ctx->err.clear();
  unsigned long long* sink;
  float* vout;
  LYA_TRY(wst(ctx, "peak_sink", 1, &sink));
  LYA_TRY(wst(ctx, "peak_out", (size_t)2 * peak_block(), &vout));
  const int blocks = 8 * ctx->n_cu;  // 32 waves per CU
  const double lanes = (double)blocks * peak_block();
  // (VALU or LDS, kind, iterations): FP32 FMA, FP64 FMA, the LDS kinds of
  // k_peaks.hip, then FP32 and u32 additions
  struct Run { int valu, kind, iters; };
  const Run runs[LYA_N_PEAKS] = {{1, 0, 40000}, {1, 1, 20000}, {0, 0, 20000}, {0, 1, 20000}, {0, 2, 20000},
                                 {0, 3, 5000},  {0, 4, 20000}, {1, 2, 40000}, {1, 3, 40000}};
  for (int r = 0; r < LYA_N_PEAKS; ++r) {
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up
      HIP_TRY(hipEventRecord(ctx->ev[6], st));
      if (runs[r].valu) HIP_TRY(launch_valu_rate(runs[r].kind, blocks, runs[r].iters, vout, st));
      else HIP_TRY(launch_lds_rate(runs[r].kind, blocks, runs[r].iters, sink, st));
      HIP_TRY(hipEventRecord(ctx->ev[7], st));
      HIP_TRY(hipEventSynchronize(ctx->ev[7]));
      HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[6], ctx->ev[7]));
    }
    const double per_lane = (double)runs[r].iters * (runs[r].valu ? peak_unroll_valu() : peak_unroll_lds());
    out[r] = ms > 0.f ? lanes * per_lane / (ms * 1e-3) : 0.0;
  }
  return LYA_OK;
}

lya_status lya_xi_means(lya_context* ctx, const lya_forests* F, const lya_grid* G, const lya_options* o,
                        void* stream, double* num, double* wsum, int64_t* npairs, double* xi,
                        double* rpar, double* rperp, double* z) {
  if (!ctx) return LYA_E_INVALID;
  if (!rpar || !rperp || !z) return fail(ctx, LYA_E_INVALID, "NULL output rpar, rperp or z");
  double* const means[3] = {rpar, rperp, z};
  return xi_impl(ctx, F, G, o, stream, nullptr, 1, num, wsum, npairs, xi, means);
}

lya_status lya_xi_subsamples(lya_context* ctx, const lya_forests* F, const lya_grid* G,
                             const lya_options* o, void* stream, const int32_t* subsample, int32_t n_sub,
                             double* num, double* wsum, int64_t* npairs, double* xi) {
  if (!ctx) return LYA_E_INVALID;
  if (!subsample) return fail(ctx, LYA_E_INVALID, "NULL subsample");
  return xi_impl(ctx, F, G, o, stream, subsample, n_sub, num, wsum, npairs, xi);
}

lya_status lya_xi_covariance(lya_context* ctx, const double* num, const double* wsum, int64_t n_sub,
                             int64_t n_bins, void* stream, double* xi, double* cov) {
  if (!ctx) return LYA_E_INVALID;
  ctx->err.clear();
  if (!num || !wsum || !xi || !cov) return fail(ctx, LYA_E_INVALID, "NULL num, wsum, xi or cov");
  if (n_sub < 1 || n_bins < 1 || n_bins > kMaxBins)
    return fail(ctx, LYA_E_INVALID, "n_sub must be >= 1 and n_bins in [1, %d]", kMaxBins);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  double* x;
  double* tw;
  LYA_TRY(wst(ctx, "cov_x", (size_t)(n_sub * n_bins), &x));
  LYA_TRY(wst(ctx, "cov_w", (size_t)n_bins, &tw));
  HIP_TRY(launch_covariance(num, wsum, n_sub, n_bins, x, tw, xi, cov, st));
  return LYA_OK;
}

// partner pixels per vertex pixel held by the wide 3PCF kernel's scratch lists
constexpr int kXi3WideCap = 32768;

namespace {

// 3PCF sums, optionally split by the subsample of each entry's main vertex
// forest (sub != nullptr: outputs [R][n_sub][n_bins]).
lya_status xi3_impl(lya_context* ctx, const lya_forests* F, const lya_grid3* G3, const lya_options* o,
                    void* stream, const int32_t* sub, int32_t n_sub, double* num, double* wsum, int64_t* ntrip,
                    double* xi) {
  if (!ctx) return LYA_E_INVALID;
  if (!G3) return fail(ctx, LYA_E_INVALID, "NULL grid");
  double r_e0, r_inv, r_max;
  bool r_uniform;
  LYA_TRY(check_axis(ctx, G3->r_edges, G3->n_r, "r", r_e0, r_inv, r_max, r_uniform));
  if (!r_uniform) return fail(ctx, LYA_E_UNSUPPORTED, "r_edges are not uniformly spaced (the 3PCF bins uniform sides only)");
  const int nt = G3->n_theta, nc = G3->n_cos;
  const double* te = G3->theta_edges;
  const double* ce = G3->cos_edges;
  if (!te || !ce) return fail(ctx, LYA_E_INVALID, "NULL theta_edges or cos_edges");
  if (nt < 1 || nc < 1) return fail(ctx, LYA_E_INVALID, "n_theta and n_cos must be >= 1");
  if (nt > 1024) return fail(ctx, LYA_E_UNSUPPORTED, "n_theta = %d exceeds 1024", nt);
  if (nc > xi3_max_cos_bins())
    return fail(ctx, LYA_E_UNSUPPORTED, "n_cos = %d exceeds %d", nc, xi3_max_cos_bins());
  for (int k = 0; k <= nt; ++k)
    if (!isfinite(te[k]) || te[k] < 0.0 || te[k] > kPi || (k > 0 && !(te[k] > te[k - 1])))
      return fail(ctx, LYA_E_INVALID, "theta_edges must increase strictly within [0, pi] (edge %d)", k);
  for (int k = 0; k <= nc; ++k)
    if (!isfinite(ce[k]) || ce[k] < -1.0 || ce[k] > 1.0 || (k > 0 && !(ce[k] > ce[k - 1])))
      return fail(ctx, LYA_E_INVALID, "cos_edges must increase strictly within [-1, 1] (edge %d)", k);
  const double cd = (ce[nc] - ce[0]) / nc;
  for (int k = 0; k <= nc; ++k)
    if (fabs(ce[k] - (ce[0] + k * cd)) > 1e-9 * cd)
      return fail(ctx, LYA_E_UNSUPPORTED, "cos_edges are not uniformly spaced (edge %d)", k);
  const int nr = G3->n_r;
  const int64_t n_bins = (int64_t)nr * nr * nc * nt * nt;
  if (n_bins > ((int64_t)1 << 30)) return fail(ctx, LYA_E_UNSUPPORTED, "%lld bins exceed 2^30", (long long)n_bins);
  // forests and options are checked as for a pair grid that boxes every side
  double box[2] = {0.0, r_max};
  const lya_grid G{1, 1, box, box};
  GridDev gd{};
  LYA_TRY(check_common(ctx, F, &G, o, gd));
  if (o->deterministic) return fail(ctx, LYA_E_UNSUPPORTED, "options.deterministic is honoured by lya_xi only");
  if (!num || !wsum || !ntrip) return fail(ctx, LYA_E_INVALID, "NULL output num, wsum or ntrip");
  if (sub && n_sub < 1) return fail(ctx, LYA_E_INVALID, "n_sub must be >= 1");
  const int64_t nslab = (int64_t)F->n_realisations * (sub ? n_sub : 1);
  if (nslab * n_bins > ((int64_t)1 << 40)) return fail(ctx, LYA_E_UNSUPPORTED, "outputs too large");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  ctx->err.clear();
  ctx->stats = lya_stats{};
  const int64_t nout = nslab * n_bins;
  Timer tm{ctx, st, o->timing != 0};
  tm.at(0);
  HIP_TRY(launch_zero(num, nout * sizeof(double), st));
  HIP_TRY(launch_zero(wsum, nout * sizeof(double), st));
  HIP_TRY(launch_zero(ntrip, nout * sizeof(int64_t), st));
  if (F->n_forests > 0 && F->n_pix > 0) {
    Prepared P;
    const bool project = o->project_deltas != 0;
    LYA_TRY(prepare(ctx, F, &G, gd, o, st, false, false, project, P));
    if (sub) {
      HIP_TRY(launch_validate_sub(sub, F->n_forests, n_sub, P.glob, st));
      HIP_TRY(hipMemcpyAsync(ctx->pinned, &P.glob->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (*(int32_t*)ctx->pinned & kBadSub) return fail(ctx, LYA_E_INVALID, "subsample id outside [0, n_sub)");
    }
    Point3* pts;
    LYA_TRY(wst(ctx, "xi3_pts", (size_t)F->n_pix, &pts));
    HIP_TRY(launch_xi3_points(F, P.finfo, project ? P.delta_proj : F->delta, pts, st));
    tm.at(1);
    Worklist W;
    LYA_TRY(build_worklist(ctx, F, gd, P, st, true, false, 0, 0, false, INT32_MAX, "x3", W));
    tm.at(2);
    ctx->stats.forest_pairs = W.n_pairs;
    ctx->stats.work_items = W.n_items;
    ctx->stats.candidate_pairs = W.candidates;
    // r edges, cosines of the theta edges, cos alpha edges
    std::vector<double> he;
    he.insert(he.end(), G3->r_edges, G3->r_edges + nr + 1);
    for (int k = 0; k <= nt; ++k) he.push_back(k == 0 && te[0] == 0.0 ? 1.0 : (te[k] == kPi ? -1.0 : cos(te[k])));
    he.insert(he.end(), ce, ce + nc + 1);
    double* de;
    LYA_TRY(wst(ctx, "xi3_edges", he.size(), &de));
    HIP_TRY(hipMemcpyAsync(de, he.data(), he.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    unsigned int* counter;
    LYA_TRY(wst(ctx, "xi3_counter", 1, &counter));
    Xi3Args a{};
    a.finfo = P.finfo;
    a.sorted = W.sorted;
    a.nbr = W.nbr;
    a.items = W.items;
    a.n_items = W.n_items;
    a.counter = counter;
    a.pts = pts;
    a.glob = P.glob;
    a.n_r = nr;
    a.n_t = nt;
    a.n_c = nc;
    a.n_bins = n_bins;
    a.r_edges = de;
    a.cos_theta_edges = de + nr + 1;
    a.cos_edges = de + nr + 1 + nt + 1;
    a.r_e0 = r_e0;
    a.r_inv = r_inv;
    a.c_e0 = ce[0];
    a.c_inv = 1.0 / cd;
    // one copy of the sums per XCD (8 on MI355X) when they fit in 1 GiB of
    // workspace: the triplet atomics spread over 8 times the addresses
    const int n_copies = nout * 24 * 8 <= ((int64_t)1 << 30) ? 8 : 1;
    double* cn = num;
    double* cw = wsum;
    unsigned long long* cc = (unsigned long long*)ntrip;
    if (n_copies > 1) {
      LYA_TRY(wst(ctx, "xi3_num_c", (size_t)(n_copies * nout), &cn));
      LYA_TRY(wst(ctx, "xi3_wsum_c", (size_t)(n_copies * nout), &cw));
      LYA_TRY(wst(ctx, "xi3_cnt_c", (size_t)(n_copies * nout), &cc));
      HIP_TRY(launch_zero(cn, (size_t)(n_copies * nout) * sizeof(double), st));
      HIP_TRY(launch_zero(cw, (size_t)(n_copies * nout) * sizeof(double), st));
      HIP_TRY(launch_zero(cc, (size_t)(n_copies * nout) * sizeof(unsigned long long), st));
    }
    a.num = cn;
    a.wsum = cw;
    a.ntrip = cc;
    a.n_copies = n_copies;
    a.copy_stride = nout;
    a.sub = sub;
    a.n_sub = sub ? n_sub : 1;
    // variant 0: the combining kernel (LDS sums per vertex and side-1 cell),
    // 1: the direct kernel, 2: the wide combining kernel (partner lists in
    // global scratch); by default 0 where the grid fits the LDS slice (else
    // 1), and 2 instead of 0 when a pixel has more partners than 0 holds
    const bool fits = xi3_can_combine(nr, nt, nc);
    if (o->variant > 2) return fail(ctx, LYA_E_INVALID, "variant %d out of range (xi3 has 3)", o->variant);
    if ((o->variant == 0 || o->variant == 2) && !fits)
      return fail(ctx, LYA_E_UNSUPPORTED, "grid too large for the combining kernels (variant %d)", o->variant);
    int kernel = o->variant >= 0 ? o->variant : (fits ? 0 : 1);
    tm.at(3);
    for (;;) {
      const int blocks = xi3_blocks_per_cu(kernel) * ctx->n_cu;
      ctx->stats.grid_blocks = blocks;
      ctx->stats.variant = kernel;
      if (kernel == 2) {
        a.w_cap = kXi3WideCap;
        LYA_TRY(wst(ctx, "xi3_wide_dbl", (size_t)blocks * 10 * kXi3WideCap, &a.w_dbl));
        LYA_TRY(wst(ctx, "xi3_wide_int", (size_t)blocks * 4 * kXi3WideCap, &a.w_int));
      }
      HIP_TRY(launch_zero(counter, 4, st));
      HIP_TRY(launch_xi3(a, kernel, blocks, st));
      HIP_TRY(hipMemcpyAsync(ctx->pinned, &P.glob->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      const int32_t flag = *(int32_t*)ctx->pinned;
      if (flag & kBadCap3)
        return fail(ctx, LYA_E_UNSUPPORTED, "more than %d partner pixels within r_max of one pixel",
                    xi3_partner_capacity());
      if (flag & kBadCapW)
        return fail(ctx, LYA_E_UNSUPPORTED, "more than %d partner pixels within r_max of one pixel",
                    kXi3WideCap);
      if (!(flag & kBadCapC)) break;
      if (o->variant == 0)
        return fail(ctx, LYA_E_UNSUPPORTED, "more than %d partner pixels within r_max of one pixel (variant 0)",
                    xi3_combine_capacity());
      // a pixel has more partners than the combining kernel holds: clear the
      // flag and the sums and run the wide kernel
      kernel = 2;
      HIP_TRY(launch_zero(&P.glob->flag, sizeof(int32_t), st));
      HIP_TRY(launch_zero(cn, (size_t)(n_copies * nout) * sizeof(double), st));
      HIP_TRY(launch_zero(cw, (size_t)(n_copies * nout) * sizeof(double), st));
      HIP_TRY(launch_zero(cc, (size_t)(n_copies * nout) * sizeof(unsigned long long), st));
    }
    if (n_copies > 1) HIP_TRY(launch_xi3_reduce(cn, cw, cc, n_copies, nout, nout, num, wsum, ntrip, st));
    tm.at(4);
  } else {
    tm.at(1);
    tm.at(2);
    tm.at(3);
    tm.at(4);
  }
  HIP_TRY(launch_finalize_xi(num, wsum, xi, nout, st));
  tm.at(5);
  return tm.finish(ctx);
}

}  // namespace

lya_status lya_xi3(lya_context* ctx, const lya_forests* F, const lya_grid3* G3, const lya_options* o,
                   void* stream, double* num, double* wsum, int64_t* ntrip, double* xi) {
  return xi3_impl(ctx, F, G3, o, stream, nullptr, 1, num, wsum, ntrip, xi);
}

lya_status lya_xi3_subsamples(lya_context* ctx, const lya_forests* F, const lya_grid3* G3,
                              const lya_options* o, void* stream, const int32_t* subsample, int32_t n_sub,
                              double* num, double* wsum, int64_t* ntrip, double* xi) {
  if (!ctx) return LYA_E_INVALID;
  if (!subsample) return fail(ctx, LYA_E_INVALID, "NULL subsample");
  return xi3_impl(ctx, F, G3, o, stream, subsample, n_sub, num, wsum, ntrip, xi);
}

lya_status lya_dmat(lya_context* ctx, const lya_forests* F, const lya_grid* G, const lya_options* o,
                    void* stream, double* dmat, double* wsum_d) {
  GridDev gd{};
  LYA_TRY(check_common(ctx, F, G, o, gd));
  if (o->deterministic) return fail(ctx, LYA_E_UNSUPPORTED, "options.deterministic is honoured by lya_xi only");
  if (!dmat || !wsum_d) return fail(ctx, LYA_E_INVALID, "NULL output dmat or wsum_d");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  ctx->err.clear();
  ctx->stats = lya_stats{};
  const int nb = gd.n_par * gd.n_perp;
  const int64_t R = F->n_realisations;
  Timer tm{ctx, st, o->timing != 0};
  tm.at(0);
  HIP_TRY(launch_zero(dmat, (size_t)R * nb * nb * sizeof(double), st));
  HIP_TRY(launch_zero(wsum_d, (size_t)R * nb * sizeof(double), st));
  if (F->n_forests > 0 && F->n_pix > 0) {
    Prepared P;
    LYA_TRY(prepare(ctx, F, G, gd, o, st, false, true, false, P));
    tm.at(1);
    const bool use_keep = o->dmat_keep_fraction < 1.0;
    const uint64_t thr = use_keep ? (uint64_t)ldexp(o->dmat_keep_fraction, 64) : ~0ull;
    Worklist W;
    LYA_TRY(build_worklist(ctx, F, gd, P, st, false, use_keep, thr, o->seed, true, 0, "dm", W));
    tm.at(2);
    ctx->stats.forest_pairs = W.n_pairs;
    ctx->stats.work_items = W.n_pairs;
    ctx->stats.candidate_pairs = W.candidates;
    unsigned int* counter;
    LYA_TRY(wst(ctx, "dm_counter", 2, &counter));
    DmatArgs a{};
    a.item_stride = 1;
    a.finfo = P.finfo;
    a.einfo = P.einfo;
    a.sorted = W.sorted;
    a.nbr = W.nbr;
    a.pair_p = W.pair_p;
    a.n_pairs = W.n_pairs;
    a.counter = counter;
    a.edges_perp = P.edges_perp;
    a.g = gd;
    // order the pairs by r_perp window so that pairs sharing a window share a tile
    {
      uint64_t *k_in, *k_out;
      int32_t *v_in, *v_out;
      LYA_TRY(wst(ctx, "dm_keys_in", (size_t)W.n_pairs, &k_in));
      LYA_TRY(wst(ctx, "dm_keys", (size_t)W.n_pairs, &k_out));
      LYA_TRY(wst(ctx, "dm_idx_in", (size_t)W.n_pairs, &v_in));
      LYA_TRY(wst(ctx, "dm_order", (size_t)W.n_pairs, &v_out));
      const size_t bytes = sort_keys_bytes(W.n_pairs);
      void* tmp;
      LYA_TRY(ws(ctx, "dm_sort_tmp", bytes, &tmp));
      HIP_TRY(launch_dmat_keys(a, k_in, v_in, st));
      HIP_TRY(launch_sort_keys(k_in, k_out, v_in, v_out, W.n_pairs, tmp, bytes, st));
      a.wkeys = k_out;
      a.worder = v_out;
      // at least ~64 items per workgroup of the widest variant, so that the
      // last items leave little idle time at the end of the launch (a forest
      // pair takes ~0.1 ms of one wave); at most kDmatChunk pairs per item
      // (each item adds its tile to the global numerator once per run)
      int max_wg = 0;
      for (int v = 0; v < dmat_num_variants(); ++v) {
        const int b = dmat_blocks_per_cu(v, o->precision);
        if (b > max_wg) max_wg = b;
      }
      const int64_t per = W.n_pairs / (64 * (int64_t)max_wg * ctx->n_cu);
      a.chunk = (int32_t)(per < 16 ? 16 : (per > kDmatChunk ? kDmatChunk : per));
      a.n_items = (W.n_pairs + a.chunk - 1) / a.chunk;
    }
    a.drec32 = P.drec32;
    a.drec64 = P.drec64;
    a.edges_par = P.edges_par;
    a.edges_perp = P.edges_perp;
    a.glob = P.glob;
    a.g = gd;
    a.dnum = dmat;
    a.wd = wsum_d;
    // the kept pair histograms of two-segment windows: one store sized for
    // the largest need over the variants (a launch indexes it by workgroup;
    // dmat_launch passes it only to a launch it covers)
    size_t hs_bytes = 0;
    for (int v = 0; v < dmat_num_variants(); ++v) {
      const size_t b = dmat_hsave_bytes_per_block(v, o->precision, kDmatHsaveRun) *
                       (size_t)dmat_blocks_per_cu(v, o->precision) * (size_t)ctx->n_cu;
      if (b > hs_bytes) hs_bytes = b;
    }
    {
      unsigned char* p = nullptr;
      if (hs_bytes > 0) LYA_TRY(wst(ctx, "dm_hsave", hs_bytes, &p));
      a.hsave = p;
      a.hsave_run = kDmatHsaveRun;
    }
    auto dmat_launch = [&](int v, const DmatArgs& args) -> hipError_t {
      const int blocks = dmat_blocks_per_cu(v, o->precision) * ctx->n_cu;
      DmatArgs x = args;
      if (dmat_hsave_bytes_per_block(v, o->precision, x.hsave_run) * (size_t)blocks > hs_bytes) x.hsave = nullptr;
      return launch_dmat(v, o->precision, x, blocks, st);
    };
    // variants: the kernels of dmat_num_variants(), then the hybrid launch:
    // the pairs whose window fits the small tile in one pass (the
    // sorted list puts them last) go to that kernel, two waves per SIMD, and
    // the wider windows to the large-tile kernel
    const int kHybrid = dmat_num_variants();
    int64_t n_wide = -1;
    auto launch_variant = [&](int v, const DmatArgs& args) -> lya_status {
      if (v < kHybrid) {
        HIP_TRY(launch_zero(counter, 4, st));
        HIP_TRY(dmat_launch(v, args));
        return LYA_OK;
      }
      constexpr int kSmall = 2, kBig = 1;  // dmat variants of the small and the large symmetric tile
      if (n_wide < 0) {
        const int max_span = 16 * dmat_wave_tile_blocks(kSmall - 1, o->precision) / gd.n_par;
        int64_t* dn;
        LYA_TRY(wst(ctx, "dm_wide", 1, &dn));
        HIP_TRY(launch_dmat_span_split(a.wkeys, a.n_pairs, max_span, dn, st));
        HIP_TRY(hipMemcpyAsync((char*)ctx->pinned + 64, dn, 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        n_wide = *(int64_t*)((char*)ctx->pinned + 64);
      }
      // (args may cover a prefix of the list: the autotuner's warm-up launch)
      DmatArgs wide = args, narrow = args;
      wide.n_pairs = n_wide < args.n_pairs ? n_wide : args.n_pairs;
      wide.n_items = (wide.n_pairs + args.chunk - 1) / args.chunk / args.item_stride;
      narrow.wkeys = args.wkeys + n_wide;
      narrow.worder = args.worder + n_wide;
      narrow.n_pairs = args.n_pairs > n_wide ? args.n_pairs - n_wide : 0;
      narrow.n_items = (narrow.n_pairs + args.chunk - 1) / args.chunk / args.item_stride;
      narrow.counter = counter + 1;
      HIP_TRY(launch_zero(counter, 8, st));
      HIP_TRY(dmat_launch(kBig, wide));
      HIP_TRY(dmat_launch(kSmall, narrow));
      return LYA_OK;
    };
    int variant = 0;
    if (o->variant >= 0) {
      if (o->variant > kHybrid)
        return fail(ctx, LYA_E_INVALID, "variant %d out of range (dmat has %d)", o->variant, kHybrid + 1);
      variant = o->variant;
    } else {
      char key[96];
      snprintf(key, sizeof key, "dmat/%d/%d", o->precision, nb);
      auto found = ctx->tuned.find(key);
      if (found != ctx->tuned.end()) {
        variant = found->second;
      } else if (o->autotune && W.n_pairs > 0 && dmat_num_variants() > 1) {
        // time each variant on a prefix of the pair list into scratch outputs
        double* sd;
        double* sw;
        LYA_TRY(wst(ctx, "tune_dnum", (size_t)R * nb * nb, &sd));
        LYA_TRY(wst(ctx, "tune_wd", (size_t)R * nb, &sw));
        DmatArgs t = a;
        t.dnum = sd;
        t.wd = sw;
        // a sample spread over the sorted pair list (window widths and pair
        // sizes change along it): every 4th chunk when there are enough, so
        // that each workgroup of each launch still takes ~16 items; one timed
        // launch per variant after a short one that loads its code
        if (a.n_items >= 4 * 64 * (int64_t)ctx->n_cu) {
          t.item_stride = 4;
          t.n_items = a.n_items / 4;
        }
        float best = 1e30f;
        for (int v = 0; v <= kHybrid; ++v) {
          float ms_v = 0.f;
          DmatArgs w = t;
          w.n_items = t.n_items < 16 ? t.n_items : 16;
          w.n_pairs = w.n_items * (int64_t)t.item_stride * t.chunk < t.n_pairs ? w.n_items * (int64_t)t.item_stride * t.chunk : t.n_pairs;
          LYA_TRY(launch_variant(v, w));
          HIP_TRY(hipEventRecord(ctx->ev[6], st));
          LYA_TRY(launch_variant(v, t));
          HIP_TRY(hipEventRecord(ctx->ev[7], st));
          HIP_TRY(hipEventSynchronize(ctx->ev[7]));
          HIP_TRY(hipEventElapsedTime(&ms_v, ctx->ev[6], ctx->ev[7]));
          if (ms_v < best) {
            best = ms_v;
            variant = v;
          }
        }
        ctx->tuned[key] = variant;
      }
    }
    const int blocks = dmat_blocks_per_cu(variant < kHybrid ? variant : 1, o->precision) * ctx->n_cu;
    ctx->stats.variant = variant;
    ctx->stats.grid_blocks = blocks;
    unsigned long long* wc = nullptr;
    if (o->counters) {
      LYA_TRY(wst(ctx, "dm_work_counters", 3, &wc));
      HIP_TRY(launch_zero(wc, 3 * sizeof(unsigned long long), st));
    }
    a.counters = wc;
    tm.at(3);
    LYA_TRY(launch_variant(variant, a));
    tm.at(4);
    if (wc) {
      HIP_TRY(hipMemcpyAsync((char*)ctx->pinned + 64, wc, 24, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      ctx->stats.ingrid_pairs = ((int64_t*)((char*)ctx->pinned + 64))[0];
      ctx->stats.outer_fmas = ((int64_t*)((char*)ctx->pinned + 64))[1];
      ctx->stats.lost_pairs = ((int64_t*)((char*)ctx->pinned + 64))[2];
    }
  } else {
    tm.at(1);
    tm.at(2);
    tm.at(3);
    tm.at(4);
  }
  HIP_TRY(launch_finalize_dmat(dmat, wsum_d, R * nb, nb, st));
  tm.at(5);
  return tm.finish(ctx);
}

lya_status lya_xi_backward(lya_context* ctx, const lya_forests* F, const lya_grid* G,
                           const lya_options* o, void* stream, const double* grad_xi,
                           const double* xi, const double* wsum, double* grad_delta,
                           double* grad_weight) {
  GridDev gd{};
  LYA_TRY(check_common(ctx, F, G, o, gd));
  if (o->deterministic) return fail(ctx, LYA_E_UNSUPPORTED, "options.deterministic is honoured by lya_xi only");
  if (!grad_xi || !xi || !wsum) return fail(ctx, LYA_E_INVALID, "NULL grad_xi, xi or wsum");
  if (!grad_delta || !grad_weight) return fail(ctx, LYA_E_INVALID, "NULL output grad_delta or grad_weight");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  ctx->err.clear();
  ctx->stats = lya_stats{};
  const int nb = gd.n_par * gd.n_perp;
  const int64_t R = F->n_realisations;
  Timer tm{ctx, st, o->timing != 0};
  tm.at(0);
  HIP_TRY(launch_zero(grad_delta, (size_t)F->n_pix * sizeof(double), st));
  HIP_TRY(launch_zero(grad_weight, (size_t)F->n_pix * sizeof(double), st));
  if (F->n_forests > 0 && F->n_pix > 0) {
    Prepared P;
    const bool project = o->project_deltas != 0;
    LYA_TRY(prepare(ctx, F, G, gd, o, st, true, false, project, P));
    tm.at(1);
    Worklist W;
    LYA_TRY(build_worklist(ctx, F, gd, P, st, true, false, 0, 0, false, INT32_MAX, "bw", W));
    tm.at(2);
    ctx->stats.forest_pairs = W.n_pairs;
    ctx->stats.work_items = W.n_items;
    ctx->stats.candidate_pairs = W.candidates;
    double2* gtab;
    LYA_TRY(wst(ctx, "bw_gamma", (size_t)R * nb, &gtab));
    HIP_TRY(launch_gamma(grad_xi, xi, wsum, gtab, R * nb, gd.n_par, gd.n_perp, st));
    unsigned int* counter;
    LYA_TRY(wst(ctx, "bw_counter", 1, &counter));
    BwdArgs a{};
    a.finfo = P.finfo;
    a.sorted = W.sorted;
    a.nbr = W.nbr;
    a.items = W.items;
    a.n_items = W.n_items;
    a.counter = counter;
    a.rec32 = P.rec32;
    a.rec64 = P.rec64;
    a.dist = F->dist;
    a.weight = F->weight;
    a.delta = project ? P.delta_proj : F->delta;
    a.edges_par = P.edges_par;
    a.edges_perp = P.edges_perp;
    a.glob = P.glob;
    a.g = gd;
    a.gtab = gtab;
    a.grad_delta = grad_delta;
    a.grad_weight = grad_weight;
    const int blocks = xi_bwd_blocks_per_cu(o->precision, nb) * ctx->n_cu;
    ctx->stats.grid_blocks = blocks;
    HIP_TRY(launch_zero(counter, 4, st));
    tm.at(3);
    HIP_TRY(launch_xi_bwd(o->precision, a, blocks, st));
    if (project) HIP_TRY(launch_project_adjoint(F, P.einfo, P.delta_proj, grad_delta, grad_weight, st));
    tm.at(4);
  } else {
    tm.at(1);
    tm.at(2);
    tm.at(3);
    tm.at(4);
  }
  tm.at(5);
  return tm.finish(ctx);
}

}  // extern "C"
