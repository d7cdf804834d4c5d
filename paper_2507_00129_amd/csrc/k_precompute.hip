// Per-forest precompute: validation, FP64 projection sums (Sec. 2.2, eta),
// optional delta projection, sky unit vectors, line-of-sight extents, and the
// packed pixel records read by the pair kernels.
#include <math.h>

#include "lya_common.h"

namespace lya {

namespace {

constexpr int kWavesPerBlock = 4;
constexpr double kLyaAlphaAngstrom = 1215.67;  // Lyman-alpha rest wavelength

// Subsample ids must lie in [0, n_sub): they index output slabs.
__global__ void validate_sub_kernel(const int32_t* sub, int64_t n, int32_t n_sub, Globals* glob) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f < n && (sub[f] < 0 || sub[f] >= n_sub)) atomicOr(&glob->flag, kBadSub);
}

// One wave per forest.  Any violation sets a bit in glob->flag.
__global__ __launch_bounds__(256) void validate_kernel(lya_forests F, Globals* glob) {
  const int lane = threadIdx.x & 63;
  const int64_t f = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (f >= F.n_forests) return;
  int bad = 0;
  const int64_t p0 = F.offsets[f], p1 = F.offsets[f + 1];
  if (lane == 0) {
    if (f == 0 && p0 != 0) bad |= kBadOffsets;
    if (p1 < p0 || p0 < 0 || p1 > F.n_pix) bad |= kBadOffsets;
    if (f == F.n_forests - 1 && p1 != F.n_pix) bad |= kBadNpix;
    if (!isfinite(F.ra[f]) || !isfinite(F.dec[f])) bad |= kBadFinite;
    if (F.realisation) {
      const int r = F.realisation[f];
      if (r < 0 || r >= F.n_realisations) bad |= kBadReal;
    }
  }
  if (!(p1 < p0 || p0 < 0 || p1 > F.n_pix)) {
    for (int64_t i = p0 + lane; i < p1; i += 64) {
      const double d = F.dist[i], de = F.delta[i], w = F.weight[i], l = F.loglam[i];
      if (!isfinite(d) || !isfinite(de) || !isfinite(w) || !isfinite(l)) bad |= kBadFinite;
      if (!(w >= 0.0)) bad |= kBadWeight;
      if (!(d > 0.0)) bad |= kBadDist;
    }
  }
  if (bad) atomicOr(&glob->flag, bad);
}

// One wave per forest: geometry, extents, eta sums, projected deltas.
__global__ __launch_bounds__(256) void forest_stats_kernel(PrecomputeArgs a, lya_forests F) {
  const int lane = threadIdx.x & 63;
  const int64_t f = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (f >= F.n_forests) return;
  const int64_t p0 = F.offsets[f], p1 = F.offsets[f + 1];
  const int n = (int)(p1 - p0);

  double dmin = INFINITY, dmax = -INFINITY, W = 0.0, WL = 0.0;
  for (int k = lane; k < n; k += 64) {
    const double d = F.dist[p0 + k], w = F.weight[p0 + k];
    dmin = fmin(dmin, d);
    dmax = fmax(dmax, d);
    W += w;
    WL += w * F.loglam[p0 + k];
  }
  dmin = wave_min(dmin);
  dmax = wave_max(dmax);
  W = wave_sum(W);
  WL = wave_sum(WL);

  const bool active = a.eta_mode != LYA_ETA_IDENTITY && W > 0.0 && n > 0;
  const double lbar = active ? WL / W : 0.0;
  double S = 0.0;
  if (active) {
    for (int k = lane; k < n; k += 64) {
      const double am = F.loglam[p0 + k] - lbar;
      S += F.weight[p0 + k] * am * am;
    }
    S = wave_sum(S);
  }
  // the slope term is dropped when Lambda has no weighted spread
  const int slope = active && a.eta_mode == LYA_ETA_MEAN_SLOPE && S > 1e-24 * W * lbar * lbar;

  if (a.project) {
    if (active) {
      double sd = 0.0, sad = 0.0;
      for (int k = lane; k < n; k += 64) {
        const double w = F.weight[p0 + k], de = F.delta[p0 + k];
        sd += w * de;
        sad += w * (F.loglam[p0 + k] - lbar) * de;
      }
      sd = wave_sum(sd);
      sad = wave_sum(sad);
      const double mean = sd / W, slope_c = slope ? sad / S : 0.0;
      for (int k = lane; k < n; k += 64) {
        const double de = F.delta[p0 + k];
        a.delta_proj[p0 + k] = slope ? (de - mean) - (F.loglam[p0 + k] - lbar) * slope_c : de - mean;
      }
    } else {
      for (int k = lane; k < n; k += 64) a.delta_proj[p0 + k] = F.delta[p0 + k];
    }
  }

  if (lane == 0) {
    const double ra = F.ra[f], dec = F.dec[f];
    const double cd = cos(dec);
    ForestInfo fi;
    fi.nx = cd * cos(ra);
    fi.ny = cd * sin(ra);
    fi.nz = sin(dec);
    fi.dmin = dmin;
    fi.dmax = dmax;
    fi.pix0 = p0;
    fi.npix = n;
    fi.real = F.realisation ? F.realisation[f] : 0;
    a.finfo[f] = fi;
    EtaInfo e;
    e.W = W;
    e.lbar = lbar;
    e.S = S;
    e.slope = slope;
    e.active = active;
    a.einfo[f] = e;
    if (n > 0) {
      // positive doubles order like their bit patterns
      atomicMin(&a.glob->dmin_bits, (unsigned long long)__double_as_longlong(dmin));
      atomicMax(&a.glob->dmax_bits, (unsigned long long)__double_as_longlong(dmax));
    }
  }
}

// Re-centring distance and FP32 edge-guard widths (single thread).
// u = 2^-24, M = max |D - dc|, N = number of bins on the axis, and
// s_max = e_perp_max / (2 Dmin), which bounds s for any pair near or inside
// the grid.  Two FP32 forms are in use:
//  r-space form, r_par = |d_i - d_j| c and r_perp = (d_i + d_j) s + fl(2 dc s),
//  then x = (r - e0) / dr:
//   |x_par32 - x_par|   <= u (2 M + 5 e_par_max + |e0|) / dr
//   |x_perp32 - x_perp| <= u (8 M s_max + 4 e_perp_max + |e0|) / dr
//  x-space form, x_par = |d_i - d_j| fl(c / dr) - fl(e0 / dr) and
//  x_perp = d_i fl(s / dr) + fl(((D_j + dc) s - e0) / dr) (one FMA each):
//   |x_par32 - x_par|   <= u ((2 M + 3 |e0|) / dr + 3 (N + 2))
//   |x_perp32 - x_perp| <= u (((3 M + 2 |dc|) s_max + |e0|) / dr + N + 2)
// The guard half-widths are twice the larger bound, in bin units.
__global__ void globals_kernel(PrecomputeArgs a) {
  Globals* g = a.glob;
  const double dmin = __longlong_as_double((long long)g->dmin_bits);
  const double dmax = __longlong_as_double((long long)g->dmax_bits);
  double dc = 0.5 * (dmin + dmax);
  if (!isfinite(dc)) dc = 0.0;
  dc = (double)(float)dc;
  const double m = fmax(fabs(dmax - dc), fabs(dc - dmin));
  g->dc = dc;
  g->m = isfinite(m) ? m : 0.0;
  const double M = g->m;
  const double u = 5.9604644775390625e-08;  // 2^-24
  const double smax = (dmin > 0.0 && isfinite(dmin)) ? fmin(1.0, a.eperp_max / (2.0 * dmin)) : 1.0;
  const double np = (a.epar_max - a.e0_par) * a.inv_par, nt = (a.eperp_max - a.e0_perp) * a.inv_perp;
  const double tp_r = u * (2.0 * M + 5.0 * a.epar_max + fabs(a.e0_par)) * a.inv_par;
  const double tt_r = u * (8.0 * M * smax + 4.0 * a.eperp_max + fabs(a.e0_perp)) * a.inv_perp;
  const double tp_x = u * ((2.0 * M + 3.0 * fabs(a.e0_par)) * a.inv_par + 3.0 * (np + 2.0));
  const double tt_x = u * (((3.0 * M + 2.0 * fabs(dc)) * smax + fabs(a.e0_perp)) * a.inv_perp + nt + 2.0);
  g->tau_par = (float)(2.0 * fmax(tp_r, tp_x));
  g->tau_perp = (float)(2.0 * fmax(tt_r, tt_x));
}

// One wave per forest: pack pixel records.
__global__ __launch_bounds__(256) void pack_kernel(PrecomputeArgs a, lya_forests F) {
  const int lane = threadIdx.x & 63;
  const int64_t f = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (f >= F.n_forests) return;
  const ForestInfo fi = a.finfo[f];
  const EtaInfo e = a.einfo[f];
  const double dc = a.glob->dc;
  const double* del = a.project ? a.delta_proj : F.delta;
  for (int k = lane; k < fi.npix; k += 64) {
    const int64_t i = fi.pix0 + k;
    const double D = F.dist[i], w = F.weight[i], de = del[i];
    const double wd = w * de;
    // fourth slot: delta, or the pixel redshift lambda / lambda_Lya - 1 with
    // lambda = exp(loglam) Angstrom (bin means)
    const double x4 = a.pack_z ? exp(F.loglam[i]) / kLyaAlphaAngstrom - 1.0 : de;
    if (a.want_xi32) a.rec32[i] = Rec32{(float)(D - dc), (float)wd, (float)w, (float)x4};
    if (a.want_xi64) a.rec64[i] = Rec64{D, wd, w, x4};
    if (a.want_d32 || a.want_d64) {
      const bool act = e.active != 0;
      const double am = act ? F.loglam[i] - e.lbar : 0.0;
      const double uu = act ? w / e.W : 0.0;
      const double bb = e.slope ? w * am / e.S : 0.0;
      const double aa = e.slope ? am : 0.0;
      if (a.want_d32) a.drec32[i] = DRec32{(float)(D - dc), (float)w, (float)aa, (float)uu, (float)bb, 0.f, D};
      if (a.want_d64) a.drec64[i] = DRec64{D, w, aa, uu, bb, 0.0};
    }
  }
}

inline unsigned blocks_for(int64_t n_forests) {
  return (unsigned)((n_forests + kWavesPerBlock - 1) / kWavesPerBlock);
}

}  // namespace

hipError_t launch_validate(const lya_forests* F, Globals* glob, hipStream_t st) {
  if (F->n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(validate_kernel, dim3(blocks_for(F->n_forests)), dim3(256), 0, st, *F, glob);
  return hipGetLastError();
}

hipError_t launch_validate_sub(const int32_t* sub, int64_t n_forests, int32_t n_sub, Globals* glob,
                               hipStream_t st) {
  if (n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(validate_sub_kernel, dim3((unsigned)((n_forests + 255) / 256)), dim3(256), 0, st, sub,
                     n_forests, n_sub, glob);
  return hipGetLastError();
}

hipError_t launch_forest_stats(const PrecomputeArgs& a, hipStream_t st) {
  if (a.F->n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(forest_stats_kernel, dim3(blocks_for(a.F->n_forests)), dim3(256), 0, st, a, *a.F);
  return hipGetLastError();
}

hipError_t launch_globals(const PrecomputeArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(globals_kernel, dim3(1), dim3(1), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pack(const PrecomputeArgs& a, hipStream_t st) {
  if (a.F->n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(a.F->n_forests)), dim3(256), 0, st, a, *a.F);
  return hipGetLastError();
}

}  // namespace lya
