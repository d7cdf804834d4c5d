// Pair binning shared by the xi, distortion and backward kernels.
//
// On a grid with non-uniform edges the coordinates below use the mean bin width
// and every pair in range takes the FP64 edge-array path (GridDev::exact_all).
//
// A pair's bin coordinates are x = (r - e0) / dr on each axis.  In FP32 the
// separations carry a bounded rounding error (tau bins, computed per call from
// the data, see globals_kernel); a pair whose coordinate lies within tau of an
// integer (a bin edge) is re-evaluated in FP64 with exactly the operations of
// the FP64 form and binned by comparison with the FP64 edge array, so FP32 and
// FP64 give the same bin for every pair.  The FP64 form uses the same scheme
// with a tau of 1e-8 bins to settle ties against the edge array.  A zero lower
// edge needs no guard because separations are never negative.
#pragma once

#include "lya_common.h"

namespace lya {

// ZLO: both first edges are exactly 0 (the usual grid); the lower-edge
// tests then vanish because separations are never negative.
template <typename T, bool ZLO = false>
struct BinK {
  T e0p, e0t, invp, invt;
  T np_hi, nt_hi, lo_p, lo_t;
  T rp_hi, rt_hi, rp_lo, rt_lo;  // conservative r-space window (rejects most pairs)
  T taup, taut;
  int NP, NT;
  bool zlp, zlt;
  const double* ep;
  const double* et;

  __device__ __forceinline__ void init(const GridDev& g, const Globals* glob, const double* edges_par,
                                       const double* edges_perp) {
    NP = g.n_par;
    NT = g.n_perp;
    e0p = (T)g.e0_par;
    e0t = (T)g.e0_perp;
    invp = (T)g.inv_par;
    invt = (T)g.inv_perp;
    if constexpr (sizeof(T) == 4) {
      taup = glob->tau_par;
      taut = glob->tau_perp;
    } else {
      taup = 1e-8;
      taut = 1e-8;
    }
    if (g.exact_all) {
      // non-uniform edges: a guard half width of a whole (mean) bin sends every
      // pair in range to the FP64 search of the edge arrays
      taup = (T)1;
      taut = (T)1;
    }
    np_hi = (T)NP + taup;
    nt_hi = (T)NT + taut;
    zlp = g.zero_lo_par;
    zlt = g.zero_lo_perp;
    lo_p = zlp ? (T)-1 : -taup;
    lo_t = zlt ? (T)-1 : -taut;
    // r-space window: the x-space window widened by one more tau, so that the
    // FP rounding of the conversion never rejects a pair the x test accepts
    rp_hi = (T)(g.emax_par + 2.0 * (double)taup / g.inv_par);
    rt_hi = (T)(g.emax_perp + 2.0 * (double)taut / g.inv_perp);
    rp_lo = zlp ? (T)-1 : (T)(g.e0_par - 2.0 * (double)taup / g.inv_par);
    rt_lo = zlt ? (T)-1 : (T)(g.e0_perp - 2.0 * (double)taut / g.inv_perp);
    ep = edges_par;
    et = edges_perp;
  }

  // Cheap conservative test: false means the pair is certainly outside the grid.
  __device__ __forceinline__ bool may_be_in(T rp, T rt) const {
    if constexpr (ZLO) return (rp < rp_hi) & (rt < rt_hi);
    else return (rp < rp_hi) & (rt < rt_hi) & (rp > rp_lo) & (rt > rt_lo);
  }

  // Local (LDS) bin index kt * NP + kp of a pair with separations (rp, rt),
  // or -1 outside the grid.  exact() returns the FP64 separations; it is
  // called only for pairs within tau of an edge.
  template <typename Exact>
  __device__ __forceinline__ int bin(T rp, T rt, Exact&& exact) const {
    if (!may_be_in(rp, rt)) return -1;
    return bin_near(rp, rt, exact);
  }

  // bin() for a pair that passed may_be_in().
  template <typename Exact>
  __device__ __forceinline__ int bin_near(T rp, T rt, Exact&& exact) const {
    if constexpr (ZLO) return bin_x(rp * invp, rt * invt, exact);
    else return bin_x((rp - e0p) * invp, (rt - e0t) * invt, exact);
  }

  // Bin of a pair from its coordinates in bin units, x = (r - e0) / dr, each
  // within tau of the exact FP64 value.  A pair within tau of an edge is binned
  // from exact()'s FP64 separations against the edge arrays; a zero lower edge
  // needs no guard (separations are never negative).  Away from the edges,
  // x < N + tau already implies x < N - tau, so no second range test is needed.
  template <typename Exact>
  __device__ __forceinline__ int bin_x(T xp, T xt, Exact&& exact) const {
    int A = -1;
    if ((xp < np_hi) & (xt < nt_hi) & (ZLO || ((xp > lo_p) & (xt > lo_t)))) {
      const T rxp = rint(xp), rxt = rint(xt);
      bool gp = fabs(xp - rxp) < taup;
      bool gt = fabs(xt - rxt) < taut;
      if constexpr (ZLO) {
        // r_par = 0 is common (aligned pixel grids); r_perp ~ 0 needs coincident
        // sky positions and is left to the exact path
        gp &= rxp != (T)0;
      } else {
        gp &= !(zlp & (rxp == (T)0));
        gt &= !(zlt & (rxt == (T)0));
      }
      if (gp | gt) {
        double rp64, rt64;
        exact(rp64, rt64);
        const int kp = bin_exact(rp64, ep, NP, (int)floor((double)xp));
        const int kt = bin_exact(rt64, et, NT, (int)floor((double)xt));
        A = (kp >= 0 && kt >= 0) ? (int)__umul24((unsigned)kt, (unsigned)NP) + kp : -1;
      } else {
        // both factors are below 2^24 (at most 4096 bins per axis): a 24-bit
        // multiply-add instead of a 64-bit one
        A = (int)__umul24((unsigned)(int)xt, (unsigned)NP) + (int)xp;
      }
    }
    return A;
  }
};

// Separations of a pixel pair in the working precision.  FP32: distances are
// re-centred (d = D - dc) and b = fl32(2 dc s), so r_perp = (d_i + d_j) s + b.
__device__ __forceinline__ void separations(float di, float dj, float c, float s, float b, float& rp,
                                            float& rt) {
  rp = fabsf(di - dj) * c;
  rt = fmaf(di + dj, s, b);
}
__device__ __forceinline__ void separations(double di, double dj, double c, double s, double,
                                            double& rp, double& rt) {
  rp = __dmul_rn(fabs(__dsub_rn(di, dj)), c);
  rt = __dmul_rn(__dadd_rn(di, dj), s);
}
// FP64 separations exactly as defined (used by the FP32 edge guard too).
__device__ __forceinline__ void separations64(double Di, double Dj, double c, double s, double& rp,
                                              double& rt) {
  rp = __dmul_rn(fabs(__dsub_rn(Di, Dj)), c);
  rt = __dmul_rn(__dadd_rn(Di, Dj), s);
}

// Global output index A = kp * NT + kt of a local index L = kt * NP + kp.
__device__ __forceinline__ int out_index(int L, int NP, int NT) {
  const int kt = L / NP, kp = L - kt * NP;
  return kp * NT + kt;
}

}  // namespace lya
