// The xi pair kernel: weighted pixel-pair histograms of Sec. 2.1,
// eq. estimator_two (numerator sum w_i d_i w_j d_j, denominator sum w_i w_j,
// pair count), over every work item of the forest-pair list.
//
// Layout of the work.  A work item is one forest f (at sorted position p)
// against up to kChunkMax neighbour forests g.  The neighbours' pixels form
// one concatenated stream; each wave takes 64 consecutive stream pixels, one
// per lane (coalesced loads, every lane busy except at the stream's end), and
// loops over the pixels of f, which are identical for all lanes and are read
// through the scalar cache.  Each lane thus evaluates one pixel pair per
// iteration: r_par = |D_i - D_j| c, r_perp = (D_i + D_j) s with the lane's own
// (s, c), then the bin and the two products.
//
// Histograms live in LDS, one copy per workgroup (FP64 sums, u32 counts), and
// are added to the global FP64 outputs when the workgroup finishes, when the
// realisation changes, or before a count could overflow.
//
// FP32 form.  Distances are re-centred on dc so FP32 keeps ~1e-4 Mpc/h.  A pair
// whose FP32 bin coordinate lies within the proven error bound (tau) of a bin
// edge is re-evaluated in FP64 with the same operations as the FP64 form and
// binned by comparison with the FP64 edges, so the FP32 and FP64 forms bin
// every pair identically.  Products are FP32 and are accumulated in FP64 in
// LDS (ds_add_f64 is native on gfx950 and moves the same bytes as a hi/lo
// pair of FP32 accumulators); with run-length accumulation, consecutive
// products of the same bin are first summed in FP32 registers (runs end at
// every 32nd pixel of f, so a run holds at most 32 products).
//
// Deterministic form (DET).  The run sums of the run-length form (at most 32
// products of one lane, summed in a fixed order in the form's arithmetic) are
// scaled by 2^s (s per realisation, from its largest |w d| and w, so that
// |run sum| 2^s <= 2^55), rounded to integers and summed exactly as two 64-bit
// words (low 28 bits and the rest), in LDS and then in global memory; integer
// addition does not depend on the order, so the sums are bitwise reproducible
// and identical for a realisation alone or batched (a run depends only on the
// forest pair and the pixel, not on how the work is split).
//
// Bin means.  The MEANS form also sums w_i w_j x_par, w_i w_j x_perp (the bin
// coordinates x = (r - e0) / dr the binning already computes) and
// w_i w_j (z_i + z_j), with the pixel redshift z packed in the record's fourth
// slot; a finalisation turns them into the weighted mean r_par, r_perp and z
// of each bin, the coordinate columns of the correlation output.
#include "lya_bin.h"
#include "lya_common.h"

namespace lya {

namespace {

constexpr unsigned kRunMax = 32;

struct NbTable {
  int64_t pix0[kChunkMax];
  int32_t pref[kChunkMax + 1];
  double s64[kChunkMax], c64[kChunkMax];
};

// Loads through the constant address space: with a wave-uniform address the
// compiler emits scalar (SMEM) loads.  Native vector types are used because
// class copies cannot bind to address-space-qualified objects.
typedef float lya_f4 __attribute__((ext_vector_type(4)));
typedef double lya_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ Rec32 load_uniform(const Rec32* p) {
  const lya_f4 v = *(const __attribute__((address_space(4))) lya_f4*)p;
  return Rec32{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ Rec64 load_uniform(const Rec64* p) {
  const lya_d4 v = *(const __attribute__((address_space(4))) lya_d4*)p;
  return Rec64{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ double load_uniform(const double* p) {
  return *(const __attribute__((address_space(4))) double*)p;
}

// Four FP32 records (64 bytes) or two FP64 records per scalar load.
typedef float lya_f16 __attribute__((ext_vector_type(16)));
typedef double lya_d8 __attribute__((ext_vector_type(8)));
template <typename Rec> struct Batch;
template <> struct Batch<Rec32> {
  static constexpr int N = 4;
  Rec32 r[4];
  __device__ __forceinline__ void load(const Rec32* p) {
    const lya_f16 v = *(const __attribute__((address_space(4))) lya_f16*)p;
    r[0] = Rec32{v[0], v[1], v[2], v[3]};
    r[1] = Rec32{v[4], v[5], v[6], v[7]};
    r[2] = Rec32{v[8], v[9], v[10], v[11]};
    r[3] = Rec32{v[12], v[13], v[14], v[15]};
  }
};
template <> struct Batch<Rec64> {
  static constexpr int N = 2;
  Rec64 r[2];
  __device__ __forceinline__ void load(const Rec64* p) {
    const lya_d8 v = *(const __attribute__((address_space(4))) lya_d8*)p;
    r[0] = Rec64{v[0], v[1], v[2], v[3]};
    r[1] = Rec64{v[4], v[5], v[6], v[7]};
  }
};

// Fixed-point terms of the deterministic form: q = rint(x), |q| <= 2^55, split
// as q = hi 2^28 + lo with 0 <= lo < 2^28; the two words are summed in separate
// 64-bit integers (two's complement for hi), exact for fewer than 2^36 terms.
// A term is a run sum of at most kRunMax = 2^5 products below m^2, so the
// scale is 2^(kDetBits - 2 e) = 2^(50 - 2 e) for m < 2^e.
constexpr int kDetShift = 28;
constexpr int kDetBits = 50;

__device__ __forceinline__ void det_add(unsigned long long* h, double x) {
  const long long q = __double2ll_rn(x);
  atomicAdd(&h[0], (unsigned long long)(q & ((1ll << kDetShift) - 1)));
  atomicAdd(&h[1], (unsigned long long)(q >> kDetShift));
}

// s for products below m^2, m given by the bits of a non-negative double:
// s = kDetBits - 2 e with m < 2^e (clamped to the double's range).  A run sum
// then stays below 2^5 m^2 2^s <= 2^55, and rounding it to an integer adds at
// most 0.5 2^-s = 2^(2 e - 51) <= 2^-49 m^2 (m >= 2^(e - 1)).
__device__ __forceinline__ int det_shift(unsigned long long mbits) {
  if (mbits == 0ull) return 0;
  const int E = (int)(mbits >> 52);
  const int e = (E == 0 ? 1 : E) - 1022;
  const int sh = kDetBits - 2 * e;
  return sh > 1000 ? 1000 : (sh < -1000 ? -1000 : sh);
}

template <typename T> struct RecOf;
template <> struct RecOf<float> { using type = Rec32; };
template <> struct RecOf<double> { using type = Rec64; };

// LDS histograms: hNW[2 L] = sum w_i d_i w_j d_j, hNW[2 L + 1] = sum w_i w_j
// (interleaved, so one address serves both), hn[L] = pair count; with MEANS,
// hM[3 L + c] = sum w_i w_j (x_par, x_perp, z_i + z_j)[c].
template <int BLOCK, bool MEANS>
__device__ void flush_hist(const XiArgs& a, double* hNW, double* hM, unsigned* hn, int real) {
  const int NP = a.g.n_par, NT = a.g.n_perp, nb = NP * NT;
  const int64_t base = (int64_t)real * nb;
  const int64_t nout = a.n_out;
  for (int L = threadIdx.x; L < nb; L += BLOCK) {
    const unsigned c = hn[L];
    if (c) {
      const int kp = L % NP, kt = L / NP;
      const int64_t A = base + (int64_t)kp * NT + kt;
      atomicAdd(&a.num[A], hNW[2 * L]);
      atomicAdd(&a.wsum[A], hNW[2 * L + 1]);
      atomicAdd(&a.npairs[A], (unsigned long long)c);
      if constexpr (MEANS) {
        atomicAdd(&a.msum[A], hM[3 * L]);
        atomicAdd(&a.msum[nout + A], hM[3 * L + 1]);
        atomicAdd(&a.msum[2 * nout + A], hM[3 * L + 2]);
      }
    }
    hNW[2 * L] = 0.0;
    hNW[2 * L + 1] = 0.0;
    if constexpr (MEANS) {
      hM[3 * L] = 0.0;
      hM[3 * L + 1] = 0.0;
      hM[3 * L + 2] = 0.0;
    }
    hn[L] = 0u;
  }
}

// Deterministic form's LDS sums: hq[4 L + c] (N low, N high, W low, W high),
// hn[L] = pair count.
template <int BLOCK>
__device__ void flush_det(const XiArgs& a, unsigned long long* hq, unsigned* hn, int real) {
  const int NP = a.g.n_par, NT = a.g.n_perp, nb = NP * NT;
  const int64_t base = (int64_t)real * nb;
  for (int L = threadIdx.x; L < nb; L += BLOCK) {
    const unsigned c = hn[L];
    if (c) {
      const int kp = L % NP, kt = L / NP;
      const int64_t A = base + (int64_t)kp * NT + kt;
#pragma unroll
      for (int w = 0; w < 4; ++w) atomicAdd(&a.det_acc[4 * A + w], hq[4 * L + w]);
      atomicAdd(&a.npairs[A], (unsigned long long)c);
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) hq[4 * L + w] = 0ull;
    hn[L] = 0u;
  }
}

template <typename T, int BLOCK, bool RLE, bool ZLO, bool MEANS, bool DET = false>
__global__ __launch_bounds__(BLOCK) void xi_kernel(XiArgs a) {
  static_assert(RLE || !MEANS, "bin means are accumulated by the run-length form");
  static_assert(!(DET && MEANS), "the deterministic form has no bin means");
  using Rec = typename RecOf<T>::type;
  extern __shared__ double smem[];
  __shared__ NbTable tb;
  __shared__ int64_t s_item;

  const int NP = a.g.n_par, NT = a.g.n_perp, nb = NP * NT;
  double* hNW = smem;
  double* hM = smem + 2 * nb;
  unsigned* hn = (unsigned*)(smem + (DET ? 4 : (MEANS ? 5 : 2)) * nb);
  unsigned long long* hq = (unsigned long long*)smem;  // DET
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  for (int L = threadIdx.x; L < nb; L += BLOCK) {
    if constexpr (DET) {
      hq[4 * L] = hq[4 * L + 1] = hq[4 * L + 2] = hq[4 * L + 3] = 0ull;
      hn[L] = 0u;
      continue;
    }
    hNW[2 * L] = 0.0;
    hNW[2 * L + 1] = 0.0;
    if constexpr (MEANS) {
      hM[3 * L] = 0.0;
      hM[3 * L + 1] = 0.0;
      hM[3 * L + 2] = 0.0;
    }
    hn[L] = 0u;
  }

  const Rec* __restrict__ recs;
  if constexpr (sizeof(T) == 4) recs = a.rec32; else recs = a.rec64;

  BinK<T, ZLO> K;
  K.init(a.g, a.glob, a.edges_par, a.edges_perp);
  // x-space constants: x_par = |d_i - d_j| cp + mep, x_perp = d_i st + bt_j
  const double dcx = sizeof(T) == 4 ? a.glob->dc : 0.0;  // FP32 distances are re-centred
  const double invp = a.g.inv_par, invt = a.g.inv_perp, e0t = a.g.e0_perp;
  const T mep = (T)(-a.g.e0_par * a.g.inv_par);

  int cur_key = -1;
  double pending = 0.0;  // upper bound on pairs added to any bin since the last flush
  double scN = 1.0, scW = 1.0;  // DET: 2^s of the current realisation
  __syncthreads();

  for (;;) {
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t it = s_item;
    if (it >= a.n_items) break;
    const Item item = a.items[it];
    const int f = a.sorted[item.p];
    const ForestInfo fi = a.finfo[f];
    const int nbc = item.nb_count;

    // neighbour table: geometry per forest pair, prefix of pixel counts
    if (threadIdx.x < 64) {
      int n = 0;
      if (lane < nbc) {
        const int g = a.sorted[a.nbr[item.nb_begin + lane]];
        const ForestInfo gi = a.finfo[g];
        double s, c;
        pair_sc(fi, gi, s, c);
        tb.pix0[lane] = gi.pix0;
        tb.s64[lane] = s;
        tb.c64[lane] = c;
        n = gi.npix;
      }
      int incl = n;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
      }
      if (lane < nbc) tb.pref[lane + 1] = incl;
      if (lane == 0) tb.pref[0] = 0;
    }
    __syncthreads();
    const int total = tb.pref[nbc];

    // output slab: the realisation, or realisation * n_sub + subsample of f
    const int okey = a.sub ? fi.real * a.n_sub + a.sub[f] : fi.real;
    if (okey != cur_key || pending + (double)total * fi.npix > a.flush_pairs) {
      if (cur_key >= 0) {
        if constexpr (DET) flush_det<BLOCK>(a, hq, hn, cur_key); else flush_hist<BLOCK, MEANS>(a, hNW, hM, hn, cur_key);
        __syncthreads();
      }
      cur_key = okey;
      pending = 0.0;
      if constexpr (DET) {
        scN = ldexp(1.0, det_shift(a.det_max[2 * okey]));
        scW = ldexp(1.0, det_shift(a.det_max[2 * okey + 1]));
      }
    }
    pending += (double)total * fi.npix;

    const Rec* __restrict__ rf = recs + fi.pix0;
    const int nf = fi.npix;

    for (int base = wave * 64; base < total; base += BLOCK) {
      const int q = base + lane;
      int k = 0;
      {
        int lo = 0, hi = nbc;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (tb.pref[mid] <= q) lo = mid; else hi = mid;
        }
        k = lo;
      }
      T dj, wdj, wj, zj = 0, cp, st, bt;
      double Dj64 = 0.0, s64 = 0.0, c64 = 1.0;
      if (q < total) {
        const int64_t j = tb.pix0[k] + (q - tb.pref[k]);
        const Rec rj = recs[j];
        dj = rj.d;
        wdj = rj.wd;
        wj = rj.w;
        zj = rj.del;  // the pixel redshift when the records carry z (MEANS)
        s64 = tb.s64[k];
        c64 = tb.c64[k];
        if constexpr (sizeof(T) == 4) Dj64 = a.dist[j]; else Dj64 = rj.d;
        cp = (T)(c64 * invp);
        st = (T)(s64 * invt);
        bt = (T)(((Dj64 + dcx) * s64 - e0t) * invt);
      } else {
        // out-of-range lane: a far-away pixel, never in the grid
        dj = (T)1e30;
        wdj = 0;
        wj = 0;
        cp = 1;
        st = 0;
        bt = (T)1e30;
      }

      // bin of the pair (pixel i of f, this lane's pixel), or -1; xp, xt are
      // its coordinates in bin units
      auto bin_of = [&](const Rec& ri, int i, T& xp, T& xt) -> int {
        const T ad = fabs(ri.d - dj);
        if constexpr (ZLO) xp = ad * cp; else xp = fma(ad, cp, mep);
        xt = fma(ri.d, st, bt);
        return K.bin_x(xp, xt, [&](double& rp64, double& rt64) {
          double Di64;
          if constexpr (sizeof(T) == 4) Di64 = load_uniform(a.dist + fi.pix0 + i); else Di64 = ri.d;
          separations64(Di64, Dj64, c64, s64, rp64, rt64);
        });
      };
      constexpr int NB = Batch<Rec>::N;

      if constexpr (RLE) {
        // runs of equal bins along f, ended at every kRunMax-th pixel of f (a run
        // sum holds at most kRunMax FP32 products); out-of-grid pairs form runs
        // with A = -1 that are never added
        for (int c0 = 0; c0 < nf; c0 += (int)kRunMax) {
          const int c1 = min(nf, c0 + (int)kRunMax);
          int curA = -1, ist = c0;
          T accN = 0, accW = 0, accP = 0, accT = 0, accZ = 0;
          auto add_run = [&](int A, int count) {
            if constexpr (DET) {
              det_add(&hq[4 * A], __dmul_rn((double)accN, scN));
              det_add(&hq[4 * A + 2], __dmul_rn((double)accW, scW));
              atomicAdd(&hn[A], (unsigned)count);
              return;
            }
            atomicAdd(&hNW[2 * A], (double)accN);
            atomicAdd(&hNW[2 * A + 1], (double)accW);
            atomicAdd(&hn[A], (unsigned)count);
            if constexpr (MEANS) {
              atomicAdd(&hM[3 * A], (double)accP);
              atomicAdd(&hM[3 * A + 1], (double)accT);
              atomicAdd(&hM[3 * A + 2], (double)accZ);
            }
          };
          auto pair = [&](const Rec& ri, int i) {
            T xp, xt;
            const int A = bin_of(ri, i, xp, xt);
            if (A != curA) {
              if (curA >= 0) add_run(curA, i - ist);
              curA = A;
              accN = 0;
              accW = 0;
              if constexpr (MEANS) {
                accP = 0;
                accT = 0;
                accZ = 0;
              }
              ist = i;
            }
            accN = fma(ri.wd, wdj, accN);
            if constexpr (MEANS) {
              const T ww = ri.w * wj;
              accW += ww;
              accP = fma(ww, xp, accP);
              accT = fma(ww, xt, accT);
              accZ = fma(ww, ri.del + zj, accZ);
            } else {
              accW = fma(ri.w, wj, accW);
            }
          };
          int i = c0;
          for (; i + NB <= c1; i += NB) {
            Batch<Rec> b;
            b.load(rf + i);
#pragma unroll
            for (int u = 0; u < NB; ++u) pair(b.r[u], i + u);
          }
          for (; i < c1; ++i) pair(load_uniform(rf + i), i);
          if (curA >= 0) add_run(curA, c1 - ist);
        }
      } else {
        auto pair = [&](const Rec& ri, int i) {
          T xp, xt;
          const int A = bin_of(ri, i, xp, xt);
          if (A >= 0) {
            if constexpr (DET) {
              det_add(&hq[4 * A], __dmul_rn((double)(ri.wd * wdj), scN));
              det_add(&hq[4 * A + 2], __dmul_rn((double)(ri.w * wj), scW));
            } else {
              atomicAdd(&hNW[2 * A], (double)(ri.wd * wdj));
              atomicAdd(&hNW[2 * A + 1], (double)(ri.w * wj));
            }
            atomicAdd(&hn[A], 1u);
          }
        };
        int i = 0;
        for (; i + NB <= nf; i += NB) {
          Batch<Rec> b;
          b.load(rf + i);
#pragma unroll
          for (int u = 0; u < NB; ++u) pair(b.r[u], i + u);
        }
        for (; i < nf; ++i) pair(load_uniform(rf + i), i);
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (cur_key >= 0) {
    if constexpr (DET) flush_det<BLOCK>(a, hq, hn, cur_key); else flush_hist<BLOCK, MEANS>(a, hNW, hM, hn, cur_key);
  }
}

struct Variant {
  const char* name;
  int block;
  bool rle;
};
constexpr Variant kVariants[] = {
    {"b256", 256, false},
    {"b512", 512, false},
    {"b256-rle", 256, true},
    {"b512-rle", 512, true},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <bool MEANS, bool DET = false>
constexpr size_t smem_per_bin() {
  return (DET ? 4 : (MEANS ? 5 : 2)) * sizeof(double) + sizeof(unsigned);
}

template <typename T, int BLOCK, bool RLE, bool ZLO, bool MEANS = false, bool DET = false>
hipError_t launch_one(const XiArgs& a, int blocks, hipStream_t st) {
  const size_t smem = (size_t)a.g.n_par * a.g.n_perp * smem_per_bin<MEANS, DET>();
  auto kern = xi_kernel<T, BLOCK, RLE, ZLO, MEANS, DET>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(BLOCK), smem, st, a);
  return hipGetLastError();
}

template <typename T, bool ZLO>
hipError_t launch_z(int v, const XiArgs& a, int blocks, hipStream_t st) {
  switch (v) {
    case 0: return launch_one<T, 256, false, ZLO>(a, blocks, st);
    case 1: return launch_one<T, 512, false, ZLO>(a, blocks, st);
    case 2: return launch_one<T, 256, true, ZLO>(a, blocks, st);
    case 3: return launch_one<T, 512, true, ZLO>(a, blocks, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_t(int v, const XiArgs& a, int blocks, hipStream_t st) {
  const bool zlo = a.g.zero_lo_par && a.g.zero_lo_perp;
  return zlo ? launch_z<T, true>(v, a, blocks, st) : launch_z<T, false>(v, a, blocks, st);
}

template <typename T, int BLOCK, bool RLE, bool MEANS = false, bool DET = false>
int occupancy(int n_bins) {
  const size_t smem = (size_t)n_bins * smem_per_bin<MEANS, DET>();
  auto kern = xi_kernel<T, BLOCK, RLE, true, MEANS, DET>;
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess) return 1;
  int nblk = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, kern, BLOCK, smem) != hipSuccess) return 1;
  return nblk > 0 ? nblk : 1;
}

template <typename T>
int occ_t(int v, int n_bins) {
  switch (v) {
    case 0: return occupancy<T, 256, false>(n_bins);
    case 1: return occupancy<T, 512, false>(n_bins);
    case 2: return occupancy<T, 256, true>(n_bins);
    case 3: return occupancy<T, 512, true>(n_bins);
  }
  return 1;
}

__global__ void zero_kernel(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Bin means from the sums of w_i w_j x (x in bin units) and w_i w_j (z_i + z_j):
// r = e0 + dr * sum(ww x) / W, z = sum(ww (z_i + z_j)) / (2 W); 0 where W = 0.
__global__ void finalize_means_kernel(const double* wsum, const double* msum, int64_t n, GridDev g,
                                      double* rpar, double* rperp, double* z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = wsum[i];
  const bool e = w == 0.0;
  rpar[i] = e ? 0.0 : g.e0_par + (msum[i] / w) / g.inv_par;
  rperp[i] = e ? 0.0 : g.e0_perp + (msum[n + i] / w) / g.inv_perp;
  z[i] = e ? 0.0 : 0.5 * (msum[2 * n + i] / w);
}

// Largest |w delta| and w of each realisation, as bits of non-negative doubles
// (their order is the doubles' order), one wave per forest.
__global__ __launch_bounds__(256) void det_max_kernel(lya_forests F, const ForestInfo* finfo, const double* delta,
                                                    unsigned long long* det_max) {
  const int lane = threadIdx.x & 63;
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (f >= F.n_forests) return;
  const ForestInfo fi = finfo[f];
  double mwd = 0.0, mw = 0.0;
  for (int k = lane; k < fi.npix; k += 64) {
    const int64_t i = fi.pix0 + k;
    const double w = F.weight[i];
    mwd = fmax(mwd, fabs(__dmul_rn(w, delta[i])));
    mw = fmax(mw, w);
  }
  for (int o = 32; o > 0; o >>= 1) {
    mwd = fmax(mwd, __shfl_xor(mwd, o, 64));
    mw = fmax(mw, __shfl_xor(mw, o, 64));
  }
  if (lane == 0) {
    atomicMax(&det_max[2 * fi.real], (unsigned long long)__double_as_longlong(mwd));
    atomicMax(&det_max[2 * fi.real + 1], (unsigned long long)__double_as_longlong(mw));
  }
}

// N, W from the integer sums: (hi 2^28 + lo) 2^-s.
__global__ void finalize_det_kernel(const unsigned long long* acc, const unsigned long long* det_max,
                                    const unsigned long long* npairs, int64_t n, int n_bins, double* num,
                                    double* wsum, Globals* glob) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t r = i / n_bins;
  const int sN = det_shift(det_max[2 * r]), sW = det_shift(det_max[2 * r + 1]);
  const double vn = __dadd_rn(ldexp((double)(long long)acc[4 * i + 1], kDetShift), (double)acc[4 * i]);
  const double vw = __dadd_rn(ldexp((double)(long long)acc[4 * i + 3], kDetShift), (double)acc[4 * i + 2]);
  num[i] = ldexp(vn, -sN);
  wsum[i] = ldexp(vw, -sW);
  if (npairs[i] >= (1ull << 36)) atomicOr(&glob->flag, kBadDet);
}

__global__ void finalize_xi_kernel(const double* num, const double* wsum, double* xi, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = wsum[i];
  xi[i] = w != 0.0 ? num[i] / w : 0.0;
}

}  // namespace

int xi_num_variants() { return kNumVariants; }
const char* xi_variant_name(int v) { return (v >= 0 && v < kNumVariants) ? kVariants[v].name : "?"; }

hipError_t launch_xi(int variant, int precision, const XiArgs& a, int blocks, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  return precision == LYA_FP64 ? launch_t<double>(variant, a, blocks, st)
                               : launch_t<float>(variant, a, blocks, st);
}

int xi_blocks_per_cu(int variant, int precision, int n_bins) {
  return precision == LYA_FP64 ? occ_t<double>(variant, n_bins) : occ_t<float>(variant, n_bins);
}

// The deterministic form: the run-length form with 1024 threads (its 36 B
// of LDS per bin leave one workgroup per CU at 2500 bins).
constexpr int kDetBlock = 1024;

hipError_t launch_xi_det(int precision, const XiArgs& a, int blocks, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  const bool zlo = a.g.zero_lo_par && a.g.zero_lo_perp;
  if (precision == LYA_FP64)
    return zlo ? launch_one<double, kDetBlock, true, true, false, true>(a, blocks, st)
               : launch_one<double, kDetBlock, true, false, false, true>(a, blocks, st);
  return zlo ? launch_one<float, kDetBlock, true, true, false, true>(a, blocks, st)
             : launch_one<float, kDetBlock, true, false, false, true>(a, blocks, st);
}

int xi_det_blocks_per_cu(int precision, int n_bins) {
  return precision == LYA_FP64 ? occupancy<double, kDetBlock, true, false, true>(n_bins)
                               : occupancy<float, kDetBlock, true, false, true>(n_bins);
}

hipError_t launch_det_max(const lya_forests* F, const ForestInfo* finfo, const double* delta,
                          unsigned long long* det_max, hipStream_t st) {
  if (F->n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(det_max_kernel, dim3((unsigned)((F->n_forests + 3) / 4)), dim3(256), 0, st, *F, finfo, delta,
                     det_max);
  return hipGetLastError();
}

hipError_t launch_finalize_det(const unsigned long long* det_acc, const unsigned long long* det_max,
                               const unsigned long long* npairs, int64_t n_out, int n_bins, double* num,
                               double* wsum, Globals* glob, hipStream_t st) {
  if (n_out == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_det_kernel, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st, det_acc, det_max,
                     npairs, n_out, n_bins, num, wsum, glob);
  return hipGetLastError();
}

// The bin-means form: one run-length variant, kMeansBlock threads (its
// histograms need 110 KB of LDS at 2500 bins, so one workgroup per CU; 16
// waves hide latency better than 8: 246 against 340 ms on the eBOSS-like
// workload).
constexpr int kMeansBlock = 1024;

hipError_t launch_xi_means(int precision, const XiArgs& a, int blocks, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  const bool zlo = a.g.zero_lo_par && a.g.zero_lo_perp;
  if (precision == LYA_FP64)
    return zlo ? launch_one<double, kMeansBlock, true, true, true>(a, blocks, st)
               : launch_one<double, kMeansBlock, true, false, true>(a, blocks, st);
  return zlo ? launch_one<float, kMeansBlock, true, true, true>(a, blocks, st)
             : launch_one<float, kMeansBlock, true, false, true>(a, blocks, st);
}

int xi_means_blocks_per_cu(int precision, int n_bins) {
  return precision == LYA_FP64 ? occupancy<double, kMeansBlock, true, true>(n_bins)
                               : occupancy<float, kMeansBlock, true, true>(n_bins);
}

hipError_t launch_finalize_means(const double* wsum, const double* msum, int64_t n, const GridDev& g,
                                 double* rpar, double* rperp, double* z, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_means_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, wsum, msum,
                     n, g, rpar, rperp, z);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const size_t n = bytes / 4;
  const unsigned blocks = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
}

hipError_t launch_finalize_xi(const double* num, const double* wsum, double* xi, int64_t n,
                              hipStream_t st) {
  if (n == 0 || xi == nullptr) return hipSuccess;
  hipLaunchKernelGGL(finalize_xi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, num, wsum, xi, n);
  return hipGetLastError();
}

}  // namespace lya
