// Distortion matrix (Sec. 2.2, eq. distortion):
//   D_AB = w_A^-1 sum_{(i,j) in A} w_i w_j sum_{(i',j') in B} eta_ii' eta_jj'
// over the kept forest pairs, with eta_ii' = delta_ii' - p_i . q_i',
// p_i = (1, a_i), q_i' = (u_i', b_i')  (a = L - Lbar, u = w/W, b = w a / S).
//
// Expanding eta_ii' eta_jj' turns the four nested sums of one forest pair into
//   num_AB = w_A^{fg} [A = B]
//          - sum_i w_i sum_l R^l_i[A] G^l_i[B]     (row i of f, j and j' in g)
//          - sum_j w_j sum_k C^k_j[A] F^k_j[B]     (row j of g, i and i' in f)
//          + sum_kl H^kl_A Q^kl_B
// with row histograms R^l_i[A] = sum_{j: A(i,j)=A} w_j p_j^l,
// G^l_i[B] = sum_{j: A(i,j)=B} q_j^l (C, F alike with f and g swapped) and
// pair histograms H^kl_A = sum_{A} w_i p_i^k w_j p_j^l, Q^kl_B = sum_B q_i^k q_j^l.
//
// Work layout.  A forest pair only reaches the r_perp bins between
// (Dmin_f + Dmin_g) s and (Dmax_f + Dmax_g) s, a "window" of a few k_perp
// rows, so D is banded in k_perp.  Kept pairs are sorted by (realisation,
// first k_perp, span); a work item is a chunk of consecutive sorted pairs, and
// all pairs of a chunk that share a window accumulate into one FP64 LDS tile
// over that window (in blocks of kTileW x kTileW window bins when the window
// is wider), which is added to the global FP64 numerator once per chunk.  The
// waves of a workgroup process different forest pairs of the chunk at the same
// time; within a wave the lanes sweep the pixels of one forest against one
// pixel of the other, building the row histograms (and, in the first sweep,
// H and Q) in wave-private LDS, and each row's outer product is added to the
// tile.  Bins come from the shared binner, so a pixel pair falls in the same
// bin here as in the xi kernel.
#include "lya_bin.h"
#include "lya_common.h"

namespace lya {

namespace {

constexpr int kTileW = 100;  // window bins per tile side: 100 x 100 FP64 = 80 KB

template <typename T> struct DRecOf;
template <> struct DRecOf<float> { using type = DRec32; };
template <> struct DRecOf<double> { using type = DRec64; };

// Per-wave scratch.  R and G hold the two components (l = 0, 1) of a row
// histogram interleaved, so one 2-element load fetches both.  Flags are whole
// dwords: lanes flagging neighbouring bins must not share a dword.
template <typename T>
struct WaveBuf {
  T H[4][kTileW];
  T Q[4][kTileW];
  __attribute__((aligned(16))) T R[kTileW][2];
  __attribute__((aligned(16))) T G[kTileW][2];
  uint32_t fA[kTileW], fB[kTileW], fH[kTileW], fQ[kTileW];
  uint8_t lA[kTileW], lB[kTileW], lH[kTileW], lQ[kTileW];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Compacts the flagged entries of fl[0..n) into list (ascending) and clears
// the flags.  Returns the count (wave-uniform).
__device__ __forceinline__ int wave_compact(uint32_t* fl, uint8_t* list, int n, int lane) {
  int m = 0;
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int x0 = 0; x0 < n; x0 += 64) {
    const int x = x0 + lane;
    const bool on = x < n && fl[x];
    const uint64_t b = __ballot(on);
    if (on) {
      list[m + __popcll(b & lt)] = (uint8_t)x;
      fl[x] = 0;
    }
    m += __popcll(b);
  }
  return m;
}

// Calls f(x, y) for every x in la[0..ma), y in lb[0..mb), spread over the
// lanes: lane k starts at flat index k = u mb + v and advances by 64 with an
// incremental (u, v) update instead of a division.
template <typename F>
__device__ __forceinline__ void wave_outer(const uint8_t* la, int ma, const uint8_t* lb, int mb, int lane,
                                           F&& f) {
  if (ma == 0 || mb == 0) return;
  const int du = 64 / mb, dv = 64 - du * mb;
  int u = lane / mb, v = lane - (lane / mb) * mb;
  for (; u < ma;) {
    f((int)la[u], (int)lb[v]);
    u += du;
    v += dv;
    if (v >= mb) {
      v -= mb;
      ++u;
    }
  }
}

template <typename T, int BLOCK, bool ZLO>
__global__ __launch_bounds__(BLOCK) void dmat_kernel(DmatArgs a) {
  using Rec = typename DRecOf<T>::type;
  constexpr int NW = BLOCK / 64, TW = kTileW;
  __shared__ double tile[TW * TW];
  __shared__ double wdacc[TW];
  __shared__ WaveBuf<T> wbuf[NW];
  __shared__ int64_t s_item;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  BinK<T, ZLO> K;
  K.init(a.g, a.glob, a.edges_par, a.edges_perp);
  const int NP = K.NP, NT = K.NT, nb = NP * NT;
  const double dc2 = 2.0 * a.glob->dc;
  const Rec* __restrict__ recs;
  if constexpr (sizeof(T) == 4) recs = a.drec32; else recs = a.drec64;
  WaveBuf<T>& W = wbuf[wave];
  for (int x = lane; x < TW; x += 64) {
    for (int m = 0; m < 4; ++m) {
      W.H[m][x] = 0;
      W.Q[m][x] = 0;
    }
    W.R[x][0] = W.R[x][1] = W.G[x][0] = W.G[x][1] = 0;
    W.fA[x] = W.fB[x] = W.fH[x] = W.fQ[x] = 0;
  }
  unsigned long long n_in = 0, n_fma = 0, n_lost = 0;  // statistics only

  for (;;) {
    if (tid == 0) s_item = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t it = s_item;
    if (it >= a.n_items) break;
    const int64_t k0 = it * a.chunk;
    const int64_t k1 = min(a.n_pairs, k0 + (int64_t)a.chunk);
    for (int64_t r0 = k0; r0 < k1;) {
      const uint64_t key = a.wkeys[r0];
      int64_t lo = r0 + 1, hi = k1;  // end of the run of equal keys
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.wkeys[mid] == key) lo = mid + 1; else hi = mid;
      }
      const int64_t r1 = lo;
      if (key == ~0ull) {
        r0 = r1;
        continue;
      }
      const int real = (int)(key >> 40);
      const int kt0 = (int)((key >> 16) & 0xFFFFFF);
      const int span = (int)(key & 0xFFFF);
      const int nwin = span * NP;
      const int base_L = kt0 * NP;  // window index w = L - kt0 NP
      const int nblk = (nwin + TW - 1) / TW;
      const int64_t obase = (int64_t)real * nb;
      auto win_out = [&](int w) { return out_index(w + base_L, NP, NT); };

      for (int ab = 0; ab < nblk; ++ab) {
        const int a0 = ab * TW, na = min(TW, nwin - a0);
        for (int bb = 0; bb < nblk; ++bb) {
          const int b0 = bb * TW, nbk = min(TW, nwin - b0);
          for (int e = tid; e < na * nbk; e += BLOCK) tile[e] = 0.0;
          for (int x = tid; x < na; x += BLOCK) wdacc[x] = 0.0;
          __syncthreads();
          const bool first_pass = ab == 0 && bb == 0;

          for (int64_t kk = r0 + wave; kk < r1; kk += NW) {
            const int q = a.worder[kk];
            const ForestInfo fi = a.finfo[a.sorted[a.pair_p[q]]];
            const ForestInfo gi = a.finfo[a.sorted[a.nbr[q]]];
            double s64, c64;
            pair_sc(fi, gi, s64, c64);
            const T s = (T)s64, c = (T)c64;
            const T bsep = sizeof(T) == 4 ? (T)(dc2 * s64) : (T)0;
            const Rec* __restrict__ rf = recs + fi.pix0;
            const Rec* __restrict__ rg = recs + gi.pix0;
            const int nf = fi.npix, ng = gi.npix;

            // window index of pixel pair (ri in f, rj in g), or -1
            auto wbin = [&](const Rec& ri, const Rec& rj) -> int {
              T rp, rt;
              separations(ri.d, rj.d, c, s, bsep, rp, rt);
              if (!K.may_be_in(rp, rt)) return -1;
              const int L = K.bin_near(rp, rt, [&](double& rp64, double& rt64) {
                if constexpr (sizeof(T) == 4) {
                  separations64(ri.D, rj.D, c64, s64, rp64, rt64);
                } else {
                  rp64 = rp;
                  rt64 = rt;
                }
              });
              if (L < 0) return -1;
              const int w = L - base_L;
              if ((unsigned)w >= (unsigned)nwin) {
                ++n_lost;
                return -1;
              }
              return w;
            };

            // ---- sweep 1: rows i of f; R, G per row and the pair histograms H, Q
            for (int i = 0; i < nf; ++i) {
              const Rec ri = rf[i];
              for (int j = lane; j < ng; j += 64) {
                const Rec rj = rg[j];
                const int w = wbin(ri, rj);
                if (w < 0) continue;
                if (first_pass) ++n_in;
                const int x = w - a0, y = w - b0;
                if ((unsigned)x < (unsigned)na) {
                  const T ww = ri.w * rj.w;
                  atomicAdd(&W.R[x][0], rj.w);
                  atomicAdd(&W.R[x][1], rj.w * rj.a);
                  atomicAdd(&W.H[0][x], ww);
                  atomicAdd(&W.H[1][x], ww * rj.a);
                  atomicAdd(&W.H[2][x], ri.a * ww);
                  atomicAdd(&W.H[3][x], ri.a * ww * rj.a);
                  W.fA[x] = 1;
                  W.fH[x] = 1;
                }
                if ((unsigned)y < (unsigned)nbk) {
                  atomicAdd(&W.G[y][0], rj.u);
                  atomicAdd(&W.G[y][1], rj.b);
                  atomicAdd(&W.Q[0][y], ri.u * rj.u);
                  atomicAdd(&W.Q[1][y], ri.u * rj.b);
                  atomicAdd(&W.Q[2][y], ri.b * rj.u);
                  atomicAdd(&W.Q[3][y], ri.b * rj.b);
                  W.fB[y] = 1;
                  W.fQ[y] = 1;
                }
              }
              wave_sync();
              const int mA = wave_compact(W.fA, W.lA, na, lane);
              const int mB = wave_compact(W.fB, W.lB, nbk, lane);
              wave_sync();
              const T wneg = -ri.w;
              wave_outer(W.lA, mA, W.lB, mB, lane, [&](int x, int y) {
                atomicAdd(&tile[x * nbk + y], (double)(wneg * (W.R[x][0] * W.G[y][0] + W.R[x][1] * W.G[y][1])));
              });
              if (lane == 0) n_fma += 2ull * (unsigned long long)(mA * mB);
              wave_sync();
              for (int u = lane; u < mA; u += 64) W.R[W.lA[u]][0] = W.R[W.lA[u]][1] = 0;
              for (int v = lane; v < mB; v += 64) W.G[W.lB[v]][0] = W.G[W.lB[v]][1] = 0;
              wave_sync();
            }

            // ---- H (x) Q and the Kronecker term of this pair
            {
              const int mH = wave_compact(W.fH, W.lH, na, lane);
              const int mQ = wave_compact(W.fQ, W.lQ, nbk, lane);
              wave_sync();
              wave_outer(W.lH, mH, W.lQ, mQ, lane, [&](int x, int y) {
                double v = (double)(W.H[0][x] * W.Q[0][y] + W.H[1][x] * W.Q[1][y] +
                                    W.H[2][x] * W.Q[2][y] + W.H[3][x] * W.Q[3][y]);
                if (a0 + x == b0 + y) v += (double)W.H[0][x];
                atomicAdd(&tile[x * nbk + y], v);
              });
              if (bb == 0)
                for (int u = lane; u < mH; u += 64) atomicAdd(&wdacc[W.lH[u]], (double)W.H[0][W.lH[u]]);
              if (lane == 0) n_fma += 4ull * (unsigned long long)(mH * mQ);
              wave_sync();
              for (int u = lane; u < mH; u += 64) {
                const int x = W.lH[u];
                W.H[0][x] = W.H[1][x] = W.H[2][x] = W.H[3][x] = 0;
              }
              for (int v = lane; v < mQ; v += 64) {
                const int y = W.lQ[v];
                W.Q[0][y] = W.Q[1][y] = W.Q[2][y] = W.Q[3][y] = 0;
              }
              wave_sync();
            }

            // ---- sweep 2: rows j of g; C, F per row (roles of f and g swapped)
            for (int j = 0; j < ng; ++j) {
              const Rec rj = rg[j];
              for (int i = lane; i < nf; i += 64) {
                const Rec ri = rf[i];
                const int w = wbin(ri, rj);
                if (w < 0) continue;
                const int x = w - a0, y = w - b0;
                if ((unsigned)x < (unsigned)na) {
                  atomicAdd(&W.R[x][0], ri.w);
                  atomicAdd(&W.R[x][1], ri.w * ri.a);
                  W.fA[x] = 1;
                }
                if ((unsigned)y < (unsigned)nbk) {
                  atomicAdd(&W.G[y][0], ri.u);
                  atomicAdd(&W.G[y][1], ri.b);
                  W.fB[y] = 1;
                }
              }
              wave_sync();
              const int mA = wave_compact(W.fA, W.lA, na, lane);
              const int mB = wave_compact(W.fB, W.lB, nbk, lane);
              wave_sync();
              const T wneg = -rj.w;
              wave_outer(W.lA, mA, W.lB, mB, lane, [&](int x, int y) {
                atomicAdd(&tile[x * nbk + y], (double)(wneg * (W.R[x][0] * W.G[y][0] + W.R[x][1] * W.G[y][1])));
              });
              if (lane == 0) n_fma += 2ull * (unsigned long long)(mA * mB);
              wave_sync();
              for (int u = lane; u < mA; u += 64) W.R[W.lA[u]][0] = W.R[W.lA[u]][1] = 0;
              for (int v = lane; v < mB; v += 64) W.G[W.lB[v]][0] = W.G[W.lB[v]][1] = 0;
              wave_sync();
            }
          }
          __syncthreads();

          // ---- add the tile block to the global numerator (and w_A)
          for (int e = tid; e < na * nbk; e += BLOCK) {
            const double v = tile[e];
            if (v != 0.0) {
              const int x = e / nbk, y = e - x * nbk;
              atomicAdd(&a.dnum[(obase + win_out(a0 + x)) * nb + win_out(b0 + y)], v);
            }
          }
          if (bb == 0)
            for (int x = tid; x < na; x += BLOCK)
              if (wdacc[x] != 0.0) atomicAdd(&a.wd[obase + win_out(a0 + x)], wdacc[x]);
          __syncthreads();
        }
      }
      r0 = r1;
    }
  }
  if (a.counters) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      n_in += __shfl_xor(n_in, o, 64);
      n_fma += __shfl_xor(n_fma, o, 64);
      n_lost += __shfl_xor(n_lost, o, 64);
    }
    if (lane == 0) {
      atomicAdd(&a.counters[0], n_in);
      atomicAdd(&a.counters[1], n_fma);
      atomicAdd(&a.counters[2], n_lost);
    }
  }
}

// Window key of each kept pair from its exact r_perp range.  Every pixel pair
// has r_perp in [(Dmin_f + Dmin_g) s, (Dmax_f + Dmax_g) s] (monotone rounding),
// and every bin decision (FP64, or FP32 away from edges) agrees with the FP64
// edge comparison, so the k_perp of every in-grid pixel pair is inside.
__global__ void dmat_keys_kernel(DmatArgs a, uint64_t* keys, int32_t* idx) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.n_pairs) return;
  const ForestInfo fi = a.finfo[a.sorted[a.pair_p[q]]];
  const ForestInfo gi = a.finfo[a.sorted[a.nbr[q]]];
  double s, c;
  pair_sc(fi, gi, s, c);
  const double rmin = __dmul_rn(__dadd_rn(fi.dmin, gi.dmin), s);
  const double rmax = __dmul_rn(__dadd_rn(fi.dmax, gi.dmax), s);
  const int NT = a.g.n_perp;
  const double* et = a.edges_perp;
  uint64_t key = ~0ull;
  if (rmin < et[NT] && rmax >= et[0]) {
    const int lo = rmin < et[0] ? 0 : bin_exact(rmin, et, NT, (int)((rmin - a.g.e0_perp) * a.g.inv_perp));
    const int hi = rmax >= et[NT] ? NT - 1 : bin_exact(rmax, et, NT, (int)((rmax - a.g.e0_perp) * a.g.inv_perp));
    if (lo >= 0 && hi >= lo)
      key = ((uint64_t)fi.real << 40) | ((uint64_t)lo << 16) | (uint64_t)(hi - lo + 1);
  }
  keys[q] = key;
  idx[q] = (int32_t)q;
}

constexpr int kNumVariants = 2;
const char* const kNames[kNumVariants] = {"fp32:b512/fp64:b256", "b256"};

template <typename T, int BLOCK>
hipError_t launch_one(const DmatArgs& a, int blocks, hipStream_t st) {
  if (a.g.zero_lo_par && a.g.zero_lo_perp)
    hipLaunchKernelGGL((dmat_kernel<T, BLOCK, true>), dim3(blocks), dim3(BLOCK), 0, st, a);
  else
    hipLaunchKernelGGL((dmat_kernel<T, BLOCK, false>), dim3(blocks), dim3(BLOCK), 0, st, a);
  return hipGetLastError();
}

template <typename T, int BLOCK>
int occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, dmat_kernel<T, BLOCK, true>, BLOCK, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

__global__ void finalize_dmat_kernel(double* d, const double* wd, int64_t n_rows, int nb) {
  const int64_t row = blockIdx.x;
  if (row >= n_rows) return;
  const double w = wd[row];
  double* r = d + row * nb;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) r[b] = w != 0.0 ? r[b] / w : 0.0;
}

}  // namespace

int dmat_num_variants() { return kNumVariants; }
const char* dmat_variant_name(int v) { return (v >= 0 && v < kNumVariants) ? kNames[v] : "?"; }

hipError_t launch_dmat_keys(const DmatArgs& a, uint64_t* keys, int32_t* idx, hipStream_t st) {
  if (a.n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(dmat_keys_kernel, dim3((unsigned)((a.n_pairs + 255) / 256)), dim3(256), 0, st, a, keys, idx);
  return hipGetLastError();
}

hipError_t launch_dmat(int variant, int precision, const DmatArgs& a, int blocks, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  if (precision == LYA_FP64) return launch_one<double, 256>(a, blocks, st);
  return variant == 0 ? launch_one<float, 512>(a, blocks, st) : launch_one<float, 256>(a, blocks, st);
}

int dmat_blocks_per_cu(int variant, int precision) {
  if (precision == LYA_FP64) return occupancy<double, 256>();
  return variant == 0 ? occupancy<float, 512>() : occupancy<float, 256>();
}

hipError_t launch_finalize_dmat(double* d, const double* wd, int64_t n_rows, int nb, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_dmat_kernel, dim3((unsigned)n_rows), dim3(256), 0, st, d, wd, n_rows, nb);
  return hipGetLastError();
}

}  // namespace lya
