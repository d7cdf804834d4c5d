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
// One workgroup handles one forest pair at a time (persistent, atomic work
// counter).  The bins the pair touches are compacted to local indices; the
// local x local block of D is accumulated in an LDS tile (in column/row
// blocks of TB if the pair touches more than TB bins) and added to the global
// FP64 numerator with atomics.  Bins are computed by the shared binner, so a
// pixel pair falls in the same bin here as in the xi kernel.
#include "lya_bin.h"
#include "lya_common.h"

namespace lya {

namespace {

template <typename T> struct DRecOf;
template <> struct DRecOf<float> { using type = DRec32; };
template <> struct DRecOf<double> { using type = DRec64; };

template <typename T, int BLOCK, int TB>
struct DmatSmem {
  static constexpr int NW = BLOCK / 64;
  uint16_t lidx[kMaxBins];   // local grid bin L -> compact index (0xFFFF: untouched)
  uint16_t lbins[kMaxBins];  // compact index -> L
  T tile[TB * TB];
  T H[4][TB];
  T Q[4][TB];
  T rowR[NW][2][TB];
  T rowG[NW][2][TB];
  uint8_t flA[NW][TB];
  uint8_t flB[NW][TB];
  uint8_t listA[NW][TB];
  uint8_t listB[NW][TB];
  int32_t scan[NW + 1];
  int64_t item;
  int32_t ntouch;
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T, int BLOCK, int TB, bool ZLO>
__global__ __launch_bounds__(BLOCK) void dmat_kernel(DmatArgs a) {
  static_assert(TB <= 255, "compact lists use 8-bit indices");
  using Rec = typename DRecOf<T>::type;
  constexpr int NW = BLOCK / 64;
  __shared__ DmatSmem<T, BLOCK, TB> sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  BinK<T, ZLO> K;
  K.init(a.g, a.glob, a.edges_par, a.edges_perp);
  const int NP = K.NP, NT = K.NT, nb = NP * NT;
  const double dc2 = 2.0 * a.glob->dc;
  const Rec* __restrict__ recs;
  if constexpr (sizeof(T) == 4) recs = a.drec32; else recs = a.drec64;

  for (int L = tid; L < nb; L += BLOCK) sm.lidx[L] = 0xFFFF;
  for (int x = tid; x < NW * TB; x += BLOCK) {
    (&sm.flA[0][0])[x] = 0;
    (&sm.flB[0][0])[x] = 0;
  }
  for (int x = tid; x < NW * 2 * TB; x += BLOCK) {
    (&sm.rowR[0][0][0])[x] = 0;
    (&sm.rowG[0][0][0])[x] = 0;
  }
  __syncthreads();
  unsigned long long n_in = 0, n_fma = 0;  // work counters (statistics only)

  for (;;) {
    if (tid == 0) sm.item = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t k = sm.item;
    if (k >= a.n_pairs) break;
    const ForestInfo fi = a.finfo[a.sorted[a.pair_p[k]]];
    const ForestInfo gi = a.finfo[a.sorted[a.nbr[k]]];
    double s64, c64;
    pair_sc(fi, gi, s64, c64);
    const T s = (T)s64, c = (T)c64;
    const T bsep = sizeof(T) == 4 ? (T)(dc2 * s64) : (T)0;
    const Rec* __restrict__ rf = recs + fi.pix0;
    const Rec* __restrict__ rg = recs + gi.pix0;
    const int nf = fi.npix, ng = gi.npix;

    auto pair_bin = [&](const Rec& ri, const Rec& rj) -> int {
      T rp, rt;
      separations(ri.d, rj.d, c, s, bsep, rp, rt);
      return K.bin(rp, rt, [&](double& rp64, double& rt64) {
        if constexpr (sizeof(T) == 4) {
          separations64(ri.D, rj.D, c64, s64, rp64, rt64);
        } else {
          rp64 = rp;
          rt64 = rt;
        }
      });
    };

    // ---- touched bins and their compact indices
    for (int i = wave; i < nf; i += NW) {
      const Rec ri = rf[i];
      for (int j = lane; j < ng; j += 64) {
        const int L = pair_bin(ri, rg[j]);
        if (L >= 0) {
          sm.lidx[L] = 0;
          ++n_in;
        }
      }
    }
    __syncthreads();
    {
      const int C = (nb + BLOCK - 1) / BLOCK;
      const int L0 = tid * C, L1 = min(nb, L0 + C);
      int cnt = 0;
      for (int L = L0; L < L1; ++L) cnt += sm.lidx[L] == 0;
      int incl = cnt;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
      }
      if (lane == 63) sm.scan[wave + 1] = incl;
      __syncthreads();
      if (tid == 0) {
        sm.scan[0] = 0;
        for (int w = 1; w <= NW; ++w) sm.scan[w] += sm.scan[w - 1];
        sm.ntouch = sm.scan[NW];
      }
      __syncthreads();
      int pos = sm.scan[wave] + incl - cnt;
      for (int L = L0; L < L1; ++L)
        if (sm.lidx[L] == 0) {
          sm.lidx[L] = (uint16_t)pos;
          sm.lbins[pos] = (uint16_t)L;
          ++pos;
        }
    }
    __syncthreads();
    const int Tn = sm.ntouch;
    const int nblk = (Tn + TB - 1) / TB;
    const int64_t obase = (int64_t)fi.real * nb;

    for (int ab = 0; ab < nblk; ++ab) {
      const int a0 = ab * TB, na = min(TB, Tn - a0);
      for (int bb = 0; bb < nblk; ++bb) {
        const int b0 = bb * TB, nbk = min(TB, Tn - b0);
        for (int x = tid; x < na * nbk; x += BLOCK) sm.tile[x] = 0;
        for (int x = tid; x < 4 * TB; x += BLOCK) {
          (&sm.H[0][0])[x] = 0;
          (&sm.Q[0][0])[x] = 0;
        }
        __syncthreads();

        // ---- pair histograms H (rows of this block) and Q (columns)
        for (int i = wave; i < nf; i += NW) {
          const Rec ri = rf[i];
          for (int j = lane; j < ng; j += 64) {
            const Rec rj = rg[j];
            const int L = pair_bin(ri, rj);
            if (L < 0) continue;
            const int la = sm.lidx[L];
            const int x = la - a0, y = la - b0;
            if ((unsigned)x < (unsigned)na) {
              const T ww = ri.w * rj.w;
              atomicAdd(&sm.H[0][x], ww);
              atomicAdd(&sm.H[1][x], ww * rj.a);
              atomicAdd(&sm.H[2][x], ri.a * ww);
              atomicAdd(&sm.H[3][x], ri.a * ww * rj.a);
            }
            if ((unsigned)y < (unsigned)nbk) {
              atomicAdd(&sm.Q[0][y], ri.u * rj.u);
              atomicAdd(&sm.Q[1][y], ri.u * rj.b);
              atomicAdd(&sm.Q[2][y], ri.b * rj.u);
              atomicAdd(&sm.Q[3][y], ri.b * rj.b);
            }
          }
        }

        // ---- row outer products: rows of f (side 0) then rows of g (side 1)
        T* R0 = sm.rowR[wave][0];
        T* R1 = sm.rowR[wave][1];
        T* G0 = sm.rowG[wave][0];
        T* G1 = sm.rowG[wave][1];
        uint8_t* fA = sm.flA[wave];
        uint8_t* fB = sm.flB[wave];
        uint8_t* lA = sm.listA[wave];
        uint8_t* lB = sm.listB[wave];
        const uint64_t lt_mask = (1ull << lane) - 1ull;
        for (int side = 0; side < 2; ++side) {
          const Rec* __restrict__ rrow = side ? rg : rf;
          const Rec* __restrict__ rcol = side ? rf : rg;
          const int nrow = side ? ng : nf, ncol = side ? nf : ng;
          for (int i = wave; i < nrow; i += NW) {
            const Rec ri = rrow[i];
            for (int j = lane; j < ncol; j += 64) {
              const Rec rj = rcol[j];
              const int L = pair_bin(ri, rj);
              if (L < 0) continue;
              const int la = sm.lidx[L];
              const int x = la - a0, y = la - b0;
              if ((unsigned)x < (unsigned)na) {
                atomicAdd(&R0[x], rj.w);
                atomicAdd(&R1[x], rj.w * rj.a);
                fA[x] = 1;
              }
              if ((unsigned)y < (unsigned)nbk) {
                atomicAdd(&G0[y], rj.u);
                atomicAdd(&G1[y], rj.b);
                fB[y] = 1;
              }
            }
            wave_sync();
            int mA = 0, mB = 0;
            for (int x0 = 0; x0 < na; x0 += 64) {
              const int x = x0 + lane;
              const bool on = x < na && fA[x];
              const uint64_t m = __ballot(on);
              if (on) {
                lA[mA + __popcll(m & lt_mask)] = (uint8_t)x;
                fA[x] = 0;
              }
              mA += __popcll(m);
            }
            for (int y0 = 0; y0 < nbk; y0 += 64) {
              const int y = y0 + lane;
              const bool on = y < nbk && fB[y];
              const uint64_t m = __ballot(on);
              if (on) {
                lB[mB + __popcll(m & lt_mask)] = (uint8_t)y;
                fB[y] = 0;
              }
              mB += __popcll(m);
            }
            wave_sync();
            const int tot = mA * mB;
            if (lane == 0) n_fma += 2ull * (unsigned long long)tot;
            const T wneg = -ri.w;
            const float inv = mB ? 1.0f / (float)mB : 0.f;
            for (int idx = lane; idx < tot; idx += 64) {
              int u = (int)((float)idx * inv);
              if (u * mB > idx) --u;
              else if ((u + 1) * mB <= idx) ++u;
              const int x = lA[u], y = lB[idx - u * mB];
              atomicAdd(&sm.tile[x * nbk + y], wneg * (R0[x] * G0[y] + R1[x] * G1[y]));
            }
            wave_sync();
            for (int u = lane; u < mA; u += 64) {
              const int x = lA[u];
              R0[x] = 0;
              R1[x] = 0;
            }
            for (int v = lane; v < mB; v += 64) {
              const int y = lB[v];
              G0[y] = 0;
              G1[y] = 0;
            }
            wave_sync();
          }
        }
        __syncthreads();

        // ---- H (x) Q and the Kronecker term, then flush to the global numerator
        if (tid == 0) n_fma += 4ull * (unsigned long long)(na * nbk);
        for (int idx = tid; idx < na * nbk; idx += BLOCK) {
          const int x = idx / nbk, y = idx - x * nbk;
          T v = sm.H[0][x] * sm.Q[0][y] + sm.H[1][x] * sm.Q[1][y] + sm.H[2][x] * sm.Q[2][y] +
                sm.H[3][x] * sm.Q[3][y];
          if (a0 + x == b0 + y) v += sm.H[0][x];
          v += sm.tile[idx];
          if (v != (T)0) {
            const int A = out_index(sm.lbins[a0 + x], NP, NT);
            const int B = out_index(sm.lbins[b0 + y], NP, NT);
            atomicAdd(&a.dnum[(obase + A) * nb + B], (double)v);
          }
        }
        if (bb == 0)
          for (int x = tid; x < na; x += BLOCK)
            atomicAdd(&a.wd[obase + out_index(sm.lbins[a0 + x], NP, NT)], (double)sm.H[0][x]);
        __syncthreads();
      }
    }
    for (int x = tid; x < Tn; x += BLOCK) sm.lidx[sm.lbins[x]] = 0xFFFF;
    __syncthreads();
  }
  if (a.counters) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      n_in += __shfl_xor(n_in, o, 64);
      n_fma += __shfl_xor(n_fma, o, 64);
    }
    if (lane == 0) {
      atomicAdd(&a.counters[0], n_in);
      atomicAdd(&a.counters[1], n_fma);
    }
  }
}

struct Variant {
  const char* name;
};
constexpr Variant kVariants[] = {{"b512-t128/88"}, {"b256-t64/48"}};
constexpr int kNumVariants = 2;

template <typename T> constexpr int tb_big() { return sizeof(T) == 4 ? 128 : 88; }
template <typename T> constexpr int tb_small() { return sizeof(T) == 4 ? 64 : 48; }

template <typename T, int BLOCK, int TB>
hipError_t launch_one(const DmatArgs& a, int blocks, hipStream_t st) {
  if (a.g.zero_lo_par && a.g.zero_lo_perp)
    hipLaunchKernelGGL((dmat_kernel<T, BLOCK, TB, true>), dim3(blocks), dim3(BLOCK), 0, st, a);
  else
    hipLaunchKernelGGL((dmat_kernel<T, BLOCK, TB, false>), dim3(blocks), dim3(BLOCK), 0, st, a);
  return hipGetLastError();
}

template <typename T, int BLOCK, int TB>
int occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, dmat_kernel<T, BLOCK, TB, true>, BLOCK, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

template <typename T>
hipError_t launch_t(int v, const DmatArgs& a, int blocks, hipStream_t st) {
  if (v == 0) return launch_one<T, 512, tb_big<T>()>(a, blocks, st);
  return launch_one<T, 256, tb_small<T>()>(a, blocks, st);
}

template <typename T>
int occ_t(int v) {
  if (v == 0) return occupancy<T, 512, tb_big<T>()>();
  return occupancy<T, 256, tb_small<T>()>();
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
const char* dmat_variant_name(int v) { return (v >= 0 && v < kNumVariants) ? kVariants[v].name : "?"; }

hipError_t launch_dmat(int variant, int precision, const DmatArgs& a, int blocks, hipStream_t st) {
  if (a.n_pairs == 0) return hipSuccess;
  return precision == LYA_FP64 ? launch_t<double>(variant, a, blocks, st)
                               : launch_t<float>(variant, a, blocks, st);
}

int dmat_blocks_per_cu(int variant, int precision) {
  return precision == LYA_FP64 ? occ_t<double>(variant) : occ_t<float>(variant);
}

hipError_t launch_finalize_dmat(double* d, const double* wd, int64_t n_rows, int nb, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_dmat_kernel, dim3((unsigned)n_rows), dim3(256), 0, st, d, wd, n_rows, nb);
  return hipGetLastError();
}

}  // namespace lya
