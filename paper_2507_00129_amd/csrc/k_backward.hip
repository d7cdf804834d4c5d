// Backward pass of the xi estimator (Sec. 2.1, eq. estimator_two):
// with gamma_A = (dL/dxi_A) / W_A,
//   dL/d delta_i = w_i sum_j gamma_{A(i,j)} w_j delta_j
//   dL/d w_i     = sum_j gamma_{A(i,j)} w_j (delta_i delta_j - xi_{A(i,j)})
//                = delta_i S1_i - S2_i,  S1_i = sum_j gamma w_j delta_j,
//                                        S2_i = sum_j gamma xi w_j
// over every pixel j of every other forest of the same realisation.
//
// Work item = one forest f with all of its neighbours (a symmetric neighbour
// list), so every contribution to f's pixels is summed inside one workgroup
// and written with plain stores.  Lanes own pixels i of f; the neighbour's
// pixels j are wave-uniform (scalar loads, several records at a time); the
// bin of each pair comes from the shared binner, and over a run of
// consecutive pixels j in one bin the lane sums w_j delta_j and w_j before it
// gathers gamma, gamma*xi from an LDS table once for the run.  Waves
// split the neighbours; each lane sums a neighbour's contributions in the
// working precision, adds them to FP64 registers, and the waves combine their
// FP64 sums through LDS.
#include "lya_bin.h"
#include "lya_common.h"

namespace lya {

namespace {

constexpr int kGroup = 2048;  // pixels of f handled per pass (LDS accumulators)

template <typename R>
__device__ __forceinline__ R load_u(const R* p);
typedef float bw_f4 __attribute__((ext_vector_type(4)));
typedef double bw_d4 __attribute__((ext_vector_type(4)));
template <>
__device__ __forceinline__ Rec32 load_u(const Rec32* p) {
  const bw_f4 v = *(const __attribute__((address_space(4))) bw_f4*)p;
  return Rec32{v.x, v.y, v.z, v.w};
}
template <>
__device__ __forceinline__ Rec64 load_u(const Rec64* p) {
  const bw_d4 v = *(const __attribute__((address_space(4))) bw_d4*)p;
  return Rec64{v.x, v.y, v.z, v.w};
}
// Four (FP32) or two (FP64) consecutive records with one scalar load.
template <typename R> struct BwBatch;
typedef float bw_f16 __attribute__((ext_vector_type(16)));
typedef double bw_d8 __attribute__((ext_vector_type(8)));
template <> struct BwBatch<Rec32> {
  static constexpr int N = 4;
  Rec32 r[4];
  __device__ __forceinline__ void load(const Rec32* p) {
    const bw_f16 v = *(const __attribute__((address_space(4))) bw_f16*)p;
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = Rec32{v[4 * u], v[4 * u + 1], v[4 * u + 2], v[4 * u + 3]};
  }
};
template <> struct BwBatch<Rec64> {
  static constexpr int N = 2;
  Rec64 r[2];
  __device__ __forceinline__ void load(const Rec64* p) {
    const bw_d8 v = *(const __attribute__((address_space(4))) bw_d8*)p;
#pragma unroll
    for (int u = 0; u < 2; ++u) r[u] = Rec64{v[4 * u], v[4 * u + 1], v[4 * u + 2], v[4 * u + 3]};
  }
};

__device__ __forceinline__ double load_ud(const double* p) {
  return *(const __attribute__((address_space(4))) double*)p;
}

template <typename T> struct RecOfB;
template <> struct RecOfB<float> { using type = Rec32; };
template <> struct RecOfB<double> { using type = Rec64; };

template <typename T, int BLOCK, bool ZLO>
__global__ __launch_bounds__(BLOCK) void xi_bwd_kernel(BwdArgs a) {
  using Rec = typename RecOfB<T>::type;
  constexpr int NW = BLOCK / 64;
  extern __shared__ double smem[];
  const int NP = a.g.n_par, NT = a.g.n_perp, nb = NP * NT;
  double* acc1 = smem;                 // [kGroup]
  double* acc2 = smem + kGroup;        // [kGroup]
  T* tab = (T*)(smem + 2 * kGroup);    // [nb][2]: gamma, gamma * xi  (local layout)
  __shared__ int64_t s_item;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  BinK<T, ZLO> K;
  K.init(a.g, a.glob, a.edges_par, a.edges_perp);
  const double dc2 = 2.0 * a.glob->dc;
  const Rec* __restrict__ recs;
  if constexpr (sizeof(T) == 4) recs = a.rec32; else recs = a.rec64;

  int cur_real = -1;
  for (;;) {
    if (tid == 0) s_item = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t it = s_item;
    if (it >= a.n_items) break;
    const Item item = a.items[it];
    const ForestInfo fi = a.finfo[a.sorted[item.p]];
    if (fi.real != cur_real) {
      const double2* src = a.gtab + (int64_t)fi.real * nb;
      for (int L = tid; L < nb; L += BLOCK) {
        const double2 v = src[L];
        tab[2 * L] = (T)v.x;
        tab[2 * L + 1] = (T)v.y;
      }
      cur_real = fi.real;
    }
    const Rec* __restrict__ rf = recs + fi.pix0;
    const int nf = fi.npix;

    for (int g0 = 0; g0 < nf; g0 += kGroup) {
      const int ng0 = min(kGroup, nf - g0);
      for (int x = tid; x < ng0; x += BLOCK) {
        acc1[x] = 0.0;
        acc2[x] = 0.0;
      }
      __syncthreads();
      for (int ib = 0; ib < ng0; ib += 64) {
        const int i = g0 + ib + lane;
        const bool valid = ib + lane < ng0;
        Rec ri;
        double Di64 = 0.0;
        if (valid) {
          ri = rf[i];
          if constexpr (sizeof(T) == 4) Di64 = a.dist[fi.pix0 + i];
        } else {
          ri.d = (T)1e30;  // far away: never in the grid
          ri.wd = 0;
          ri.w = 0;
          ri.del = 0;
        }
        double s1 = 0.0, s2 = 0.0;
        for (int k = wave; k < item.nb_count; k += NW) {
          const ForestInfo gi = a.finfo[a.sorted[a.nbr[item.nb_begin + k]]];
          double s64, c64;
          pair_sc(fi, gi, s64, c64);
          const T s = (T)s64, c = (T)c64;
          const T bsep = sizeof(T) == 4 ? (T)(dc2 * s64) : (T)0;
          const Rec* __restrict__ rg = recs + gi.pix0;
          // runs of consecutive pixels j in one bin: their w delta and w are
          // summed first and gamma, gamma xi gathered once per run
          T p1 = 0, p2 = 0, awd = 0, aw = 0;
          int cur = -1;
          auto pair = [&](const Rec& rj, int j) __attribute__((always_inline)) {
            T rp, rt;
            separations(ri.d, rj.d, c, s, bsep, rp, rt);
            const int L = K.bin(rp, rt, [&](double& rp64, double& rt64) {
              if constexpr (sizeof(T) == 4) {
                separations64(Di64, load_ud(a.dist + gi.pix0 + j), c64, s64, rp64, rt64);
              } else {
                rp64 = rp;
                rt64 = rt;
              }
            });
            if (L != cur) {
              if (cur >= 0) {
                p1 += tab[2 * cur] * awd;
                p2 += tab[2 * cur + 1] * aw;
              }
              cur = L;
              awd = 0;
              aw = 0;
            }
            awd += rj.wd;
            aw += rj.w;
          };
          constexpr int NBAT = BwBatch<Rec>::N;
          int j = 0;
          for (; j + NBAT <= gi.npix; j += NBAT) {
            BwBatch<Rec> b;
            b.load(rg + j);
#pragma unroll
            for (int u = 0; u < NBAT; ++u) pair(b.r[u], j + u);
          }
          for (; j < gi.npix; ++j) pair(load_u(rg + j), j);
          if (cur >= 0) {
            p1 += tab[2 * cur] * awd;
            p2 += tab[2 * cur + 1] * aw;
          }
          s1 += (double)p1;
          s2 += (double)p2;
        }
        if (valid) {
          atomicAdd(&acc1[ib + lane], s1);
          atomicAdd(&acc2[ib + lane], s2);
        }
      }
      __syncthreads();
      for (int x = tid; x < ng0; x += BLOCK) {
        const int64_t i = fi.pix0 + g0 + x;
        const double w = a.weight[i], de = a.delta[i];
        a.grad_delta[i] = w * acc1[x];
        a.grad_weight[i] = de * acc1[x] - acc2[x];
      }
      __syncthreads();
    }
  }
}

// gamma_A = dL/dxi_A / W_A (0 where W_A = 0) and gamma_A xi_A, in the local
// (LDS) bin order L = kt * NP + kp.
__global__ void gamma_kernel(const double* grad_xi, const double* xi, const double* wsum,
                             double2* out, int64_t n, int NP, int NT) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int nb = NP * NT;
  const int64_t r = idx / nb;
  const int L = (int)(idx - r * nb);
  const int kt = L / NP, kp = L - kt * NP;
  const int64_t A = r * nb + (int64_t)kp * NT + kt;
  const double w = wsum[A];
  const double g = w != 0.0 ? grad_xi[A] / w : 0.0;
  out[idx] = make_double2(g, g * xi[A]);
}

// Adjoint of the per-forest projection delta' = eta delta (Sec. 2.2) applied
// to the gradient.  eta moves with w through W, the weighted mean of Lambda
// and S; differentiating delta'_i = delta_i - m - a_i t (m = sum w delta / W,
// t = sum w a delta / S, a = Lambda - Lambda_bar) and collapsing the sums
// gives, with g'_k = dL/d delta'_k and h'_k = dL/dw_k at fixed delta':
//   c_k = G0 / W + a_k G1 / S,  G0 = sum_i g'_i,  G1 = sum_i a_i g'_i,
//   dL/d delta_k = g'_k - w_k c_k,   dL/dw_k = h'_k - delta'_k c_k.
// The slope part is used only where the forward used the slope term, and
// c = 0 where eta = I (identity mode, or a forest with W = 0).  One wave per
// forest, FP64, in place.
__global__ __launch_bounds__(256) void project_adjoint_kernel(lya_forests F, const EtaInfo* einfo,
                                                              const double* delta_proj,
                                                              double* grad_delta, double* grad_weight) {
  const int lane = threadIdx.x & 63;
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (f >= F.n_forests) return;
  const EtaInfo e = einfo[f];
  if (!e.active) return;
  const int64_t p0 = F.offsets[f], p1 = F.offsets[f + 1];
  double g0 = 0.0, g1 = 0.0;
  for (int64_t k = p0 + lane; k < p1; k += 64) {
    const double g = grad_delta[k];
    g0 += g;
    g1 += (F.loglam[k] - e.lbar) * g;
  }
  g0 = wave_sum(g0);
  g1 = wave_sum(g1);
  const double c0 = g0 / e.W, c1 = e.slope ? g1 / e.S : 0.0;
  for (int64_t k = p0 + lane; k < p1; k += 64) {
    const double c = c0 + (F.loglam[k] - e.lbar) * c1;
    grad_delta[k] -= F.weight[k] * c;
    grad_weight[k] -= delta_proj[k] * c;
  }
}

template <typename T, int BLOCK>
hipError_t launch_one(const BwdArgs& a, int blocks, hipStream_t st) {
  const size_t smem = 2 * kGroup * sizeof(double) + (size_t)a.g.n_par * a.g.n_perp * 2 * sizeof(T);
  auto kern = (a.g.zero_lo_par && a.g.zero_lo_perp) ? xi_bwd_kernel<T, BLOCK, true> : xi_bwd_kernel<T, BLOCK, false>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(BLOCK), smem, st, a);
  return hipGetLastError();
}

template <typename T, int BLOCK>
int occupancy(int n_bins) {
  const size_t smem = 2 * kGroup * sizeof(double) + (size_t)n_bins * 2 * sizeof(T);
  auto kern = xi_bwd_kernel<T, BLOCK, true>;
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess) return 1;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, BLOCK, smem) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

}  // namespace

hipError_t launch_gamma(const double* grad_xi, const double* xi, const double* wsum, double2* out,
                        int64_t n, int NP, int NT, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gamma_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, grad_xi, xi, wsum,
                     out, n, NP, NT);
  return hipGetLastError();
}

hipError_t launch_project_adjoint(const lya_forests* F, const EtaInfo* einfo, const double* delta_proj,
                                  double* grad_delta, double* grad_weight, hipStream_t st) {
  if (F->n_forests == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((F->n_forests + 3) / 4);
  hipLaunchKernelGGL(project_adjoint_kernel, dim3(blocks), dim3(256), 0, st, *F, einfo, delta_proj,
                     grad_delta, grad_weight);
  return hipGetLastError();
}

hipError_t launch_xi_bwd(int precision, const BwdArgs& a, int blocks, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  return precision == LYA_FP64 ? launch_one<double, 512>(a, blocks, st) : launch_one<float, 512>(a, blocks, st);
}

int xi_bwd_blocks_per_cu(int precision, int n_bins) {
  return precision == LYA_FP64 ? occupancy<double, 512>(n_bins) : occupancy<float, 512>(n_bins);
}

}  // namespace lya
