// Covariance of the correlation function from subsample sums (the paper
// estimates the covariance by subsampling the forests in sky pixels, Sec. 2.1
// and the discussion of its 3PCF errors).  With N_sA, W_sA the sums of
// subsample s and N_A, W_A, xi_A = N_A / W_A their totals:
//   C_AB = sum_s W_sA W_sB (xi_sA - xi_A)(xi_sB - xi_B) / (W_A W_B)
//        = sum_s x_sA x_sB / (W_A W_B),   x_sA = N_sA - W_sA xi_A,
// 0 where W_A W_B = 0 (x_sA is defined even where W_sA = 0).
#include "lya_common.h"

namespace lya {

namespace {

// totals and x_sA, one thread per bin
__global__ void cov_prep_kernel(const double* num, const double* wsum, int64_t n_sub, int64_t nb, double* x,
                                double* tot_w, double* xi) {
  const int64_t A = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= nb) return;
  double n = 0.0, w = 0.0;
  for (int64_t s = 0; s < n_sub; ++s) {
    n += num[s * nb + A];
    w += wsum[s * nb + A];
  }
  const double xa = w != 0.0 ? n / w : 0.0;
  tot_w[A] = w;
  xi[A] = xa;
  for (int64_t s = 0; s < n_sub; ++s) x[s * nb + A] = num[s * nb + A] - wsum[s * nb + A] * xa;
}

// C = X^T X / (W W^T): 64 x 64 output tiles, 16 x 16 threads with 4 x 4 each,
// the subsample dimension staged through LDS 16 at a time
constexpr int kT = 64, kS = 16;
__global__ __launch_bounds__(256) void cov_kernel(const double* x, const double* tot_w, int64_t n_sub, int64_t nb,
                                                  double* cov) {
  __shared__ double xa[kS][kT], xb[kS][kT];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t a0 = (int64_t)blockIdx.y * kT, b0 = (int64_t)blockIdx.x * kT;
  double acc[4][4] = {};
  for (int64_t s0 = 0; s0 < n_sub; s0 += kS) {
    for (int e = threadIdx.x; e < kS * kT; e += 256) {
      const int s = e / kT, c = e % kT;
      const bool in_s = s0 + s < n_sub;
      xa[s][c] = (in_s && a0 + c < nb) ? x[(s0 + s) * nb + a0 + c] : 0.0;
      xb[s][c] = (in_s && b0 + c < nb) ? x[(s0 + s) * nb + b0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int s = 0; s < kS; ++s) {
      double va[4], vb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        va[i] = xa[s][ty + 16 * i];
        vb[i] = xb[s][tx + 16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(va[i], vb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t A = a0 + ty + 16 * i;
    if (A >= nb) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t B = b0 + tx + 16 * j;
      if (B >= nb) continue;
      const double d = tot_w[A] * tot_w[B];
      cov[A * nb + B] = d != 0.0 ? acc[i][j] / d : 0.0;
    }
  }
}

}  // namespace

hipError_t launch_covariance(const double* num, const double* wsum, int64_t n_sub, int64_t nb, double* x,
                             double* tot_w, double* xi, double* cov, hipStream_t st) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(cov_prep_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, num, wsum, n_sub, nb,
                     x, tot_w, xi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned nt = (unsigned)((nb + kT - 1) / kT);
  hipLaunchKernelGGL(cov_kernel, dim3(nt, nt), dim3(256), 0, st, x, tot_w, n_sub, nb, cov);
  return hipGetLastError();
}

}  // namespace lya
