// Microbenchmarks of the rates the pair kernels are bound by: LDS atomic adds
// (FP32, FP64, u32; conflict-free and with four lanes per address), plain LDS
// stores, non-packed FP32 / FP64 VALU fused multiply-adds, and plain FP32 and
// u32 VALU additions.  Each kernel
// issues long runs of independent operations from many waves per SIMD; the
// host divides the lane-operations by the event-timed kernel duration.
#include "lya_common.h"

namespace lya {

namespace {

constexpr int kPeakBlock = 256;   // 4 waves
constexpr int kUnroll = 8;        // independent operations per loop trip
constexpr int kRegion = 512;      // LDS elements per wave

enum : int { kLdsAddF32 = 0, kLdsAddF64 = 1, kLdsAddU32 = 2, kLdsAddF32Shared4 = 3, kLdsWrite32 = 4 };

template <int KIND>
__global__ __launch_bounds__(kPeakBlock) void lds_rate_kernel(unsigned long long* sink, int iters) {
  __shared__ double sd[kRegion * (kPeakBlock / 64)];
  float* sf = (float*)sd;
  unsigned* su = (unsigned*)sd;
  for (int i = threadIdx.x; i < kRegion * (kPeakBlock / 64); i += kPeakBlock) sd[i] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int base = wave * kRegion;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      // conflict-free: 64 consecutive elements per instruction, rotating through the region
      const int a = base + (((u + it) * 64 + lane) & (kRegion - 1));
      if constexpr (KIND == kLdsAddF32) atomicAdd(&sf[a], 1.0f);
      if constexpr (KIND == kLdsAddF64) atomicAdd(&sd[a], 1.0);
      if constexpr (KIND == kLdsAddU32) atomicAdd(&su[a], 1u);
      if constexpr (KIND == kLdsAddF32Shared4) atomicAdd(&sf[base + (((u + it) * 16 + (lane >> 2)) & (kRegion - 1))], 1.0f);
      if constexpr (KIND == kLdsWrite32) sf[a] = (float)(it + u);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(sink, (unsigned long long)(su[1] & 1u));
}

template <typename T>
__global__ __launch_bounds__(kPeakBlock) void valu_rate_kernel(T* out, int iters, T x) {
  // eight independent FMA chains per lane
  T a0 = x + (T)threadIdx.x, a1 = a0 + (T)1, a2 = a0 + (T)2, a3 = a0 + (T)3;
  T a4 = a0 + (T)4, a5 = a0 + (T)5, a6 = a0 + (T)6, a7 = a0 + (T)7;
  const T m = (T)0.9999, c = (T)0.5;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a0 = fma(a0, m, c); a1 = fma(a1, m, c); a2 = fma(a2, m, c); a3 = fma(a3, m, c);
      a4 = fma(a4, m, c); a5 = fma(a5, m, c); a6 = fma(a6, m, c); a7 = fma(a7, m, c);
    }
  }
  const T s = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
  if (s == (T)-12345) out[threadIdx.x] = s;  // never true: keeps the chains alive
}

// The same eight chains of one plain instruction, written in assembly so that
// the compiler can neither fold a chain of additions nor pick another opcode:
// OP 0 = v_add_f32, OP 1 = v_add_u32.
template <int OP>
__global__ __launch_bounds__(kPeakBlock) void valu_add_rate_kernel(float* out, int iters, float x) {
  float f[8];
  unsigned u[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    f[k] = x + (float)(threadIdx.x + k);
    u[k] = threadIdx.x + k;
  }
  const float cf = 1.0e-7f;
  const unsigned cu = 3u;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if constexpr (OP == 0) asm volatile("v_add_f32 %0, %0, %1" : "+v"(f[k]) : "v"(cf));
        else asm volatile("v_add_u32 %0, %0, %1" : "+v"(u[k]) : "v"(cu));
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += f[k] + (float)u[k];
  if (s == -12345.f) out[threadIdx.x] = s;  // never true
}

}  // namespace

hipError_t launch_lds_rate(int kind, int blocks, int iters, unsigned long long* sink, hipStream_t st) {
  switch (kind) {
    case kLdsAddF32: hipLaunchKernelGGL(lds_rate_kernel<kLdsAddF32>, dim3(blocks), dim3(kPeakBlock), 0, st, sink, iters); break;
    case kLdsAddF64: hipLaunchKernelGGL(lds_rate_kernel<kLdsAddF64>, dim3(blocks), dim3(kPeakBlock), 0, st, sink, iters); break;
    case kLdsAddU32: hipLaunchKernelGGL(lds_rate_kernel<kLdsAddU32>, dim3(blocks), dim3(kPeakBlock), 0, st, sink, iters); break;
    case kLdsAddF32Shared4:
      hipLaunchKernelGGL(lds_rate_kernel<kLdsAddF32Shared4>, dim3(blocks), dim3(kPeakBlock), 0, st, sink, iters);
      break;
    case kLdsWrite32: hipLaunchKernelGGL(lds_rate_kernel<kLdsWrite32>, dim3(blocks), dim3(kPeakBlock), 0, st, sink, iters); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_valu_rate(int kind, int blocks, int iters, void* out, hipStream_t st) {
  switch (kind) {
    case 0: hipLaunchKernelGGL(valu_rate_kernel<float>, dim3(blocks), dim3(kPeakBlock), 0, st, (float*)out, iters, 1.0f); break;
    case 1: hipLaunchKernelGGL(valu_rate_kernel<double>, dim3(blocks), dim3(kPeakBlock), 0, st, (double*)out, iters, 1.0); break;
    case 2: hipLaunchKernelGGL(valu_add_rate_kernel<0>, dim3(blocks), dim3(kPeakBlock), 0, st, (float*)out, iters, 1.0f); break;
    case 3: hipLaunchKernelGGL(valu_add_rate_kernel<1>, dim3(blocks), dim3(kPeakBlock), 0, st, (float*)out, iters, 1.0f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int peak_block() { return kPeakBlock; }
int peak_unroll_lds() { return kUnroll; }
int peak_unroll_valu() { return 32; }

}  // namespace lya
