// Forest-pair work list (the neighbourhood pre-ordering of Sec. 2.1).
//
// Forests are sorted by (realisation, declination strip, right ascension).
// The strip height is at least the largest angle theta_max at which any pixel
// pair can still have r_perp inside the grid, so every neighbour of a forest
// lies in its own strip or the two adjacent ones.  Within a strip (a cell of
// the sorted order) a neighbour's right ascension differs by at most
// asin(sin theta_max / cos dec_max), dec_max the largest |dec| of the two
// strips, so the candidates of the forest at sorted position p are at most two
// RA intervals (one more where the interval wraps past 2 pi) per cell, found by
// bisection of the sorted keys; each candidate is kept by the exact
// conservative cut pair_may_bin.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "lya_common.h"

namespace lya {

namespace {

constexpr double kPi = 3.141592653589793;

__global__ void keys_kernel(WorklistArgs a) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= a.n_forests) return;
  const double dec = a.dec[f];
  int strip = (int)floor((dec + 0.5 * kPi) / a.strip_h);
  strip = strip < 0 ? 0 : (strip >= a.n_strips ? a.n_strips - 1 : strip);
  double t = a.ra[f] / (2.0 * kPi);
  t -= floor(t);
  uint32_t raq = (uint32_t)fmin(t * 4294967296.0, 4294967295.0);
  const uint64_t real = (uint64_t)a.finfo[f].real;
  a.keys[f] = (real << 44) | ((uint64_t)strip << 32) | raq;
  a.ids[f] = (int32_t)f;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__device__ __forceinline__ int cell_of(uint64_t key, int n_strips) {
  return (int)(key >> 44) * n_strips + (int)((key >> 32) & 0xFFF);
}

__global__ void cells_kernel(WorklistArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_forests) return;
  const int c = cell_of(a.keys_sorted[p], a.n_strips);
  if (p == 0 || cell_of(a.keys_sorted[p - 1], a.n_strips) != c) a.cell_begin[c] = (int32_t)p;
  if (p == a.n_forests - 1 || cell_of(a.keys_sorted[p + 1], a.n_strips) != c) a.cell_end[c] = (int32_t)(p + 1);
}

// First sorted position in [lo, hi) whose key is >= k (hi if none).
__device__ __forceinline__ int64_t lower_key(const uint64_t* keys, int64_t lo, int64_t hi, uint64_t k) {
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (keys[m] < k) lo = m + 1; else hi = m;
  }
  return lo;
}

// Half-width in RA (turns, quantised as the keys) of the window that holds
// every forest within theta of any forest in strips s and t, or -1 when the
// strips come closer than theta to a pole (then the whole cell is scanned).
__device__ __forceinline__ int64_t ra_halfwidth(const WorklistArgs& a, int s, int t) {
  if (a.theta >= 0.5 * kPi) return -1;
  const int lo = s < t ? s : t, hi = s < t ? t : s;
  const double d0 = -0.5 * kPi + lo * a.strip_h, d1 = -0.5 * kPi + (hi + 1) * a.strip_h;
  const double dmax = fmax(fabs(d0), fabs(d1));
  const double cs = cos(dmax), sn = sin(a.theta);
  if (!(cs > sn * (1.0 + 1e-6))) return -1;
  const double dra = asin(sn / cs) * (1.0 + 1e-6) + 1e-9;  // radians, widened past rounding
  if (dra >= kPi) return -1;
  return (int64_t)ceil(dra / (2.0 * kPi) * 4294967296.0) + 2;
}

// The candidate intervals of sorted position p in cell c (strip t): positions
// whose RA lies within the window around p's, restricted to positions > p
// unless the lists are symmetric.  Appends up to 2 intervals to iv.
__device__ __forceinline__ void cell_intervals(const WorklistArgs& a, int64_t p, uint64_t key, int s, int t,
                                               int c, int64_t (*iv)[2], int& n) {
  int64_t b = a.cell_begin[c], e = a.cell_end[c];
  if (b < 0) return;  // empty cell
  if (!a.symmetric && b <= p) b = p + 1;
  if (b >= e) return;
  const int64_t hw = ra_halfwidth(a, s, t);
  const uint64_t cellkey = (key & ~(((uint64_t)1 << 44) - 1)) | ((uint64_t)t << 32);  // realisation, strip t
  if (hw < 0) {
    iv[n][0] = b;
    iv[n][1] = e;
    ++n;
    return;
  }
  const int64_t full = (int64_t)1 << 32;
  if (2 * hw + 1 >= full) {
    iv[n][0] = b;
    iv[n][1] = e;
    ++n;
    return;
  }
  const int64_t ra = (int64_t)(key & 0xFFFFFFFFull), lo = ra - hw, hi = ra + hw;  // inclusive RA bounds
  // RA intervals in [0, 2^32): the window, split where it wraps
  int64_t r[2][2];
  int nr = 0;
  if (lo < 0 && hi >= full) {
    r[nr][0] = 0; r[nr][1] = full - 1; ++nr;
  } else if (lo < 0) {
    r[nr][0] = 0; r[nr][1] = hi; ++nr;
    r[nr][0] = lo + full; r[nr][1] = full - 1; ++nr;
  } else if (hi >= full) {
    r[nr][0] = 0; r[nr][1] = hi - full; ++nr;
    r[nr][0] = lo; r[nr][1] = full - 1; ++nr;
  } else {
    r[nr][0] = lo; r[nr][1] = hi; ++nr;
  }
  for (int k = 0; k < nr; ++k) {
    const int64_t x = lower_key(a.keys_sorted, b, e, cellkey | (uint64_t)r[k][0]);
    const int64_t y = r[k][1] + 1 >= full ? e : lower_key(a.keys_sorted, b, e, cellkey | (uint64_t)(r[k][1] + 1));
    if (x < y) {
      iv[n][0] = x;
      iv[n][1] = y;
      ++n;
    }
  }
}

// Candidate intervals of sorted positions for position p, in increasing order.
__device__ __forceinline__ int candidate_intervals(const WorklistArgs& a, int64_t p, int64_t (*iv)[2]) {
  const uint64_t key = a.keys_sorted[p];
  const int s = (int)((key >> 32) & 0xFFF);
  const int c = cell_of(key, a.n_strips);
  int n = 0;
  if (a.symmetric && s > 0) cell_intervals(a, p, key, s, s - 1, c - 1, iv, n);
  cell_intervals(a, p, key, s, s, c, iv, n);
  if (s + 1 < a.n_strips) cell_intervals(a, p, key, s, s + 1, c + 1, iv, n);
  return n;
}

__device__ __forceinline__ bool keep_pair(const WorklistArgs& a, int f, int g) {
  if (!a.use_keep) return true;
  const uint64_t lo = (uint64_t)(f < g ? f : g), hi = (uint64_t)(f < g ? g : f);
  return splitmix64(a.seed ^ ((lo << 32) | hi)) < a.keep_thr;
}

// One wave per sorted position; lanes stride over the candidate range.
template <bool kFill>
__global__ __launch_bounds__(256) void neighbours_kernel(WorklistArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= a.n_forests) return;
  const int f = a.sorted[p];
  const ForestInfo fi = a.finfo[f];
  int64_t iv[6][2];
  const int niv = fi.npix > 0 ? candidate_intervals(a, p, iv) : 0;
  int64_t count = 0;
  int64_t out = kFill ? a.nb_off[p] : 0;
  unsigned long long pix = 0;
  for (int k = 0; k < niv; ++k) {
    const int64_t lo = iv[k][0], hi = iv[k][1];
    for (int64_t q0 = lo; q0 < hi; q0 += 64) {
      const int64_t q = q0 + lane;
      bool ok = false;
      if (q < hi && q != p) {
        const int g = a.sorted[q];
        const ForestInfo gi = a.finfo[g];
        ok = gi.npix > 0 && (!a.own_by_index || g > f) && pair_may_bin(fi, gi, a.eperp_max, a.epar_max) &&
             keep_pair(a, f, g);
        if (!kFill && ok) pix += (unsigned long long)gi.npix;
      }
      const uint64_t m = __ballot(ok);
      if (kFill && ok) {
        const int r = __popcll(m & ((1ull << lane) - 1ull));
        a.nbr[out + r] = (int32_t)q;
        if (a.pair_p) a.pair_p[out + r] = (int32_t)p;
      }
      const int c = __popcll(m);
      out += c;
      count += c;
    }
  }
  if (!kFill) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pix += __shfl_xor(pix, o, 64);
    if (lane == 0) {
      a.cnt[p] = count;
      if (a.cand && pix) atomicAdd(a.cand, pix * (unsigned long long)fi.npix);
    }
  }
}

__global__ void count_items_kernel(WorklistArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_forests) return;
  a.item_cnt[p] = (a.cnt[p] + a.chunk - 1) / a.chunk;
}

__global__ void fill_items_kernel(WorklistArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_forests) return;
  const int64_t n = a.cnt[p], base = a.nb_off[p], o = a.item_off[p];
  for (int64_t k = 0; k * a.chunk < n; ++k) {
    Item it;
    it.nb_begin = base + k * a.chunk;
    it.p = (int32_t)p;
    const int64_t left = n - k * a.chunk;
    it.nb_count = (int32_t)(left < a.chunk ? left : a.chunk);
    a.items[o + k] = it;
  }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

size_t worklist_cub_bytes(int64_t n) {
  size_t b1 = 0, b2 = 0;
  rocprim::radix_sort_pairs(nullptr, b1, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                            (int32_t*)nullptr, (size_t)n);
  rocprim::exclusive_scan(nullptr, b2, (int64_t*)nullptr, (int64_t*)nullptr, (int64_t)0, (size_t)n,
                          rocprim::plus<int64_t>());
  return (b1 > b2 ? b1 : b2) + 256;
}

hipError_t launch_sort_forests(WorklistArgs& a, hipStream_t st) {
  if (a.n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(keys_kernel, dim3(nblk(a.n_forests, 256)), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t bytes = a.cub_bytes;
  e = rocprim::radix_sort_pairs(a.cub_tmp, bytes, a.keys, a.keys_sorted, a.ids, a.sorted, (size_t)a.n_forests,
                                0, 64, st);
  if (e != hipSuccess) return e;
  const size_t ncell = (size_t)a.n_real * a.n_strips;
  // empty cells read -1 (a fill kernel rather than a memset node)
  hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk((int64_t)ncell, 256)), dim3(256), 0, st, a.cell_begin,
                     (int64_t)ncell, -1);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk((int64_t)ncell, 256)), dim3(256), 0, st, a.cell_end,
                     (int64_t)ncell, -1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cells_kernel, dim3(nblk(a.n_forests, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_count_neighbours(const WorklistArgs& a, hipStream_t st) {
  if (a.n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(neighbours_kernel<false>, dim3(nblk(a.n_forests, 4)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill_neighbours(const WorklistArgs& a, hipStream_t st) {
  if (a.n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(neighbours_kernel<true>, dim3(nblk(a.n_forests, 4)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scan(const int64_t* in, int64_t* out, int64_t n, void* tmp, size_t bytes,
                       hipStream_t st) {
  if (n == 0) return hipSuccess;
  return rocprim::exclusive_scan(tmp, bytes, in, out, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), st);
}

size_t sort_keys_bytes(int64_t n) {
  size_t b = 0;
  rocprim::radix_sort_pairs(nullptr, b, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                            (int32_t*)nullptr, (size_t)n);
  return b + 256;
}

hipError_t launch_sort_keys(uint64_t* keys_in, uint64_t* keys_out, int32_t* v_in, int32_t* v_out,
                            int64_t n, void* tmp, size_t bytes, hipStream_t st) {
  if (n == 0) return hipSuccess;
  return rocprim::radix_sort_pairs(tmp, bytes, keys_in, keys_out, v_in, v_out, (size_t)n, 0, 64, st);
}

hipError_t launch_count_items(const WorklistArgs& a, hipStream_t st) {
  if (a.n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(count_items_kernel, dim3(nblk(a.n_forests, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill_items(const WorklistArgs& a, hipStream_t st) {
  if (a.n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_items_kernel, dim3(nblk(a.n_forests, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace lya
