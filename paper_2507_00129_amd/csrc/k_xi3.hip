// Anisotropic three-point function (Sec. 2.3, eq. estimator_three):
//   xi3_A = sum_A w_i d_i w_j d_j w_k d_k / sum_A w_i w_j w_k
// over triplets of pixels from three distinct forests of one realisation.  A
// triangle is binned from a main vertex i by its sides r1 = x_j - x_i and
// r2 = x_k - x_i (x = D n): lengths r1, r2 in [r_0, r_max), angles theta1,
// theta2 to the line of sight of the vertex's quasar, and the cosine of the
// inner angle, flattened as A = (((k_r1 n_r + k_r2) n_c + k_c) n_t + k_t1) n_t
// + k_t2.  Every vertex and both side orders are entered, so an unordered
// triplet contributes six entries.  theta and cos alpha bins are half-open
// with the last one closed; a side of zero length is left out.
//
// Work layout.  A work item is one vertex forest f with all of its neighbour
// forests (a symmetric neighbour list with the box cut r_par, r_perp < r_max,
// which every side shorter than r_max passes).  The workgroup takes f's pixels
// one at a time: its waves scan the neighbours' pixels (one forest per wave,
// lanes over pixels) and append every partner j with r_j in the r grid to an
// LDS list (unit vector, side bins, w d, w, forest); then all threads run
// over the ordered partner pairs (j, k) of different forests, bin cos alpha
// and add the triplet to the global FP64 sums with atomics (the 5-d histogram
// is far larger than LDS).  Everything is FP64; the geometry is written with
// explicit operation order so it rounds like its definition.
#include "lya_common.h"

namespace lya {

namespace {

constexpr int kBlock3 = 512;
constexpr int kCap3 = 3072;  // partner pixels of one vertex held in LDS

struct Xi3Smem {
  double ux[kCap3], uy[kCap3], uz[kCap3];  // unit vector of the side to each partner
  double wd[kCap3], w[kCap3];
  int32_t key[kCap3];   // k_r | k_t << 16
  int32_t fid[kCap3];   // partner's forest
  int32_t m;            // partners appended
  int64_t item;
};

// The XCD (accelerator complex die) the wave runs on, from the XCC_ID hardware
// register (any value is correct: it only picks a copy of the sums).
__device__ __forceinline__ unsigned xcd_id() {
  unsigned x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
  return x;
}

// Bin of x on a uniform axis [e0, e0 + n / inv), with the guess corrected by
// comparisons against the edge array; closed_last puts x == e_n in bin n - 1.
__device__ __forceinline__ int uniform_bin(double x, const double* e, int n, double e0, double inv,
                                           bool closed_last) {
  if (x < e[0]) return -1;
  if (x >= e[n]) return (closed_last && x == e[n]) ? n - 1 : -1;
  int k = (int)__dmul_rn(__dsub_rn(x, e0), inv);
  k = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
  while (k > 0 && x < e[k]) --k;
  while (k < n - 1 && x >= e[k + 1]) ++k;
  return k;
}

__global__ __launch_bounds__(kBlock3) void xi3_kernel(Xi3Args a) {
  __shared__ Xi3Smem sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = kBlock3 / 64;
  const int nr = a.n_r, nt = a.n_t, nc = a.n_c;

  for (;;) {
    __syncthreads();  // every thread has read the previous item
    if (tid == 0) sm.item = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t it = sm.item;
    if (it >= a.n_items) break;
    const Item item = a.items[it];
    const int f = a.sorted[item.p];
    const ForestInfo fi = a.finfo[f];
    // with one copy of the sums per XCD, the copy of this workgroup's XCD (the
    // copies spread the device-wide atomics over more addresses: 10 % faster on
    // the benchmark grid); a second kernel adds them up
    const int copy = a.n_copies > 1 ? (int)(xcd_id() % (unsigned)a.n_copies) : 0;
    const int64_t obase = (int64_t)copy * a.copy_stride + (int64_t)fi.real * a.n_bins;

    for (int i = 0; i < fi.npix; ++i) {
      const int64_t pi = fi.pix0 + i;
      const double xi = a.pts[pi].x, yi = a.pts[pi].y, zi = a.pts[pi].z;
      const double wdi = a.pts[pi].wd, wi = a.pts[pi].w;
      __syncthreads();  // the previous vertex's pairs have been read
      if (tid == 0) sm.m = 0;
      __syncthreads();

      // ---- partners of vertex i
      for (int t = wave; t < item.nb_count; t += NW) {
        const int g = a.sorted[a.nbr[item.nb_begin + t]];
        const ForestInfo gi = a.finfo[g];
        for (int e0 = 0; e0 < gi.npix; e0 += 64) {
          const int e = e0 + lane;
          bool keep = false;
          double ux = 0.0, uy = 0.0, uz = 0.0;
          int kr = -1, kt = 0;
          const int64_t pj = gi.pix0 + e;
          if (e < gi.npix) {
            const double dx = __dsub_rn(a.pts[pj].x, xi), dy = __dsub_rn(a.pts[pj].y, yi),
                         dz = __dsub_rn(a.pts[pj].z, zi);
            const double r = sqrt(__dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)));
            kr = r > 0.0 ? uniform_bin(r, a.r_edges, nr, a.r_e0, a.r_inv, false) : -1;
            if (kr >= 0) {
              ux = __ddiv_rn(dx, r);
              uy = __ddiv_rn(dy, r);
              uz = __ddiv_rn(dz, r);
              double ct = __dadd_rn(__dadd_rn(__dmul_rn(ux, fi.nx), __dmul_rn(uy, fi.ny)), __dmul_rn(uz, fi.nz));
              ct = fmin(1.0, fmax(-1.0, ct));
              // theta >= t_k  <=>  cos theta <= cos t_k (theta in [0, pi])
              kt = 0;
              for (int k = 1; k < nt; ++k) kt += ct <= a.cos_theta_edges[k] ? 1 : 0;
              keep = ct <= a.cos_theta_edges[0] && ct >= a.cos_theta_edges[nt];
            }
          }
          const uint64_t bal = __ballot(keep);
          if (bal == 0ull) continue;
          int base = 0;
          if (lane == 0) base = atomicAdd(&sm.m, __popcll(bal));
          base = __shfl(base, 0, 64);
          if (keep) {
            const int slot = base + __popcll(bal & ((1ull << lane) - 1ull));
            if (slot < kCap3) {
              sm.ux[slot] = ux;
              sm.uy[slot] = uy;
              sm.uz[slot] = uz;
              sm.wd[slot] = a.pts[pj].wd;
              sm.w[slot] = a.pts[pj].w;
              sm.key[slot] = kr | (kt << 16);
              sm.fid[slot] = g;
            }
          }
        }
      }
      __syncthreads();
      const int m = sm.m;
      if (m > kCap3) {
        // the call reports the overflow and its sums are not used
        if (tid == 0) atomicOr(&a.glob->flag, kBadCap3);
        continue;
      }
      if (m < 2) continue;

      // ---- ordered partner pairs (j, k) of different forests, t = j m + k
      const int64_t total = (int64_t)m * m;
      int j = tid / m, k = tid - (tid / m) * m;
      const int dj = kBlock3 / m, dk = kBlock3 - dj * m;
      for (int64_t t = tid; t < total; t += kBlock3) {
        if (sm.fid[j] != sm.fid[k]) {
          double ca = __dadd_rn(__dadd_rn(__dmul_rn(sm.ux[j], sm.ux[k]), __dmul_rn(sm.uy[j], sm.uy[k])),
                                __dmul_rn(sm.uz[j], sm.uz[k]));
          ca = fmin(1.0, fmax(-1.0, ca));
          const int kc = uniform_bin(ca, a.cos_edges, nc, a.c_e0, a.c_inv, true);
          if (kc >= 0) {
            const int kj = sm.key[j], kk = sm.key[k];
            const int64_t A = ((((int64_t)(kj & 0xffff) * nr + (kk & 0xffff)) * nc + kc) * nt + (kj >> 16)) * nt +
                              (kk >> 16);
            const double pn = __dmul_rn(__dmul_rn(wdi, sm.wd[j]), sm.wd[k]);
            const double pw = __dmul_rn(__dmul_rn(wi, sm.w[j]), sm.w[k]);
            atomicAdd(&a.num[obase + A], pn);
            atomicAdd(&a.wsum[obase + A], pw);
            atomicAdd(&a.ntrip[obase + A], 1ull);
          }
        }
        k += dk;
        j += dj;
        if (k >= m) {
          k -= m;
          ++j;
        }
      }
    }
  }
}

// out = sum over the copies (copy c at c * stride).
__global__ void xi3_reduce_kernel(const double* num_c, const double* wsum_c, const unsigned long long* cnt_c,
                                  int n_copies, int64_t stride, int64_t n, double* num, double* wsum,
                                  int64_t* ntrip) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double sn = 0.0, sw = 0.0;
    unsigned long long sc = 0;
    for (int c = 0; c < n_copies; ++c) {
      sn += num_c[c * stride + i];
      sw += wsum_c[c * stride + i];
      sc += cnt_c[c * stride + i];
    }
    num[i] = sn;
    wsum[i] = sw;
    ntrip[i] = (int64_t)sc;
  }
}

// Pixel positions x = D n and the products w d, w (FP64), one wave per forest.
__global__ __launch_bounds__(256) void xi3_points_kernel(lya_forests F, const ForestInfo* finfo,
                                                       const double* delta, Point3* pts) {
  const int lane = threadIdx.x & 63;
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (f >= F.n_forests) return;
  const ForestInfo fi = finfo[f];
  for (int k = lane; k < fi.npix; k += 64) {
    const int64_t i = fi.pix0 + k;
    const double D = F.dist[i], w = F.weight[i];
    Point3 p;
    p.x = __dmul_rn(D, fi.nx);
    p.y = __dmul_rn(D, fi.ny);
    p.z = __dmul_rn(D, fi.nz);
    p.wd = __dmul_rn(w, delta[i]);
    p.w = w;
    p.pad = 0.0;
    pts[i] = p;
  }
}

}  // namespace

hipError_t launch_xi3_points(const lya_forests* F, const ForestInfo* finfo, const double* delta, Point3* pts,
                             hipStream_t st) {
  if (F->n_forests == 0) return hipSuccess;
  hipLaunchKernelGGL(xi3_points_kernel, dim3((unsigned)((F->n_forests + 3) / 4)), dim3(256), 0, st, *F, finfo,
                     delta, pts);
  return hipGetLastError();
}

hipError_t launch_xi3_reduce(const double* num_c, const double* wsum_c, const unsigned long long* cnt_c,
                             int n_copies, int64_t stride, int64_t n, double* num, double* wsum, int64_t* ntrip,
                             hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(xi3_reduce_kernel, dim3(blocks), dim3(256), 0, st, num_c, wsum_c, cnt_c, n_copies, stride, n,
                     num, wsum, ntrip);
  return hipGetLastError();
}

hipError_t launch_xi3(const Xi3Args& a, int blocks, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(xi3_kernel, dim3(blocks), dim3(kBlock3), 0, st, a);
  return hipGetLastError();
}

int xi3_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, xi3_kernel, kBlock3, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

int xi3_partner_capacity() { return kCap3; }

}  // namespace lya
