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
// lanes over pixels) and append every partner j with r_j in the r grid to a
// list (unit vector, side bins, w d, w, forest); then the ordered partner
// pairs (j, k) of different forests are binned in cos alpha.  The 5-d
// histogram is far larger than LDS.  Three kernels: the combining kernel
// (list in LDS) orders the partners by the (r, theta) cell of their side and
// sums each cell's entries in an LDS slice of the histogram before adding the
// slice to the global FP64 sums; the wide kernel does the same with the list
// in a per-workgroup global scratch, for pixels with thousands of partners;
// the direct kernel adds every entry to the global sums (grids whose slice
// does not fit LDS).  Everything is FP64; the geometry is written with
// explicit operation order so it rounds like its definition.
#include "lya_common.h"

namespace lya {

namespace {

constexpr int kBlock3 = 1024;
constexpr int kCap3 = 3072;    // partner pixels of one vertex held in LDS (direct kernel)
constexpr int kCapC = 2048;    // the same for the combining kernel
constexpr int kSliceC = 2048;  // bins of the combining kernel's LDS histogram slice
constexpr int kCellC = 1024;   // (r, theta) cells of a side, combining kernel
constexpr int kCosC = 256;     // cos alpha bins held in LDS (all kernels)
constexpr int kJStage = 512;   // side-1 partners staged in LDS at a time (wide kernel)

// Partners of one vertex pixel: unit vector of the side, w d, w, the side's
// bins k_r | k_t << 16 and the partner's forest.
template <int CAP>
struct Partners {
  double ux[CAP], uy[CAP], uz[CAP];
  double wd[CAP], w[CAP];
  int32_t key[CAP];
  int32_t fid[CAP];
};

struct Xi3Smem {
  Partners<kCap3> p;
  double ce[kCosC + 1];  // cos alpha edges
  int32_t m;  // partners appended
  int64_t item;
};

struct Xi3SmemC {
  Partners<kCapC> p;
  double hn[kSliceC], hw[kSliceC];  // slice of the sums: side-2 r bins [r_lo, r_lo + rb) x cos x theta
  uint32_t hc[kSliceC];
  uint16_t perm[kCapC];             // partners ordered by cell k_r n_t + k_t
  int32_t cstart[kCellC + 1];       // first position of each cell in perm
  int32_t cfill[kCellC];
  double ce[kCosC + 1];             // cos alpha edges
  int32_t m;
  int32_t stop;                     // another workgroup overflowed: leave the item
  int64_t item;
};

struct Xi3SmemW {
  double jx[kJStage], jy[kJStage], jz[kJStage], jwd[kJStage], jw[kJStage];  // staged side-1 partners
  int32_t jfid[kJStage];
  double hn[kSliceC], hw[kSliceC];
  uint32_t hc[kSliceC];
  int32_t cstart[kCellC + 1];
  int32_t cfill[kCellC];
  double ce[kCosC + 1];
  int32_t m;
  int64_t item;
};

// A partner list in global memory (structure of arrays, cap entries each).
struct GPartners {
  double *ux, *uy, *uz, *wd, *w;
  int32_t *key, *fid;
  __device__ __forceinline__ void operator()(int s, double x, double y, double z, double pwd, double pw, int k,
                                             int f) const {
    ux[s] = x;
    uy[s] = y;
    uz[s] = z;
    wd[s] = pwd;
    w[s] = pw;
    key[s] = k;
    fid[s] = f;
  }
};

// This workgroup's two lists (as gathered, and ordered by cell) in the scratch.
__device__ __forceinline__ GPartners scratch_list(const Xi3Args& a, int which) {
  const int64_t cap = a.w_cap;
  double* d = a.w_dbl + ((int64_t)blockIdx.x * 2 + which) * 5 * cap;
  int32_t* i = a.w_int + ((int64_t)blockIdx.x * 2 + which) * 2 * cap;
  return GPartners{d, d + cap, d + 2 * cap, d + 3 * cap, d + 4 * cap, i, i + cap};
}

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

// Stores every pixel of the item's neighbour forests whose side from the
// vertex (xi, yi, zi) has its length in the r grid and its angle to the line of
// sight n of the vertex forest in the theta grid, as
// store(slot, ux, uy, uz, w d, w, k_r | k_t << 16, forest).  A wave per
// neighbour forest, lanes over its pixels; one LDS atomic per wave reserves
// the slots.  *m counts every partner, also those beyond cap (not stored).
template <typename Store>
__device__ __forceinline__ void gather_partners(const Xi3Args& a, const Item& item, const ForestInfo& fi,
                                                double xi, double yi, double zi, int cap, int32_t* m,
                                                Store&& store) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kBlock3 / 64;
  const int nr = a.n_r, nt = a.n_t;
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
      if (lane == 0) base = atomicAdd(m, __popcll(bal));
      base = __shfl(base, 0, 64);
      if (keep) {
        const int slot = base + __popcll(bal & ((1ull << lane) - 1ull));
        if (slot < cap) store(slot, ux, uy, uz, a.pts[pj].wd, a.pts[pj].w, kr | (kt << 16), g);
      }
    }
  }
}

// The cos alpha axis with its edges in LDS and the end edges in registers (a
// load from the edge array in global memory would be a vector load waited for
// on every entry: the sums the kernels write could alias it).
struct CosAxis {
  const double* e;  // LDS copy, [n + 1]
  double lo, hi, inv;
  int n;
};

// Bin of x on the cos alpha axis, the last bin closed (-1 outside).  The host
// accepts only edges within 1e-9 bins of lo + k d, and t = (x - lo) / d is
// computed to ~1e-13 bins, so a fractional part of t farther than 1e-8 from
// 0 and 1 puts x strictly inside bin floor(t); only closer values are settled
// by comparison with the edges.
__device__ __forceinline__ int cos_axis_bin(const CosAxis& c, double x) {
  if (x < c.lo) return -1;
  if (x >= c.hi) return x == c.hi ? c.n - 1 : -1;
  const double t = __dmul_rn(__dsub_rn(x, c.lo), c.inv);
  int k = (int)t;
  k = k < 0 ? 0 : (k > c.n - 1 ? c.n - 1 : k);
  const double fr = __dsub_rn(t, (double)k);
  if (fr > 1e-8 && fr < 1.0 - 1e-8) return k;
  while (k > 0 && x < c.e[k]) --k;
  while (k < c.n - 1 && x >= c.e[k + 1]) ++k;
  return k;
}

// Copies the cos alpha edges to LDS (the caller synchronises before use).
__device__ __forceinline__ CosAxis load_cos_axis(const Xi3Args& a, double* lds) {
  for (int k = threadIdx.x; k <= a.n_c; k += kBlock3) lds[k] = a.cos_edges[k];
  return CosAxis{lds, a.cos_edges[0], a.cos_edges[a.n_c], a.c_inv, a.n_c};
}

template <int CAP>
struct LdsStore {
  Partners<CAP>& P;
  __device__ __forceinline__ void operator()(int s, double ux, double uy, double uz, double wd, double w, int key,
                                             int fid) const {
    P.ux[s] = ux;
    P.uy[s] = uy;
    P.uz[s] = uz;
    P.wd[s] = wd;
    P.w[s] = w;
    P.key[s] = key;
    P.fid[s] = fid;
  }
};

// cos alpha bin of the partners j, k (-1 outside the grid).
template <int CAP>
__device__ __forceinline__ int cos_bin(const CosAxis& cx, const Partners<CAP>& P, int j, int k) {
  double ca = __dadd_rn(__dadd_rn(__dmul_rn(P.ux[j], P.ux[k]), __dmul_rn(P.uy[j], P.uy[k])),
                        __dmul_rn(P.uz[j], P.uz[k]));
  ca = fmin(1.0, fmax(-1.0, ca));
  return cos_axis_bin(cx, ca);
}

// The sums this workgroup adds to for vertex forest f (input index): the slab
// of f's realisation (and subsample), in the copy of the workgroup's XCD when
// there is one copy per XCD (the copies spread the device-wide atomics over
// more addresses; a second kernel adds them up).
__device__ __forceinline__ int64_t sums_base(const Xi3Args& a, const ForestInfo& fi, int f) {
  const int copy = a.n_copies > 1 ? (int)(xcd_id() % (unsigned)a.n_copies) : 0;
  const int64_t slab = a.sub ? (int64_t)fi.real * a.n_sub + a.sub[f] : (int64_t)fi.real;
  return (int64_t)copy * a.copy_stride + slab * a.n_bins;
}

// Direct kernel: every entry goes to the global sums with three atomics.
__global__ __launch_bounds__(kBlock3) void xi3_kernel(Xi3Args a) {
  __shared__ Xi3Smem sm;
  const int tid = threadIdx.x;
  const int nr = a.n_r, nt = a.n_t, nc = a.n_c;
  const CosAxis cx = load_cos_axis(a, sm.ce);

  for (;;) {
    __syncthreads();  // every thread has read the previous item
    if (tid == 0) sm.item = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t it = sm.item;
    if (it >= a.n_items) break;
    const Item item = a.items[it];
    const int f = a.sorted[item.p];
    const ForestInfo fi = a.finfo[f];
    const int64_t obase = sums_base(a, fi, f);

    for (int i = 0; i < fi.npix; ++i) {
      const int64_t pi = fi.pix0 + i;
      const double wdi = a.pts[pi].wd, wi = a.pts[pi].w;
      __syncthreads();  // the previous vertex's pairs have been read
      if (tid == 0) sm.m = 0;
      __syncthreads();
      gather_partners(a, item, fi, a.pts[pi].x, a.pts[pi].y, a.pts[pi].z, kCap3, &sm.m, LdsStore<kCap3>{sm.p});
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
        if (sm.p.fid[j] != sm.p.fid[k]) {
          const int kc = cos_bin(cx, sm.p, j, k);
          if (kc >= 0) {
            const int kj = sm.p.key[j], kk = sm.p.key[k];
            const int64_t A = ((((int64_t)(kj & 0xffff) * nr + (kk & 0xffff)) * nc + kc) * nt + (kj >> 16)) * nt +
                              (kk >> 16);
            const double pn = __dmul_rn(__dmul_rn(wdi, sm.p.wd[j]), sm.p.wd[k]);
            const double pw = __dmul_rn(__dmul_rn(wi, sm.p.w[j]), sm.p.w[k]);
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

// Combining kernel.  Entries of one vertex whose first side lies in one
// (r, theta) cell differ only in (k_r2, k_c, k_t2): the partners are ordered by
// cell, and for each cell of the first side (and each block of rb side-2 r
// bins) the entries are summed in an LDS slice of n_t n_c rb bins with LDS
// atomics, then the slice's non-zero bins go to the global sums with three
// atomics each.  On the eBOSS-like workload this takes the global atomics
// down ~7x.
__global__ __launch_bounds__(kBlock3) void xi3c_kernel(Xi3Args a) {
  __shared__ Xi3SmemC sm;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int NW = kBlock3 / 64;
  const int nr = a.n_r, nt = a.n_t, nc = a.n_c;
  const int ncell = nr * nt;
  const int rb = kSliceC / (nc * nt);  // >= 1, checked by the host
  const int nblk = (nr + rb - 1) / rb;
  const CosAxis cx = load_cos_axis(a, sm.ce);

  for (int s = tid; s < kSliceC; s += kBlock3) {
    sm.hn[s] = 0.0;
    sm.hw[s] = 0.0;
    sm.hc[s] = 0u;
  }

  for (;;) {
    __syncthreads();  // every thread has read the previous item
    if (tid == 0) {
      // after an overflow the direct kernel redoes the call: stop early
      const bool over = __hip_atomic_load(&a.glob->flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kBadCapC;
      sm.item = over ? a.n_items : (int64_t)atomicAdd(a.counter, 1u);
    }
    __syncthreads();
    const int64_t it = sm.item;
    if (it >= a.n_items) break;
    const Item item = a.items[it];
    const int f = a.sorted[item.p];
    const ForestInfo fi = a.finfo[f];
    const int64_t obase = sums_base(a, fi, f);

    for (int i = 0; i < fi.npix; ++i) {
      const int64_t pi = fi.pix0 + i;
      const double wdi = a.pts[pi].wd, wi = a.pts[pi].w;
      __syncthreads();  // the previous vertex's partners have been read
      if (tid == 0) {
        sm.m = 0;
        sm.stop = __hip_atomic_load(&a.glob->flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kBadCapC;
      }
      for (int c = tid; c < ncell; c += kBlock3) sm.cfill[c] = 0;
      __syncthreads();
      if (sm.stop) break;  // the host re-runs the call with the wide kernel
      gather_partners(a, item, fi, a.pts[pi].x, a.pts[pi].y, a.pts[pi].z, kCapC, &sm.m, LdsStore<kCapC>{sm.p});
      __syncthreads();
      const int m = sm.m;
      if (m > kCapC) {
        // the host runs the direct kernel instead
        if (tid == 0) atomicOr(&a.glob->flag, kBadCapC);
        continue;
      }
      if (m < 2) continue;

      // ---- order the partners by cell: counts, exclusive scan, scatter
      for (int j = tid; j < m; j += kBlock3) {
        const int key = sm.p.key[j];
        atomicAdd(&sm.cfill[(key & 0xffff) * nt + (key >> 16)], 1);
      }
      __syncthreads();
      if (tid < 64) {
        const int per = (ncell + 63) / 64, c0 = lane * per, c1 = min(ncell, c0 + per);
        int own = 0;
        for (int c = c0; c < c1; ++c) own += sm.cfill[c];
        int incl = own;
        for (int d = 1; d < 64; d <<= 1) {
          const int v = __shfl_up(incl, d, 64);
          if (lane >= d) incl += v;
        }
        int run = incl - own;
        for (int c = c0; c < c1; ++c) {
          sm.cstart[c] = run;
          run += sm.cfill[c];
          sm.cfill[c] = 0;
        }
        if (lane == 63) sm.cstart[ncell] = incl;
      }
      __syncthreads();
      for (int j = tid; j < m; j += kBlock3) {
        const int key = sm.p.key[j];
        const int c = (key & 0xffff) * nt + (key >> 16);
        sm.perm[sm.cstart[c] + atomicAdd(&sm.cfill[c], 1)] = (uint16_t)j;
      }
      __syncthreads();

      // ---- one pass per (cell of side 1, block of side-2 r bins)
      for (int c1 = 0; c1 < ncell; ++c1) {
        const int j0 = sm.cstart[c1], nj = sm.cstart[c1 + 1] - j0;
        if (nj == 0) continue;
        const int kr1 = c1 / nt, kt1 = c1 - kr1 * nt;
        for (int b = 0; b < nblk; ++b) {
          const int r_lo = b * rb, r_hi = min(nr, r_lo + rb);
          const int k0 = sm.cstart[r_lo * nt], mk = sm.cstart[r_hi * nt] - k0;
          if (mk == 0) continue;
          // units of (64 side-2 partners, a part of the side-1 partners), a
          // wave per unit: the side-2 partners stay in registers while the
          // wave runs over its side-1 partners, and the lanes take partners
          // spread over the cells (fewer lanes adding to one LDS bin at once)
          const int nkc = (mk + 63) >> 6;
          int P = (2 * NW + nkc - 1) / nkc;
          P = P < nj ? P : nj;
          const int U = nkc * P;
          for (int u = wv; u < U; u += NW) {
            const int c = u % nkc, pp = u / nkc;
            const int kk = lane * nkc + c;
            const bool kon = kk < mk;
            double kx = 0.0, ky = 0.0, kz = 0.0, kwd = 0.0, kw = 0.0;
            int kfid = -1, sk = 0;
            if (kon) {
              const int k = sm.perm[k0 + kk];
              kx = sm.p.ux[k];
              ky = sm.p.uy[k];
              kz = sm.p.uz[k];
              kwd = sm.p.wd[k];
              kw = sm.p.w[k];
              kfid = sm.p.fid[k];
              const int kq = sm.p.key[k];
              sk = ((kq & 0xffff) - r_lo) * nc * nt + (kq >> 16);
            }
            const int jb = pp * nj / P, je = (pp + 1) * nj / P;
            int rs = -1;
            unsigned rc = 0u;
            double rn = 0.0, rw = 0.0;
            for (int jj = jb; jj < je; ++jj) {
              const int j = sm.perm[j0 + jj];
              if (kon && sm.p.fid[j] != kfid) {
                double ca = __dadd_rn(__dadd_rn(__dmul_rn(sm.p.ux[j], kx), __dmul_rn(sm.p.uy[j], ky)),
                                      __dmul_rn(sm.p.uz[j], kz));
                ca = fmin(1.0, fmax(-1.0, ca));
                const int kc = cos_axis_bin(cx, ca);
                if (kc >= 0) {
                  const int s = sk + kc * nt;
                  const double pn = __dmul_rn(__dmul_rn(wdi, sm.p.wd[j]), kwd);
                  const double pw = __dmul_rn(__dmul_rn(wi, sm.p.w[j]), kw);
                  if (s != rs) {
                    if (rs >= 0) {
                      atomicAdd(&sm.hc[rs], rc);
                      atomicAdd(&sm.hn[rs], rn);
                      atomicAdd(&sm.hw[rs], rw);
                    }
                    rs = s;
                    rc = 0u;
                    rn = 0.0;
                    rw = 0.0;
                  }
                  ++rc;
                  rn = __dadd_rn(rn, pn);
                  rw = __dadd_rn(rw, pw);
                }
              }
            }
            if (rs >= 0) {
              atomicAdd(&sm.hc[rs], rc);
              atomicAdd(&sm.hn[rs], rn);
              atomicAdd(&sm.hw[rs], rw);
            }
          }
          __syncthreads();
          // ---- flush the slice's non-zero bins and clear them (a scan of the
          // slice costs less than keeping a list of the bins touched)
          const int nsl = min(nr - r_lo, rb) * nc * nt;
          for (int s = tid; s < nsl; s += kBlock3) {
            const uint32_t vc = sm.hc[s];
            if (vc == 0u) continue;
            const double vn = sm.hn[s], vw = sm.hw[s];
            sm.hn[s] = 0.0;
            sm.hw[s] = 0.0;
            sm.hc[s] = 0u;
            const int kt2 = s % nt, q2 = s / nt, kc = q2 % nc, kr2 = r_lo + q2 / nc;
            const int64_t A = ((((int64_t)kr1 * nr + kr2) * nc + kc) * nt + kt1) * nt + kt2;
            atomicAdd(&a.num[obase + A], vn);
            atomicAdd(&a.wsum[obase + A], vw);
            atomicAdd(&a.ntrip[obase + A], (unsigned long long)vc);
          }
          __syncthreads();
        }
      }
    }
  }
}

// Wide kernel: the combining kernel's passes for vertex pixels with more
// partners than LDS holds (up to a.w_cap).  The partner list is gathered into
// the workgroup's scratch in global memory and copied there in cell order;
// each pass stages the side-1 partners of its cell in LDS (kJStage at a time)
// and the waves read their 64 side-2 partners from the ordered list.
__global__ __launch_bounds__(kBlock3) void xi3w_kernel(Xi3Args a) {
  __shared__ Xi3SmemW sm;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int NW = kBlock3 / 64;
  const int nr = a.n_r, nt = a.n_t, nc = a.n_c;
  const int ncell = nr * nt;
  const int rb = kSliceC / (nc * nt);  // >= 1, checked by the host
  const int nblk = (nr + rb - 1) / rb;
  const CosAxis cx = load_cos_axis(a, sm.ce);
  const GPartners L0 = scratch_list(a, 0), L1 = scratch_list(a, 1);

  for (int s = tid; s < kSliceC; s += kBlock3) {
    sm.hn[s] = 0.0;
    sm.hw[s] = 0.0;
    sm.hc[s] = 0u;
  }

  for (;;) {
    __syncthreads();  // every thread has read the previous item
    if (tid == 0) {
      const bool over = __hip_atomic_load(&a.glob->flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kBadCapW;
      sm.item = over ? a.n_items : (int64_t)atomicAdd(a.counter, 1u);
    }
    __syncthreads();
    const int64_t it = sm.item;
    if (it >= a.n_items) break;
    const Item item = a.items[it];
    const int f = a.sorted[item.p];
    const ForestInfo fi = a.finfo[f];
    const int64_t obase = sums_base(a, fi, f);

    for (int i = 0; i < fi.npix; ++i) {
      const int64_t pi = fi.pix0 + i;
      const double wdi = a.pts[pi].wd, wi = a.pts[pi].w;
      __syncthreads();  // the previous vertex's partners have been read
      if (tid == 0) sm.m = 0;
      for (int c = tid; c < ncell; c += kBlock3) sm.cfill[c] = 0;
      __syncthreads();
      gather_partners(a, item, fi, a.pts[pi].x, a.pts[pi].y, a.pts[pi].z, a.w_cap, &sm.m, L0);
      __syncthreads();
      const int m = sm.m;
      if (m > a.w_cap) {
        if (tid == 0) atomicOr(&a.glob->flag, kBadCapW);
        continue;
      }
      if (m < 2) continue;

      // ---- order the partners by cell into the second list
      for (int j = tid; j < m; j += kBlock3) {
        const int key = L0.key[j];
        atomicAdd(&sm.cfill[(key & 0xffff) * nt + (key >> 16)], 1);
      }
      __syncthreads();
      if (tid < 64) {
        const int per = (ncell + 63) / 64, c0 = lane * per, c1 = min(ncell, c0 + per);
        int own = 0;
        for (int c = c0; c < c1; ++c) own += sm.cfill[c];
        int incl = own;
        for (int d = 1; d < 64; d <<= 1) {
          const int v = __shfl_up(incl, d, 64);
          if (lane >= d) incl += v;
        }
        int run = incl - own;
        for (int c = c0; c < c1; ++c) {
          sm.cstart[c] = run;
          run += sm.cfill[c];
          sm.cfill[c] = 0;
        }
        if (lane == 63) sm.cstart[ncell] = incl;
      }
      __syncthreads();
      for (int j = tid; j < m; j += kBlock3) {
        const int key = L0.key[j];
        const int c = (key & 0xffff) * nt + (key >> 16);
        const int q = sm.cstart[c] + atomicAdd(&sm.cfill[c], 1);
        L1(q, L0.ux[j], L0.uy[j], L0.uz[j], L0.wd[j], L0.w[j], key, L0.fid[j]);
      }
      __syncthreads();  // the ordered list is complete (workgroup-scope fence)

      // ---- one pass per (cell of side 1, block of side-2 r bins)
      for (int c1 = 0; c1 < ncell; ++c1) {
        const int j0 = sm.cstart[c1], nj = sm.cstart[c1 + 1] - j0;
        if (nj == 0) continue;
        const int kr1 = c1 / nt, kt1 = c1 - kr1 * nt;
        for (int b = 0; b < nblk; ++b) {
          const int r_lo = b * rb, r_hi = min(nr, r_lo + rb);
          const int k0 = sm.cstart[r_lo * nt], mk = sm.cstart[r_hi * nt] - k0;
          if (mk == 0) continue;
          for (int jc = 0; jc < nj; jc += kJStage) {
            const int njc = min(kJStage, nj - jc);
            __syncthreads();  // the previous stage has been read
            for (int t = tid; t < njc; t += kBlock3) {
              const int q = j0 + jc + t;
              sm.jx[t] = L1.ux[q];
              sm.jy[t] = L1.uy[q];
              sm.jz[t] = L1.uz[q];
              sm.jwd[t] = L1.wd[q];
              sm.jw[t] = L1.w[q];
              sm.jfid[t] = L1.fid[q];
            }
            __syncthreads();
            // units of (64 side-2 partners spread over the cells, a part of
            // the staged side-1 partners), a wave per unit
            const int nkc = (mk + 63) >> 6;
            int P = (2 * NW + nkc - 1) / nkc;
            P = P < njc ? P : njc;
            const int U = nkc * P;
            for (int u = wv; u < U; u += NW) {
              const int c = u % nkc, pp = u / nkc;
              const int kk = lane * nkc + c;
              const bool kon = kk < mk;
              double kx = 0.0, ky = 0.0, kz = 0.0, kwd = 0.0, kw = 0.0;
              int kfid = -1, sk = 0;
              if (kon) {
                const int k = k0 + kk;
                kx = L1.ux[k];
                ky = L1.uy[k];
                kz = L1.uz[k];
                kwd = L1.wd[k];
                kw = L1.w[k];
                kfid = L1.fid[k];
                const int kq = L1.key[k];
                sk = ((kq & 0xffff) - r_lo) * nc * nt + (kq >> 16);
              }
              const int jb = pp * njc / P, je = (pp + 1) * njc / P;
              int rs = -1;
              unsigned rc = 0u;
              double rn = 0.0, rw = 0.0;
              for (int jj = jb; jj < je; ++jj) {
                if (kon && sm.jfid[jj] != kfid) {
                  double ca = __dadd_rn(__dadd_rn(__dmul_rn(sm.jx[jj], kx), __dmul_rn(sm.jy[jj], ky)),
                                        __dmul_rn(sm.jz[jj], kz));
                  ca = fmin(1.0, fmax(-1.0, ca));
                  const int kc = cos_axis_bin(cx, ca);
                  if (kc >= 0) {
                    const int s = sk + kc * nt;
                    const double pn = __dmul_rn(__dmul_rn(wdi, sm.jwd[jj]), kwd);
                    const double pw = __dmul_rn(__dmul_rn(wi, sm.jw[jj]), kw);
                    if (s != rs) {
                      if (rs >= 0) {
                        atomicAdd(&sm.hc[rs], rc);
                        atomicAdd(&sm.hn[rs], rn);
                        atomicAdd(&sm.hw[rs], rw);
                      }
                      rs = s;
                      rc = 0u;
                      rn = 0.0;
                      rw = 0.0;
                    }
                    ++rc;
                    rn = __dadd_rn(rn, pn);
                    rw = __dadd_rn(rw, pw);
                  }
                }
              }
              if (rs >= 0) {
                atomicAdd(&sm.hc[rs], rc);
                atomicAdd(&sm.hn[rs], rn);
                atomicAdd(&sm.hw[rs], rw);
              }
            }
          }
          __syncthreads();
          // ---- flush the slice's non-zero bins and clear them
          const int nsl = (r_hi - r_lo) * nc * nt;
          for (int s = tid; s < nsl; s += kBlock3) {
            const uint32_t vc = sm.hc[s];
            if (vc == 0u) continue;
            const double vn = sm.hn[s], vw = sm.hw[s];
            sm.hn[s] = 0.0;
            sm.hw[s] = 0.0;
            sm.hc[s] = 0u;
            const int kt2 = s % nt, q2 = s / nt, kc = q2 % nc, kr2 = r_lo + q2 / nc;
            const int64_t A = ((((int64_t)kr1 * nr + kr2) * nc + kc) * nt + kt1) * nt + kt2;
            atomicAdd(&a.num[obase + A], vn);
            atomicAdd(&a.wsum[obase + A], vw);
            atomicAdd(&a.ntrip[obase + A], (unsigned long long)vc);
          }
          __syncthreads();
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

hipError_t launch_xi3(const Xi3Args& a, int kernel, int blocks, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  if (kernel == 0)
    hipLaunchKernelGGL(xi3c_kernel, dim3(blocks), dim3(kBlock3), 0, st, a);
  else if (kernel == 1)
    hipLaunchKernelGGL(xi3_kernel, dim3(blocks), dim3(kBlock3), 0, st, a);
  else
    hipLaunchKernelGGL(xi3w_kernel, dim3(blocks), dim3(kBlock3), 0, st, a);
  return hipGetLastError();
}

int xi3_blocks_per_cu(int kernel) {
  int n = 0;
  const hipError_t e = kernel == 0   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, xi3c_kernel, kBlock3, 0)
                       : kernel == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, xi3_kernel, kBlock3, 0)
                                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, xi3w_kernel, kBlock3, 0);
  if (e != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

int xi3_partner_capacity() { return kCap3; }

int xi3_combine_capacity() { return kCapC; }

bool xi3_can_combine(int n_r, int n_t, int n_c) {
  return (int64_t)n_r * n_t <= kCellC && (int64_t)n_c * n_t <= kSliceC;
}

int xi3_max_cos_bins() { return kCosC; }

}  // namespace lya
