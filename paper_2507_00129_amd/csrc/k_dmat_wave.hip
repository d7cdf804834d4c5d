// Distortion matrix, one- and two-wave form (Sec. 2.2, eq. distortion).
//
// With eta_ii' = delta_ii' - p_i . q_i', p = (1, a), q = w p (1/W, 1/S) per
// forest (a = L - Lbar), the numerator of one kept forest pair (f, g) is
//   num_AB = w_A [A = B]
//          - sum_{i in f} w_i sum_l c_gl R^l_i[A] R^l_i[B]
//          - sum_{j in g} w_j sum_l c_fl R^l_j[A] R^l_j[B]
//          + sum_kl c_fk c_gl H^kl_A H^kl_B
// with c_X = (1/W_X, 1/S_X) (0 where the term is off), the row histograms
// R^l_i[A] = sum_{j: A(i,j) = A} w_j p^l_j (the other forest's pixels) and
// the pair histograms H^kl_A = sum_{(i,j) in A} w_i p^k_i w_j p^l_j.  Because
// q is p scaled per pixel by w and per forest by c, the second factor of each
// row term is the same histogram as the first and the fourth term is a sum of
// squares too: num is symmetric.  Only the blocks on and above the diagonal
// of a tile are accumulated; the flush writes each off-diagonal block twice.
//
// A workgroup of one wave (or two, below) owns its accumulator tile in
// registers and a small LDS area, and shares nothing with other workgroups.
// It takes work
// items (chunks of the window-sorted pair list) from an atomic counter; the
// pairs of a chunk that share a window (the k_perp rows their r_perp range
// spans) add into one tile, flushed to the global FP64 numerator once per
// run.  Per forest pair, rows are taken two at a time (the K = 4 of a 16x16x4
// MFMA step is two rows times l = 0, 1): the 64 lanes hold the other forest's
// pixels (up to PMAX each) and bin both rows against them, adding w and w a
// to the rows' histograms in LDS; the wave then reads the histograms back in
// MFMA operand layout, scaled by sqrt(w_row c_l), and issues one step for
// every tile block (bx <= by) that the union of the two rows' block masks
// covers.  Two LDS buffers alternate (three rotate with two waves), so the
// binning of the next two rows is issued while the matrix core works on the
// current ones.  The pair
// histograms H are summed in registers from the operands of the f rows; after
// them, one more step per block adds the H term (K = 4 is kl) and the
// Kronecker term w_A goes to an FP64 LDS accumulator.
//
// Two waves per workgroup (NW = 2) split the tile and the binning: wave w
// keeps the blocks (bx, by) with bx & 1 = w and bins row r + w of each step;
// the two rows' block masks meet in LDS after the step's barrier.
//
// Tiles: NB x NB blocks of 16 window bins (the upper triangle, NB (NB+1)/2
// accumulators).  Windows wider than NB blocks take several passes over the
// run, each re-binning the rows that can reach its blocks: a diagonal pass
// per segment of NB blocks, and rectangle passes of NX x NY blocks between
// segments.  In windows of two segments the large-tile kernels keep each
// pair's H (over the whole window, from the two diagonal passes) in a device
// store, so the later passes need only the rows whose own outer products
// reach their blocks.
#include <type_traits>

#include "lya_bin.h"
#include "lya_common.h"

namespace lya {

namespace {

typedef double wv_d4 __attribute__((ext_vector_type(4)));
typedef float wv_f4 __attribute__((ext_vector_type(4)));

// MFMA of each form.  16x16x4: operand A[i][k] and B[k][j] come from lane
// 16 k + i (resp. 16 k + j).  FP32: register r of lane 16 g + j holds row
// 4 g + r of column j; FP64: row g + 4 r.
template <typename T> struct WForm;
template <> struct WForm<float> {
  using Acc = wv_f4;
  using Rec = DRec32;
  __device__ __forceinline__ static int row(int g, int r) { return 4 * g + r; }
  __device__ __forceinline__ static Acc step(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // operand scale: the hardware square root (1 ulp), well inside the form's
  // FP32 rounding of the operands
  __device__ __forceinline__ static float root(float x) { return __builtin_amdgcn_sqrtf(x); }
};
template <> struct WForm<double> {
  using Acc = wv_d4;
  using Rec = DRec64;
  __device__ __forceinline__ static int row(int g, int r) { return g + 4 * r; }
  __device__ __forceinline__ static Acc step(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static double root(double x) { return sqrt(x); }
};

// OR over the wave, uniform result: four DPP steps reduce each row of 16
// lanes, four lane reads combine the rows.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  int x = (int)v;
  x |= __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  x |= __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  x |= __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false);  // row_ror:4
  x |= __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);  // row_ror:8
  return (uint32_t)(__builtin_amdgcn_readlane(x, 0) | __builtin_amdgcn_readlane(x, 16) |
                    __builtin_amdgcn_readlane(x, 32) | __builtin_amdgcn_readlane(x, 48));
}

__device__ __forceinline__ float bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float xor32(float v) { return __shfl_xor(v, 32, 64); }
__device__ __forceinline__ double xor32(double v) { return __shfl_xor(v, 32, 64); }

// One pass over a window of nblk blocks.  Diagonal pass: storage blocks
// [0, nx) hold window blocks x0 .. x0 + nx - 1 and the tile keeps the blocks
// bx <= by among them.  Rectangle pass: storage blocks [0, nx) hold window
// blocks x0 ..., storage blocks NX + [0, ny) hold window blocks y0 ..., and
// the tile keeps all nx x ny blocks (x and y ranges disjoint).
struct WPass {
  int x0, nx, y0, ny;
  bool diag;
  int ymin;  // diagonal pass: only pairs whose larger storage block is >= ymin
};

// Diagonal passes over segments of NB blocks, then for every pair of
// segments a < b rectangle passes over pieces of NX blocks of a times pieces
// of NY blocks of b.  Two segments (NB < nblk <= 2 NB, r = nblk - NB) take
// the diagonal pass over blocks [0, NB), a second diagonal pass over the last
// NB blocks [r, nblk) that keeps only the pairs reaching past block NB, and
// the rectangle [0, r) x [NB, nblk): 2 + ceil(r / NX) ceil(r / NY) passes,
// three instead of four for windows of 11 to 15 blocks.
template <int NB, int NX, int NY>
__device__ __forceinline__ int count_passes(int nblk) {
  const int nseg = (nblk + NB - 1) / NB;
  if (nseg == 2) {
    const int r = nblk - NB;
    return 2 + ((r + NX - 1) / NX) * ((r + NY - 1) / NY);
  }
  int n = nseg;
  for (int b = 1; b < nseg; ++b) {
    const int lb = min(NB, nblk - b * NB);
    n += b * ((NB + NX - 1) / NX) * ((lb + NY - 1) / NY);
  }
  return n;
}

template <int NB, int NX, int NY>
__device__ __forceinline__ WPass pass_of(int p, int nblk) {
  const int nseg = (nblk + NB - 1) / NB;
  if (nseg == 2) {
    const int r = nblk - NB;
    if (p == 0) return WPass{0, NB, 0, NB, true, 0};
    if (p == 1) return WPass{r, NB, r, NB, true, NB - r};
    const int py = (r + NY - 1) / NY, ix = (p - 2) / py, iy = (p - 2) % py;
    return WPass{ix * NX, min(NX, r - ix * NX), NB + iy * NY, min(NY, r - iy * NY), false, 0};
  }
  if (p < nseg) {
    const int n = min(NB, nblk - p * NB);
    return WPass{p * NB, n, p * NB, n, true, 0};
  }
  p -= nseg;
  constexpr int px = (NB + NX - 1) / NX;  // pieces of a full segment
  for (int b = 1; b < nseg; ++b) {
    const int lb = min(NB, nblk - b * NB), py = (lb + NY - 1) / NY;
    if (p < b * px * py) {
      const int a = p / (px * py), rem = p % (px * py), ix = rem / py, iy = rem % py;
      return WPass{a * NB + ix * NX, min(NX, NB - ix * NX), b * NB + iy * NY, min(NY, lb - iy * NY), false, 0};
    }
    p -= b * px * py;
  }
  return WPass{0, 0, 0, 0, true, 0};
}

template <int N> struct WIC { static constexpr int value = N; };

// Column by of slot j in the upper-triangle order j = by (by + 1) / 2 + bx.
constexpr int tri_row(int j) {
  int by = 0;
  while ((by + 1) * (by + 2) / 2 <= j) ++by;
  return by;
}

// Two waves per workgroup: block (bx, by) of the upper triangle belongs to
// wave bx & 1, in slot wrow_base(by) + (bx >> 1) of that wave (row by holds
// by / 2 + 1 slots; wave 1 leaves the last one of an even row unused).  Both
// waves then share the row structure, and a slot's column is 2 t + wave.
constexpr int wrow_base(int by) {
  int n = 0;
  for (int y = 0; y < by; ++y) n += y / 2 + 1;
  return n;
}
constexpr int wslot_row(int s) {
  int by = 0;
  while (wrow_base(by + 1) <= s) ++by;
  return by;
}

// f(WIC<I>{}) for I = B .. E - 1: indices into register arrays stay
// compile-time constants whatever the loop unroller decides.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(WIC<B>{});
    static_for<B + 1, E>(f);
  }
}

// Uniform pair data.
struct WPair {
  int64_t pf, pg;
  int nf, ng;
  double s, c;
  double fdmin, fdmax, gdmin, gdmax;
};

template <typename T, int NB, int PMAX, int WPE, bool ZLO, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void dmat_wave_kernel(DmatArgs a) {
  static_assert(NW == 1 || NW == 2, "one or two waves per workgroup");
  using Form = WForm<T>;
  using Acc = typename Form::Acc;
  using Rec = typename Form::Rec;
  constexpr bool kF32 = sizeof(T) == 4;
  constexpr int MB = NB * (NB + 1) / 2;  // accumulator blocks
  constexpr int MBW = NW == 1 ? MB : wrow_base(NB);  // accumulator slots of one wave
  constexpr int NBUF = NW == 1 ? 2 : 3;    // row-histogram buffers
  constexpr int NH = 2 / NW;               // rows of a step binned by one wave
  constexpr bool kTrim = NW == 2 || !kF32;  // per-pass pixel ranges (below)
  constexpr bool kReuse = kTrim && NB >= 7;  // pair histograms kept across passes (below)
  constexpr int NX = NB / 2, NY = NB - NX;  // rectangle passes: NX x NY blocks
  constexpr int SB = NB;                 // storage blocks per row and component
  constexpr int SW = 16 * SB + 16;       // storage stride (padded against bank conflicts)
  static_assert(NX + NY == SB, "a rectangle pass stores its x and y ranges side by side");
  constexpr int CH = 64 * PMAX;          // other-forest pixels held in registers at a time
  constexpr int GB = 4;                  // tile blocks staged per flush group
  // row histograms in FP64 in both forms: on gfx950 an LDS FP64 atomic add
  // runs ~24x faster than an FP32 one (measured by lya_measure_peaks)
  __shared__ double buf[NBUF][4][SW];    // [buffer][2 row + l][storage bin]
  __shared__ T stg[NW][GB * 256];        // flush stage of each wave: GB blocks of 16 x 16
  __shared__ uint32_t smask[3][NW];      // two waves: block mask of each wave's row, per buffer
  __shared__ int64_t s_item;             // two waves: the work item
  __shared__ uint8_t slot_by[MBW];       // block column of each accumulator slot
  __shared__ uint8_t slot_t[MBW];        // two waves: the slot's row position t (block row 2 t + wave)
  __shared__ double wdacc[16 * NB];      // w_A of the run (diagonal passes)
  __shared__ int32_t otab[16 * SB];      // output bin of each storage bin of the pass (-1 past the window)
  constexpr int RCH = 128;               // rows of a sweep staged at a time
  __shared__ T srow[3][RCH];             // d, w, w a of the staged rows
  __shared__ double srowD[RCH];          // FP64 distance of the staged rows (edge guard)

  const int lane = NW == 1 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int wv = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lk = lane >> 4, lm = lane & 15;
  const int rpar = lk >> 1, comp = lk & 1;  // operand slot of this lane: row of the step, l

  BinK<T, ZLO> K;
  K.init(a.g, a.glob, a.edges_par, a.edges_perp);
  const int NP = K.NP, NT = K.NT, nb = NP * NT;
  const Rec* __restrict__ recs;
  if constexpr (kF32) recs = a.drec32; else recs = a.drec64;

  for (int e = threadIdx.x; e < NBUF * 4 * SW; e += 64 * NW) (&buf[0][0][0])[e] = 0.0;
  for (int e = threadIdx.x; e < 16 * NB; e += 64 * NW) wdacc[e] = 0.0;
  for (int j = threadIdx.x; j < MBW; j += 64 * NW) {
    if constexpr (NW == 1) {
      slot_by[j] = (uint8_t)tri_row(j);
    } else {
      slot_by[j] = (uint8_t)wslot_row(j);
      slot_t[j] = (uint8_t)(j - wrow_base(wslot_row(j)));
    }
  }
  unsigned long long n_in = 0, n_lost = 0, nalg = 0;  // statistics only

  Acc acc[MBW];
#pragma unroll
  for (int j = 0; j < MBW; ++j) acc[j] = Acc{0, 0, 0, 0};
  T h0[SB], h1[SB];  // H partials: lane (row r, l, i) sums w_r p^k_r R^l_r[16 b + i], k = 0, 1
#pragma unroll
  for (int b = 0; b < SB; ++b) h0[b] = h1[b] = (T)0;

  // one MFMA step, tile[bx][by] += A[bx] B[by], for every block bx <= by of
  // the pass whose two storage blocks are set in the uniform mask u; a
  // rectangle pass keeps only bx < NX <= by (x range times y range).  Each
  // step sits in its own conditional block: the compiler then updates the
  // accumulators in place.
  // the pass type folded into two block masks up front, so that each block
  // pair costs one scalar bit test: a rectangle pass keeps the pairs with
  // bx < NX <= by, a diagonal pass every bx <= by
  // With two waves, each issues the steps of its own blocks, (2 t + wv, by).
  auto tile_steps = [&](uint32_t u, bool diag, int ymin, const T* A, const T* B) __attribute__((always_inline)) {
    constexpr uint32_t kXMask = (1u << NX) - 1u;
    const uint32_t ux = diag ? u : (u & kXMask), uy = diag ? (u & ~((1u << ymin) - 1u)) : (u & ~kXMask);
    if constexpr (NW == 1) {
      static_for<0, NB>([&](auto BY) __attribute__((always_inline)) {
        constexpr int by = decltype(BY)::value;
        if (!((uy >> by) & 1u)) return;
        static_for<0, by + 1>([&](auto BX) __attribute__((always_inline)) {
          constexpr int bx = decltype(BX)::value;
          constexpr int j = by * (by + 1) / 2 + bx;
          if ((ux >> bx) & 1u) acc[j] = Form::step(A[bx], B[by], acc[j]);
        });
      });
    } else {
      const uint32_t uxw = ux >> wv;  // bit 2 t: block 2 t + wv
      T Aw[(NB + 1) / 2];
#pragma unroll
      for (int t = 0; t < (NB + 1) / 2; ++t) Aw[t] = (2 * t + 1 < NB && wv) ? A[2 * t + 1] : A[2 * t];
      static_for<0, NB>([&](auto BY) __attribute__((always_inline)) {
        constexpr int by = decltype(BY)::value;
        if (!((uy >> by) & 1u)) return;
        static_for<0, by / 2 + 1>([&](auto TT) __attribute__((always_inline)) {
          constexpr int t = decltype(TT)::value;
          constexpr int sl = wrow_base(by) + t;
          const bool on = (2 * t == by) ? (wv == 0 && (uxw >> (2 * t)) & 1u) : ((uxw >> (2 * t)) & 1u);
          if (on) acc[sl] = Form::step(Aw[t], B[by], acc[sl]);
        });
      });
    }
  };

  for (;;) {
    __syncthreads();
    int64_t it;
    if constexpr (NW == 1) {
      unsigned itv = 0;
      if (lane == 0) itv = atomicAdd(a.counter, 1u);
      it = (int64_t)(unsigned)__builtin_amdgcn_readlane((int)itv, 0);
    } else {
      if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(a.counter, 1u);
      __syncthreads();
      it = s_item;
    }
    if (it >= a.n_items) break;
    const int64_t k0 = it * a.item_stride * a.chunk;
    const int64_t k1 = min(a.n_pairs, k0 + (int64_t)a.chunk);
    for (int64_t r0 = k0; r0 < k1;) {
      const uint64_t key = a.wkeys[r0];
      int64_t lo = r0 + 1, hi = k1;  // end of the run of equal keys
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.wkeys[mid] == key) lo = mid + 1; else hi = mid;
      }
      int64_t r1 = lo;
      if (key == ~0ull) {
        r0 = r1;
        continue;
      }
      const int real = dmat_key_real(key);
      const int kt0 = dmat_key_kt0(key);
      const int span = dmat_key_span(key);
      const int nwin = span * NP;
      const int base_L = kt0 * NP;
      const int nblk = (nwin + 15) >> 4;
      const int64_t obase = (int64_t)real * nb;
      const int npass = count_passes<NB, NX, NY>(nblk);
      // Windows of two segments (three or more passes) keep each pair's
      // histograms H between passes: the first diagonal pass stores H over the
      // window's first NB blocks, the second over the rest, and the later
      // passes read them, so that they need only the f rows whose own outer
      // products reach their blocks.  The store holds hsave_run pairs per wave,
      // so a run is cut into pieces of at most that many (each its own tile).
      const bool reuse = kReuse && a.hsave != nullptr && nblk > NB && nblk <= 2 * NB;
      if (reuse) r1 = min(r1, r0 + (int64_t)a.hsave_run);
      T* const hsbase =
          reuse ? (T*)a.hsave + ((int64_t)blockIdx.x * NW + wv) * a.hsave_run * (int64_t)(2 * NB * 64) + lane
                : nullptr;

      for (int ps = 0; ps < npass; ++ps) {
        const WPass P = pass_of<NB, NX, NY>(ps, nblk);
        __syncthreads();  // the previous pass's flush has read the table
        for (int e = threadIdx.x; e < 16 * SB; e += 64 * NW) {
          const int sb = e >> 4;
          const bool ypart = !P.diag && sb >= NX;
          const int wb = ypart ? P.y0 + (sb - NX) : P.x0 + sb;
          const int w = 16 * wb + (e & 15);
          const bool used = ypart ? sb - NX < P.ny : sb < P.nx;
          otab[e] = (used && w < nwin) ? out_index(w + base_L, NP, NT) : -1;
        }

        for (int64_t kk = r0; kk < r1; ++kk) {
          const int q = a.worder[kk];
          WPair pr;
          {
            const ForestInfo fi = a.finfo[a.sorted[a.pair_p[q]]];
            const ForestInfo gi = a.finfo[a.sorted[a.nbr[q]]];
            pair_sc(fi, gi, pr.s, pr.c);
            pr.pf = fi.pix0;
            pr.pg = gi.pix0;
            pr.nf = fi.npix;
            pr.ng = gi.npix;
            pr.fdmin = fi.dmin;
            pr.fdmax = fi.dmax;
            pr.gdmin = gi.dmin;
            pr.gdmax = gi.dmax;
          }
          // pixels within r_par reach of the other forest's extent: the first and
          // last such pixel of each forest bound the rows and the lanes' pixels
          const double reach = a.g.emax_par / pr.c * (1.0 + 1e-12) + 1e-9;
          // A window of several passes (two-wave FP32 kernel, FP64 kernels; in the
          // one-wave FP32 kernels the extra registers spilled): pixels are kept
          // only where they can reach the pass's blocks.  A pixel at distance D
          // against the other forest's extent [Omin, Omax] has r_perp in
          // [(D + Omin) s, (D + Omax) s]; window blocks B0 .. B1 hold k_perp rows
          // kt0 + floor(16 B0 / NP) .. kt0 + floor((16 B1 + 15) / NP), r_perp in
          // [e(B0), e(B1)) of the FP64 edges, and every bin decision agrees with
          // the FP64 edge comparison.  Both
          // forests' pixels are kept where they reach any block of the pass (the
          // f rows also feed H, which every block needs); the g rows of the second
          // sweep only where they reach both ranges of a rectangle pass (a row's
          // outer product there pairs a bin of each range), or the blocks from
          // ymin on of a diagonal pass.  Widened by a relative 1e-9.  Not in the
          // first pass of a counted launch, which counts the in-window pairs.
          // (with the histograms kept across passes, the f rows of the later
          // passes follow the same rule as the g rows)
          const bool frows = reuse && ps > 0;
          double ulo[2] = {-INFINITY, -INFINITY}, uhi[2] = {INFINITY, INFINITY};
          double rlo[2] = {-INFINITY, -INFINITY}, rhi[2] = {INFINITY, INFINITY};
          if (kTrim && npass > 1 && !(a.counters && ps == 0) && pr.s > 0.0) {
            auto edge_lo = [&](int B) { return K.et[kt0 + min(span - 1, (16 * B) / NP)]; };
            auto edge_hi = [&](int B) { return K.et[kt0 + min(span - 1, (16 * B + 15) / NP) + 1]; };
            const int u1 = P.diag ? P.x0 + P.nx - 1 : P.y0 + P.ny - 1;
            const double el = edge_lo(P.x0) * (1.0 - 1e-9) / pr.s, eh = edge_hi(u1) * (1.0 + 1e-9) / pr.s;
            ulo[0] = el - pr.gdmax - 1e-6;  // f against g
            uhi[0] = eh - pr.gdmin + 1e-6;
            ulo[1] = el - pr.fdmax - 1e-6;  // g against f
            uhi[1] = eh - pr.fdmin + 1e-6;
            const double erl = edge_lo(P.diag ? P.x0 + P.ymin : P.y0) * (1.0 - 1e-9) / pr.s;
            const double erh = edge_hi(P.x0 + P.nx - 1) * (1.0 + 1e-9) / pr.s;
            rlo[0] = erl - pr.gdmax - 1e-6;
            rhi[0] = erh - pr.gdmin + 1e-6;
            rlo[1] = erl - pr.fdmax - 1e-6;
            rhi[1] = erh - pr.fdmin + 1e-6;
          }
          int rng[8];
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int n = side ? pr.ng : pr.nf;
            const int64_t p0 = side ? pr.pg : pr.pf;
            const double lo_d = (side ? pr.fdmin : pr.gdmin) - reach, hi_d = (side ? pr.fdmax : pr.gdmax) + reach;
            const double lo_u = fmax(lo_d, ulo[side]), hi_u = fmin(hi_d, uhi[side]);
            const double lo_r = fmax(lo_d, rlo[side]), hi_r = fmin(hi_d, rhi[side]);
            const bool rows_own = side == 1 || frows;  // rows on their own rule
            int first = 0x7fffffff, last = -1, rfirst = 0x7fffffff, rlast = -1;
            for (int e0 = 0; e0 < n; e0 += 64) {
              const int e = e0 + lane;
              bool in = false, inr = false;
              if (e < n) {
                double D;
                if constexpr (kF32) D = recs[p0 + e].D; else D = recs[p0 + e].d;
                in = D > lo_u && D < hi_u;
                inr = D > lo_r && D < hi_r;
              }
              const uint64_t m = __ballot(in);
              if (m != 0ull) {
                first = min(first, e0 + __ffsll((long long)m) - 1);
                last = e0 + 63 - __clzll((long long)m);
              }
              if (kTrim && rows_own) {
                const uint64_t mr = __ballot(inr);
                if (mr != 0ull) {
                  rfirst = min(rfirst, e0 + __ffsll((long long)mr) - 1);
                  rlast = e0 + 63 - __clzll((long long)mr);
                }
              }
            }
            rng[2 * side] = first;
            rng[2 * side + 1] = last;
            rng[4 + 2 * side] = kTrim && rows_own ? rfirst : first;
            rng[5 + 2 * side] = kTrim && rows_own ? rlast : last;
          }
          const int f_lo = rng[0], f_n = rng[1] + 1 - rng[0];
          const int g_lo = rng[2], g_n = rng[3] + 1 - rng[2];
          const int fr_lo = rng[4], fr_n = max(0, rng[5] + 1 - rng[4]);  // f rows of the first sweep
          const int gr_lo = rng[6], gr_n = max(0, rng[7] + 1 - rng[6]);  // g rows of the second sweep
          // no pixel pair of these forests in the grid (or the pass); a pass that
          // keeps histograms still goes on without rows, to store zeros
          const bool none = f_n <= 0 || g_n <= 0;
          if (none && !(reuse && ps < 2)) continue;
          T cf0, cf1, cg0, cg1;  // c of f and g: (1 / W, 1 / S), 0 where the term is off
          {
            const EtaInfo ef = a.einfo[a.sorted[a.pair_p[q]]];
            const EtaInfo eg = a.einfo[a.sorted[a.nbr[q]]];
            cf0 = (T)(ef.active ? 1.0 / ef.W : 0.0);
            cf1 = (T)(ef.slope ? 1.0 / ef.S : 0.0);
            cg0 = (T)(eg.active ? 1.0 / eg.W : 0.0);
            cg1 = (T)(eg.slope ? 1.0 / eg.S : 0.0);
          }
          const T s = (T)pr.s, c = (T)pr.c;
          const T bsep = kF32 ? (T)(2.0 * a.glob->dc * pr.s) : (T)0;
          const bool count_in = a.counters && ps == 0;

          // the two sweeps: rows of f against g's pixels (rs = 0, which also sums
          // the pair histograms H), then rows of g against f's pixels
          uint32_t u_h = 0;  // blocks the H partials reach
#pragma unroll
          for (int b = 0; b < SB; ++b) h0[b] = h1[b] = (T)0;
#pragma unroll 1
          for (int rs = 0; rs < 2; ++rs) {
            const int nr = none ? 0 : (rs ? gr_n : fr_n), no = rs ? f_n : g_n;
            const int64_t prow0 = rs ? pr.pg + gr_lo : pr.pf + fr_lo;
            const int64_t poth0 = rs ? pr.pf + f_lo : pr.pg + g_lo;
            const T co_l = comp ? (rs ? cf1 : cg1) : (rs ? cf0 : cg0);  // c of the other forest, this lane's l
            const int nch = (no + CH - 1) / CH;
            // the other forest's pixels, CH at a time, in registers: lane l holds
            // pixels c0 + l ppl + k, k < ppl <= PMAX (blocked, so that the 64 pixels
            // of one k are spread over the forest and mostly fall in different bins)
            T od[PMAX], ow[PMAX], owa[PMAX];
            int ppl = 0, cn = 0, cload = -1;
            auto load_other = [&](int c0) {
              if (c0 == cload) return;
              cload = c0;
              cn = min(CH, no - c0);
              ppl = (cn + 63) >> 6;
#pragma unroll
              for (int k = 0; k < PMAX; ++k) {
                const int j = lane * ppl + k;
                od[k] = (T)1e30;  // far away: never in the grid
                ow[k] = owa[k] = (T)0;
                if (k < ppl && j < cn) {
                  const Rec rec = recs[poth0 + c0 + j];
                  od[k] = rec.d;
                  ow[k] = rec.w;
                  owa[k] = rec.w * rec.a;
                }
              }
            };
            // the rows, RCH at a time, staged in LDS from rbase on (rows past nr as zeros)
            int rbase = -RCH;
            auto rows_at = [&](int r) {
              const int cb = r & ~(RCH - 1);
              if (cb == rbase) return;
              rbase = cb;
              __syncthreads();
              for (int i = threadIdx.x; i < RCH; i += 64 * NW) {
                const int rr = cb + i;
                T d = 0, w = 0, wa = 0;
                double D = 0.0;
                if (rr < nr) {
                  const Rec rec = recs[prow0 + rr];
                  d = rec.d;
                  w = rec.w;
                  wa = rec.w * rec.a;
                  if constexpr (kF32) D = rec.D; else D = rec.d;
                }
                srow[0][i] = d;
                srow[1][i] = w;
                srow[2][i] = wa;
                srowD[i] = D;
              }
              __syncthreads();
            };
            // bins rows r and r + 1 into buffer bsel (w and w a added at each pair's
            // storage bin); returns the union of their block masks (uniform).  The
            // 2 x NK evaluations of a chunk run in three phases -- the FP32 bins,
            // then the FP64 edge path where some lane needs it (a uniform branch),
            // then the storage bins and the LDS adds -- so that the independent
            // evaluations interleave instead of waiting on one another.
            auto bin_chunk = [&](auto NKC, int c0, int r, int bsel, const T* rdv, bool row1ok)
                __attribute__((always_inline)) -> uint32_t {
              constexpr int NKE = decltype(NKC)::value;
              int L[NH][NKE];
              bool inr[NH][NKE], need[NH][NKE];
              bool anyneed = false;
#pragma unroll
              for (int hi = 0; hi < NH; ++hi) {
                const int h = NW == 1 ? hi : wv;  // row r + h
#pragma unroll
                for (int k = 0; k < NKE; ++k) {
                  T rp, rt;
                  separations(rdv[hi], od[k], c, s, bsep, rp, rt);
                  T xp, xt;
                  if constexpr (ZLO) {
                    xp = rp * K.invp;
                    xt = rt * K.invt;
                  } else {
                    xp = (rp - K.e0p) * K.invp;
                    xt = (rt - K.e0t) * K.invt;
                  }
                  const bool in = (h == 0 || row1ok) & (xp < K.np_hi) & (xt < K.nt_hi) &
                                  (ZLO || ((xp > K.lo_p) & (xt > K.lo_t)));
                  const T rxp = rint(xp), rxt = rint(xt);
                  bool gp = fabs(xp - rxp) < K.taup, gt = fabs(xt - rxt) < K.taut;
                  if constexpr (ZLO) {
                    gp &= rxp != (T)0;
                  } else {
                    gp &= !(K.zlp & (rxp == (T)0));
                    gt &= !(K.zlt & (rxt == (T)0));
                  }
                  // (clamped before the conversion: out-of-range lanes are discarded below)
                  L[hi][k] = (int)__umul24((unsigned)(int)fmin(xt, (T)65536), (unsigned)NP) + (int)fmin(xp, (T)65536);
                  inr[hi][k] = in;
                  need[hi][k] = in & (gp | gt);
                  anyneed |= need[hi][k];
                }
              }
              if (__ballot(anyneed)) {
                // within rounding of an edge: the FP64 separations against the edges
#pragma unroll
                for (int hi = 0; hi < NH; ++hi) {
                  const int h = NW == 1 ? hi : wv;  // row r + h
#pragma unroll
                  for (int k = 0; k < NKE; ++k) {
                    if (need[hi][k]) {
                      double rp64, rt64;
                      if constexpr (kF32) {
                        separations64(srowD[r + h - rbase], recs[poth0 + c0 + lane * ppl + k].D, pr.c, pr.s,
                                      rp64, rt64);
                      } else {
                        separations(rdv[hi], od[k], c, s, bsep, rp64, rt64);
                      }
                      const int kp = bin_exact(rp64, K.ep, NP, (int)floor((rp64 - a.g.e0_par) * a.g.inv_par));
                      const int kt = bin_exact(rt64, K.et, NT, (int)floor((rt64 - a.g.e0_perp) * a.g.inv_perp));
                      L[hi][k] = (kp >= 0 && kt >= 0) ? (int)__umul24((unsigned)kt, (unsigned)NP) + kp : -1;
                    }
                  }
                }
              }
              uint32_t bits = 0;
              int sidx[NH][NKE];
              bool ok[NH][NKE];
#pragma unroll
              for (int hi = 0; hi < NH; ++hi) {
#pragma unroll
                for (int k = 0; k < NKE; ++k) {
                  const int w = L[hi][k] - base_L;
                  const bool ing = inr[hi][k] & (L[hi][k] >= 0);
                  const bool inw = ing & ((unsigned)w < (unsigned)nwin);
                  if (a.counters) {  // statistics only (uniform)
                    n_lost += (ing & !inw) ? 1ull : 0ull;
                    if (count_in && rs == 0) n_in += inw ? 1ull : 0ull;
                  }
                  // storage bin of the pass
                  const int wx = w - 16 * P.x0, wy = w - 16 * P.y0;
                  const bool okx = (unsigned)wx < (unsigned)(16 * P.nx);
                  const bool oky = !P.diag & ((unsigned)wy < (unsigned)(16 * P.ny));
                  sidx[hi][k] = okx ? wx : 16 * NX + wy;
                  ok[hi][k] = inw & (okx | oky);
                  bits |= ok[hi][k] ? (1u << ((sidx[hi][k] >> 4) & 31)) : 0u;
                }
              }
#pragma unroll
              for (int hi = 0; hi < NH; ++hi) {
                const int h = NW == 1 ? hi : wv;  // row r + h
                double* hw = &buf[bsel][2 * h][0];
#pragma unroll
                for (int k = 0; k < NKE; ++k) {
                  if (ok[hi][k]) {
                    atomicAdd(&hw[sidx[hi][k]], (double)ow[k]);
                    atomicAdd(&hw[SW + sidx[hi][k]], (double)owa[k]);
                  }
                }
              }
              return bits;
            };
            // with two waves, wave h bins row r + h; the block masks of the two
            // rows are combined through LDS after the next barrier
            auto bin_rows = [&](int r, int bsel) -> uint32_t {
              uint32_t bits = 0;
              rows_at(r);
              T rdv[NH];
              if constexpr (NW == 1) {
                rdv[0] = srow[0][r - rbase];
                rdv[1] = srow[0][r + 1 - rbase];
              } else {
                rdv[0] = srow[0][r + wv - rbase];
              }
              const bool row1ok = r + 1 < nr;
#pragma unroll 1
              for (int c0 = 0; c0 < no; c0 += CH) {
                load_other(c0);
                // slots k >= ppl hold far-away pixels (never in the grid)
                if (ppl <= 2) bits |= bin_chunk(std::integral_constant<int, 2 < PMAX ? 2 : PMAX>{}, c0, r, bsel, rdv, row1ok);
                else bits |= bin_chunk(std::integral_constant<int, PMAX>{}, c0, r, bsel, rdv, row1ok);
              }
              return wave_or(bits);
            };

            // steps of two rows; the binning of step st + 1 is issued before the
            // matrix steps of step st, into the next buffer.  One wave reads and
            // clears its buffer in one step (two buffers); with two waves, a buffer
            // read in step st is cleared in step st + 1, after the barrier that
            // follows both waves' reads, so three buffers rotate.
            const int nsteps = (nr + 1) >> 1;
            uint32_t ucur = 0;
#pragma unroll 1
            for (int st = -1; st < nsteps; ++st) {
              T op[SB];
              T wr = 0, wra = 0;
              if (st >= 0) {
                __syncthreads();  // the rows' LDS adds (and the last clears) are complete
                const int bsel = NW == 1 ? (st & 1) : st % 3;
                if constexpr (NW == 2) ucur = (uint32_t)__builtin_amdgcn_readfirstlane((int)(smask[bsel][0] | smask[bsel][1]));
                // this lane's row (rows past nr were staged as zeros)
                wr = srow[1][2 * st + rpar - rbase];
                wra = srow[2][2 * st + rpar - rbase];
                // operands: R^l of the lane's row over every block slot (slots the
                // step does not reach hold zeros), read without branches so the
                // reads overlap; the slots are cleared for the next use of this buffer
                double ov[SB];
#pragma unroll
                for (int b = 0; b < SB; ++b) ov[b] = buf[bsel][lk][16 * b + lm];
                if constexpr (NW == 1) {
#pragma unroll
                  for (int b = 0; b < SB; ++b) {
                    op[b] = (T)ov[b];
                    buf[bsel][lk][16 * b + lm] = 0.0;
                  }
                } else {
                  const int bclr = (st + 2) % 3;  // read by both waves in step st - 1
#pragma unroll
                  for (int b = 0; b < SB; ++b) {
                    op[b] = (T)ov[b];
                    if ((b & 1) == wv) buf[bclr][lk][16 * b + lm] = 0.0;
                  }
                }
              }
              const uint32_t unext =
                  st + 1 < nsteps ? bin_rows(2 * st + 2, NW == 1 ? ((st + 1) & 1) : (st + 1) % 3) : 0u;
              if constexpr (NW == 2) {
                if (lane == 0) smask[(st + 1) % 3][wv] = unext;
              }
              if (st >= 0) {
                if (a.counters && wv == 0) {
                  // outer-product FMAs of the sparse rows: 2 per (x, y) of nonzero R bins,
                  // counted per row over the x and y ranges
                  // (a diagonal pass with ymin > 0 counts the pairs reaching block ymin:
                  // all of its pairs less those below it)
                  int cx[2] = {0, 0}, cy[2] = {0, 0}, cl[2] = {0, 0};
#pragma unroll
                  for (int b = 0; b < SB; ++b) {
                    if (!((ucur >> b) & 1u)) continue;
                    const uint64_t m = __ballot(op[b] != (T)0);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                      const int nz = __popc((uint32_t)((m >> (32 * h)) | (m >> (32 * h + 16))) & 0xFFFFu);
                      if (P.diag || b < NX) cx[h] += nz; else cy[h] += nz;
                      if (P.diag && b < P.ymin) cl[h] += nz;
                    }
                  }
#pragma unroll
                  for (int h = 0; h < 2; ++h)
                    nalg += P.diag ? 2ull * (unsigned long long)(cx[h] * cx[h] - cl[h] * cl[h])
                                   : 2ull * (unsigned long long)cx[h] * (unsigned long long)cy[h];
                }
                if (rs == 0) {
                  u_h |= ucur;
#pragma unroll
                  for (int b = 0; b < SB; ++b)
                    if ((ucur >> b) & 1u) {
                      h0[b] = fma(wr, op[b], h0[b]);
                      h1[b] = fma(wra, op[b], h1[b]);
                    }
                }
                const T sq = Form::root(wr * co_l);
#pragma unroll
                for (int b = 0; b < SB; ++b) op[b] *= sq;
                tile_steps(ucur, P.diag, P.ymin, op, op);
              }
              if constexpr (NW == 1) ucur = unext;
            }
            if constexpr (NW == 2) {
              // the last step's buffer, once both waves have read it
              if (nsteps > 0) {
                __syncthreads();
                const int bl = (nsteps - 1) % 3;
#pragma unroll
                for (int b = 0; b < SB; ++b)
                  if ((b & 1) == wv) buf[bl][lk][16 * b + lm] = 0.0;
              }
            }

          }
          // ---- the pair term H (x) H, from the f rows' histograms
          // ---- H: add the two row halves; lane (kl, i) then holds H^kl[16 b + i]
#pragma unroll
          for (int b = 0; b < SB; ++b) {
            if (!((u_h >> b) & 1u)) continue;
            const T mine = lane < 32 ? h0[b] : h1[b];
            const T give = lane < 32 ? h1[b] : h0[b];
            h0[b] = mine + xor32(give);
          }
          if (reuse) {
            // kept histograms: window block w of this pair at hs[w * 64]; the
            // first pass stores its blocks, the second its blocks from ymin on
            // (complete: every pair there has an f row that reaches them) and
            // reads the ones below, the rectangle passes read both ranges
            T* const hs = hsbase + (kk - r0) * (int64_t)(2 * NB * 64);
            if (ps < 2) {
#pragma unroll
              for (int b = 0; b < SB; ++b) {
                if (b < P.ymin) h0[b] = hs[(P.x0 + b) * 64];
                else if (b < P.nx) hs[(P.x0 + b) * 64] = h0[b];
              }
              u_h |= (1u << P.ymin) - 1u;
            } else {
#pragma unroll
              for (int b = 0; b < SB; ++b) {
                if (b < P.nx) h0[b] = hs[(P.x0 + b) * 64];
                else if (b >= NX && b - NX < P.ny) h0[b] = hs[(P.y0 + b - NX) * 64];
              }
              u_h |= ((1u << P.nx) - 1u) | (((1u << P.ny) - 1u) << NX);
            }
          }
          // H term: A = -c_fk c_gl H^kl (k = lane's row slot, l = its component), B = H^kl
          const T s4 = -(rpar ? cf1 : cf0) * (comp ? cg1 : cg0);
#pragma unroll
          for (int b = 0; b < SB; ++b) h1[b] = h0[b] * s4;
          // every block of the pass (blocks H does not reach add zeros; pairs below
          // ymin get a zero operand): the masked form of these steps came out of
          // the compiler without the H term
          T hq[SB];
#pragma unroll
          for (int b = 0; b < SB; ++b) hq[b] = b >= P.ymin ? h0[b] : (T)0;
          if constexpr (NW == 1) {
            static_for<0, NB>([&](auto BY) __attribute__((always_inline)) {
              constexpr int by = decltype(BY)::value;
              static_for<0, by + 1>([&](auto BX) __attribute__((always_inline)) {
                constexpr int bx = decltype(BX)::value;
                constexpr int j = by * (by + 1) / 2 + bx;
                constexpr bool in_rect = bx < NX && by >= NX;
                if (in_rect || P.diag) acc[j] = Form::step(h1[bx], hq[by], acc[j]);
              });
            });
          } else {
            T hw[(NB + 1) / 2];
#pragma unroll
            for (int t = 0; t < (NB + 1) / 2; ++t) hw[t] = (2 * t + 1 < NB && wv) ? h1[2 * t + 1] : h1[2 * t];
            static_for<0, NB>([&](auto BY) __attribute__((always_inline)) {
              constexpr int by = decltype(BY)::value;
              static_for<0, by / 2 + 1>([&](auto TT) __attribute__((always_inline)) {
                constexpr int t = decltype(TT)::value;
                constexpr int sl = wrow_base(by) + t;
                const int bx = 2 * t + wv;
                const bool in_rect = bx < NX && by >= NX;
                if (bx <= by && (in_rect || P.diag)) acc[sl] = Form::step(hw[t], hq[by], acc[sl]);
              });
            });
          }
          if (a.counters && wv == 0) {
            int hx = 0, qy = 0, hl = 0, ql = 0;
#pragma unroll
            for (int b = 0; b < SB; ++b) {
              if (!((u_h >> b) & 1u)) continue;
              const uint64_t m0 = __ballot(lk == 0 && h0[b] != (T)0);
              const uint64_t m3 = __ballot(lk == 3 && h0[b] != (T)0);
              const int n0 = __popcll(m0), nq = __popc((uint32_t)(m0 | (m3 >> 48)) & 0xFFFFu);
              if (P.diag || b < NX) hx += n0;
              if (P.diag || b >= NX) qy += nq;
              if (P.diag && b < P.ymin) {
                hl += n0;
                ql += nq;
              }
            }
            nalg += 4ull * (unsigned long long)(hx * qy - hl * ql);
          }
          // w_A and the Kronecker term, from H^00 (lanes 0..15)
          if (P.diag && lk == 0 && wv == 0) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
              if (((u_h >> b) & 1u) && b >= P.ymin) wdacc[16 * b + lm] += (double)h0[b];
          }
        }

        // ---- add the tile (num gets -tile) and w_A to the global sums.  The
        // blocks go through an LDS stage GB at a time, so the atomics are one
        // loop; off-diagonal blocks (bx < by, every block of a rectangle pass)
        // also go to (y, x).
        // (with two waves, each flushes its own slots)
        static_for<0, (MBW + GB - 1) / GB>([&](auto G) __attribute__((always_inline)) {
          constexpr int g = decltype(G)::value;
          __syncthreads();  // the previous group's stage has been read
          static_for<0, GB>([&](auto I) __attribute__((always_inline)) {
            constexpr int jj = g * GB + decltype(I)::value;
            if constexpr (jj < MBW) {
#pragma unroll
              for (int r = 0; r < 4; ++r) stg[wv][(decltype(I)::value * 16 + Form::row(lk, r)) * 16 + lm] = acc[jj][r];
              acc[jj] = Acc{0, 0, 0, 0};
            }
          });
          __syncthreads();
          for (int e = lane; e < GB * 256; e += 64) {
            const int jj = g * GB + (e >> 8);
            if (jj >= MBW) break;
            const double v = -(double)stg[wv][e];
            int by, bx;
            if constexpr (NW == 1) {
              by = slot_by[jj];
              bx = jj - by * (by + 1) / 2;
            } else {
              by = slot_by[jj];
              bx = 2 * slot_t[jj] + wv;
              if (bx > by) continue;  // wave 1's unused slot of an even row (zeros)
            }
            const int ox = otab[16 * bx + ((e >> 4) & 15)], oy = otab[16 * by + (e & 15)];
            if (v != 0.0 && ox >= 0 && oy >= 0) {
              atomicAdd(&a.dnum[(obase + ox) * nb + oy], v);
              if (bx != by) atomicAdd(&a.dnum[(obase + oy) * nb + ox], v);
            }
          }
        });
        if (P.diag) {
          for (int x = threadIdx.x; x < 16 * P.nx; x += 64 * NW) {
            const double v = wdacc[x];
            const int ox = otab[x];
            if (v != 0.0 && ox >= 0) {
              atomicAdd(&a.wd[obase + ox], v);
              atomicAdd(&a.dnum[(obase + ox) * nb + ox], v);
            }
            wdacc[x] = 0.0;
          }
        }
      }
      r0 = r1;
    }
  }
  if (a.counters) {
    unsigned long long ni = n_in, nl = n_lost;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      ni += __shfl_xor(ni, o, 64);
      nl += __shfl_xor(nl, o, 64);
    }
    if (lane == 0) {
      atomicAdd(&a.counters[0], ni);
      atomicAdd(&a.counters[1], nalg);
      atomicAdd(&a.counters[2], nl);
    }
  }
}

template <typename T, int NB, int PMAX, int WPE, int NW>
hipError_t launch_wave(const DmatArgs& a, int blocks, hipStream_t st) {
  if (a.g.zero_lo_par && a.g.zero_lo_perp)
    hipLaunchKernelGGL((dmat_wave_kernel<T, NB, PMAX, WPE, true, NW>), dim3(blocks), dim3(64 * NW), 0, st, a);
  else
    hipLaunchKernelGGL((dmat_wave_kernel<T, NB, PMAX, WPE, false, NW>), dim3(blocks), dim3(64 * NW), 0, st, a);
  return hipGetLastError();
}

template <typename T, int NB, int PMAX, int WPE, int NW>
int wave_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, dmat_wave_kernel<T, NB, PMAX, WPE, true, NW>, 64 * NW, 0) !=
      hipSuccess)
    return 4;
  return n > 0 ? n : 1;
}

// The two variants per form.  FP32: the larger tile (160-bin windows, three
// k_perp rows of 50 bins, in one pass) is split between the two waves of a
// workgroup, each holding half of its accumulator blocks and binning one of
// the two rows of a step, so that two waves fit on a SIMD (one wave holding
// the whole tile in AGPRs, one wave per SIMD, took 6 % longer); the smaller
// tile runs one wave per workgroup, two per SIMD.  FP64: the larger tile runs
// one wave per SIMD (split between two waves it spills registers and took 5 %
// longer), the smaller two.  All are the largest that compile without (or
// with a few bytes of) register spills.
constexpr int kNB32[2] = {10, 8};
constexpr int kNB64[2] = {7, 5};
constexpr int kPMax = 4;    // FP32: 256 pixels of the other forest in registers at a time
constexpr int kPMax64 = 3;  // FP64: 192

}  // namespace

int dmat_wave_num_variants() { return 2; }

int dmat_wave_tile_blocks(int v, int precision) { return precision == LYA_FP64 ? kNB64[v] : kNB32[v]; }

const char* dmat_wave_variant_name(int v) {
  static const char* const names[2] = {"sym-big", "sym-small"};
  return (v >= 0 && v < 2) ? names[v] : "?";
}

hipError_t launch_dmat_wave(int v, int precision, const DmatArgs& a, int blocks, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  if (precision == LYA_FP64)
    return v == 0 ? launch_wave<double, kNB64[0], kPMax64, 1, 1>(a, blocks, st)
                  : launch_wave<double, kNB64[1], kPMax64, 2, 1>(a, blocks, st);
  return v == 0 ? launch_wave<float, kNB32[0], kPMax, 2, 2>(a, blocks, st)
                : launch_wave<float, kNB32[1], kPMax, 2, 1>(a, blocks, st);
}

size_t dmat_wave_hsave_bytes_per_block(int v, int precision, int run) {
  // the large tile keeps them (NB >= 7, per-pass ranges), one copy per wave
  if (v != 0) return 0;
  if (precision == LYA_FP64) return (size_t)1 * run * 2 * kNB64[0] * 64 * sizeof(double);
  return (size_t)2 * run * 2 * kNB32[0] * 64 * sizeof(float);
}

int dmat_wave_blocks_per_cu(int v, int precision) {
  if (precision == LYA_FP64)
    return v == 0 ? wave_occupancy<double, kNB64[0], kPMax64, 1, 1>() : wave_occupancy<double, kNB64[1], kPMax64, 2, 1>();
  return v == 0 ? wave_occupancy<float, kNB32[0], kPMax, 2, 2>() : wave_occupancy<float, kNB32[1], kPMax, 2, 1>();
}

}  // namespace lya
