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
// all pairs of a chunk that share a window accumulate into one tile of D over
// that window (in blocks of TW x TW window bins when the window is wider),
// added to the global FP64 numerator once per chunk.
//
// The row terms are a contraction over rows: for a group of rows r with
// weights -w_r, tile[x][y] += sum_r sum_l (-w_r R^l_r[x]) G^l_r[y], a
// [W x 2n] by [2n x W] product.  It runs on the matrix cores: one 16x16x4
// MFMA step takes two rows for one 16 x 16 block of the tile.  A row only
// touches a few runs of bins, so each row records which blocks its R and G
// reach (one ballot gives every wave's block bits), and a step is issued only
// for the blocks that one of its two rows reaches on both sides; the work
// issued stays close to the sparse row outer products.  The tile's blocks are
// shared by 8 waves (2 per SIMD) as laid out by DLay below; operand addresses
// are per-wave bases plus compile-time offsets.
//
// Within one forest, q = (u, b) = (w / W, w a / S) is p weighted per pixel and
// scaled per forest, so the G histograms of a row are its R histograms times
// (1 / W, 1 / S) of the other forest: only R^0 = sum w and R^1 = sum w a are
// built (over a second range too when the tile's two axes cover different
// window blocks).
//
// The workgroup takes the pairs of a run one at a time.  In each sweep the
// pixels the lanes run over are staged in LDS (in chunks for long forests),
// each wave sweeps RPW rows and builds their histograms in LDS with FP64
// atomics; after a barrier every wave issues the steps of its own blocks.  The
// pair histograms H, Q follow from the sweep-1 rows and their rank-4 product
// is one more step.  The FP64 form accumulates in FP64; the FP32 form in FP32
// over a run (at most a chunk of pairs), which its 1e-5 bound allows; either
// tile is added to the global FP64 numerator once per run, and the Kronecker
// term and w_A are summed in FP64 on the side.  Bins come from the shared
// binner, so a pixel pair falls in the same bin here as in the xi kernel.
#include "lya_bin.h"
#include "lya_common.h"

namespace lya {

namespace {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

constexpr int kBlk = 16;  // MFMA block side
constexpr int kNW = 8;    // waves per workgroup
constexpr int kRPW = 2;   // rows swept per wave per group

// The MFMA of each form.  16x16x4 steps: operand A[i][k] and B[k][j] come from
// lane 16 k + i (resp. 16 k + j).  FP64 form: FP64 accumulators (8 VGPRs per
// block), register r of lane 16 g + j holds row g + 4 r, column j; a tile of
// 10 x 10 blocks.  FP32 form: FP32 accumulators (4 VGPRs per block; the
// products are of FP32 values and a run of pairs sums at most a few thousand
// of them per entry), register r of lane 16 g + j holds row 4 g + r; the same
// registers then hold 14 x 14 blocks, so windows up to 224 bins (four k_perp
// rows of 50 k_par bins) take one pass.
template <typename T> struct DTile;
template <> struct DTile<double> {
  static constexpr int NB = 10, BI = 5, NFC = 2;
  using Acc = mf_d4;
  __device__ __forceinline__ static int row(int g, int r) { return g + 4 * r; }
  __device__ __forceinline__ static Acc mfma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct DTile<float> {
  static constexpr int NB = 14, BI = 7, NFC = 3;
  using Acc = mf_f4;
  __device__ __forceinline__ static int row(int g, int r) { return 4 * g + r; }
  __device__ __forceinline__ static Acc mfma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// Block ownership.  The 8 waves (wx, wy) = (w & 1, w >> 1) share NB x NB blocks:
// wave (wx, wy) owns block rows wx + 2 i (i < BI) of the NFC full block columns
// wy + 4 k, and rows i < SP (wy < 2) or i >= SP (wy >= 2) of the extra column
// 4 NFC + (wy & 1).  Slot j < NF is (row j / NFC, column k = j % NFC); slot
// j >= NF is row j - NF (wy < 2) or j - NF + SP (wy >= 2) of the extra column.
template <typename T> struct DLay {
  static constexpr int NB = DTile<T>::NB, BI = DTile<T>::BI, NFC = DTile<T>::NFC;
  static constexpr int TW = NB * kBlk;                // window bins per tile side
  static constexpr int NF = BI * NFC;                 // slots in full columns
  static constexpr int SP = (BI + 1) / 2;             // extra-column rows of waves wy < 2
  static constexpr int MB = NF + SP;                  // slots per wave (at most)
  static constexpr int BPW = MB <= 16 ? 16 : 32;      // ballot bits per wave
  static constexpr int WPW = 64 / BPW, NWORD = kNW * BPW / 64;
  __host__ __device__ static constexpr int slot_i(int j, bool low) {
    return j < NF ? j / NFC : (low ? j - NF : j - NF + SP);
  }
  __host__ __device__ static constexpr int slot_k(int j) { return j < NF ? j % NFC : NFC; }
  __host__ __device__ static constexpr bool slot_ok(int j, bool low) { return j < MB && slot_i(j, low) < BI; }
  __host__ __device__ static constexpr int col(int wy, int k) { return k < NFC ? wy + 4 * k : 4 * NFC + (wy & 1); }
  __host__ __device__ static constexpr int bx(int wx, bool low, int j) { return wx + 2 * slot_i(j, low); }
  __host__ __device__ static constexpr int by(int wy, int j) { return col(wy, slot_k(j)); }
};

template <int N> struct IC { static constexpr int value = N; };


template <typename T> struct DCfg;
template <> struct DCfg<float> {
  using Rec = DRec32;
  static constexpr int kStage = 1024;  // pixels of the swept forest staged in LDS at a time
};
template <> struct DCfg<double> {
  using Rec = DRec64;
  static constexpr int kStage = 512;
};

template <typename T, int NW>
struct DSmem {
  static constexpr int NR = NW * kRPW;  // rows per group
  static constexpr int S = DCfg<T>::kStage;
  static constexpr int kTileW = DLay<T>::TW;
  T sd[S], sw[S], sa[S];  // staged pixels of the forest the lanes sweep
  // R^0, R^1 of each row of the group over the tile's x range, and over its y
  // range when that differs.  FP64 in both forms: LDS FP64 atomic adds run at
  // about twice the rate of FP32 ones here (measured again with the FP32 form's
  // FP32 steps: FP32 rows make the kernel 12 % slower).
  double rowR[NR][2][kTileW];
  double rowG[NR][2][kTileW];
  T rw[NR];                 // -w of each row (0: no row)
  T rowc[NR][4];            // w, w a, u, b of each sweep-1 row
  uint64_t act[NR][DLay<T>::NWORD];  // block bits of each row: BPW bits per wave
  T H[4][kTileW];           // pair histograms, written after sweep 1
  T Q[4][kTileW];
  double wdacc[kTileW];     // w_A over the run (first column pass)
  double dacc[kTileW];      // the Kronecker term w_A [A = B] of diagonal passes
  int32_t ox[kTileW], oy[kTileW];  // output bin index of each tile row / column
  int32_t rng[4];                  // pixels of f, g within reach of the other forest: [lo, hi]
  uint16_t bal[DLay<T>::NWORD][64];  // (block row | block column << 8) of ballot lane, 31 = none
  unsigned long long nalg;         // outer-product FMAs counted (statistics)
  int64_t item;
};

// OR of an NB-bit mask over the wave, one ballot per bit (no LDS round trips).
template <int NB>
__device__ __forceinline__ uint32_t wave_or_blocks(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int b = 0; b < NB; ++b) r |= (__ballot((v >> b) & 1u) != 0ull) ? (1u << b) : 0u;
  return r;
}

__device__ __forceinline__ float lane_val(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_val(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <typename T, int BLOCK, bool ZLO>
__global__ __launch_bounds__(BLOCK) void dmat_kernel(DmatArgs a) {
  using Cfg = DCfg<T>;
  using Rec = typename Cfg::Rec;
  using Lay = DLay<T>;
  using Tile = DTile<T>;
  using Acc = typename Tile::Acc;
  constexpr int NW = BLOCK / 64, S = Cfg::kStage, TW = Lay::TW;
  constexpr int RPW = kRPW, NR = NW * RPW;
  constexpr int BPW = Lay::BPW, WPW = Lay::WPW, NWORD = Lay::NWORD;
  constexpr int BI = Lay::BI, NF = Lay::NF, NFC = Lay::NFC, SP = Lay::SP, MB = Lay::MB;
  constexpr bool kF32 = sizeof(T) == 4;
  static_assert(NW == kNW && MB <= BPW && MB < 32, "wave layout");
  static_assert(NR % 2 == 0, "two rows per MFMA step");
  __shared__ DSmem<T, NW> sm;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lk = lane >> 4, lm = lane & 15;  // MFMA operand coordinates: k, and row/column in the block
  const int wx = wave & 1, wy = wave >> 1;
  const bool low = wy < 2;  // which block rows of the third column the wave owns

  BinK<T, ZLO> K;
  K.init(a.g, a.glob, a.edges_par, a.edges_perp);
  const int NP = K.NP, NT = K.NT, nb = NP * NT;
  const Rec* __restrict__ recs;
  if constexpr (kF32) recs = a.drec32; else recs = a.drec64;

  // (wave, slot) of each lane in the row activity ballots: word h covers waves
  // WPW h .. WPW h + WPW - 1 (a table in LDS rather than registers)
  for (int e = tid; e < NWORD * 64; e += BLOCK) {
    const int h = e >> 6, l = e & 63;
    const int W = WPW * h + l / BPW, j = l % BPW;
    const bool lw = (W >> 1) < 2;
    const bool ok = Lay::slot_ok(j, lw);
    sm.bal[h][l] = ok ? (uint16_t)(Lay::bx(W & 1, lw, j) | (Lay::by(W >> 1, j) << 8)) : (uint16_t)(31 | (31 << 8));
  }
  if (tid == 0) sm.nalg = 0;

  for (int e = tid; e < NR * 2 * TW; e += BLOCK) {
    (&sm.rowR[0][0][0])[e] = 0;
    (&sm.rowG[0][0][0])[e] = 0;
  }
  unsigned n_in = 0, n_lost = 0;  // statistics only
  Acc cacc[MB];  // MFMA accumulators of the wave's blocks

  for (;;) {
    __syncthreads();  // every thread has read the previous item
    if (tid == 0) sm.item = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t it = sm.item;
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
      const int64_t r1 = lo;
      if (key == ~0ull) {
        r0 = r1;
        continue;
      }
      const int real = dmat_key_real(key);
      const int kt0 = dmat_key_kt0(key);
      const int span = dmat_key_span(key);
      const int nwin = span * NP;
      const int base_L = kt0 * NP;  // window index w = L - kt0 NP
      const int npass = (nwin + TW - 1) / TW;
      const int64_t obase = (int64_t)real * nb;

      for (int ab = 0; ab < npass; ++ab) {
        const int a0 = ab * TW, na = min(TW, nwin - a0);
        for (int bb = 0; bb < npass; ++bb) {
          const int b0 = bb * TW, nbk = min(TW, nwin - b0);
          const bool first_pass = ab == 0 && bb == 0;
          const int nbx = (na + kBlk - 1) / kBlk, nby = (nbk + kBlk - 1) / kBlk;
          const bool diag = a0 == b0;  // both axes cover the same window bins
#pragma unroll
          for (int j = 0; j < MB; ++j) cacc[j] = Acc{0, 0, 0, 0};
          __syncthreads();  // the previous pass's flush has read the index tables
          for (int x = tid; x < TW; x += BLOCK) {
            sm.wdacc[x] = 0.0;
            sm.dacc[x] = 0.0;
            sm.ox[x] = x < na ? out_index(a0 + x + base_L, NP, NT) : -1;
            sm.oy[x] = x < nbk ? out_index(b0 + x + base_L, NP, NT) : -1;
          }

          for (int64_t kk = r0; kk < r1; ++kk) {
            const int q = a.worder[kk];
            int64_t pf, pg;
            int nf, ng;
            double s64, c64;
            double fdmin, fdmax, gdmin, gdmax;
            {
              const ForestInfo fi = a.finfo[a.sorted[a.pair_p[q]]];
              const ForestInfo gi = a.finfo[a.sorted[a.nbr[q]]];
              pair_sc(fi, gi, s64, c64);
              pf = fi.pix0;
              pg = gi.pix0;
              nf = fi.npix;
              ng = gi.npix;
              fdmin = fi.dmin;
              fdmax = fi.dmax;
              gdmin = gi.dmin;
              gdmax = gi.dmax;
            }
            // Only pixels within reach of the other forest's extent can pair in the
            // grid: r_par = |D_i - D_j| c >= e_par_max once |D_i - D_j| >= reach (the
            // margin covers the rounding of the FP64 separations).  The first and
            // last such pixel of each forest bound the rows and lanes of the sweeps.
            __syncthreads();  // the previous pair's ranges have been read
            if (tid < 4) sm.rng[tid] = (tid & 1) ? -1 : 0x7fffffff;
            __syncthreads();
            {
              const double reach = a.g.emax_par / c64 * (1.0 + 1e-12) + 1e-9;
#pragma unroll
              for (int side = 0; side < 2; ++side) {
                const int n = side ? ng : nf;
                const int64_t p0 = side ? pg : pf;
                const double lo = (side ? fdmin : gdmin) - reach, hi = (side ? fdmax : gdmax) + reach;
                for (int e0 = wave * 64; e0 < n; e0 += BLOCK) {
                  const int e = e0 + lane;
                  bool in = false;
                  if (e < n) {
                    double D;
                    if constexpr (kF32) D = recs[p0 + e].D; else D = recs[p0 + e].d;
                    in = D > lo && D < hi;
                  }
                  const uint64_t m = __ballot(in);
                  if (m != 0ull && lane == 0) {
                    atomicMin(&sm.rng[2 * side], e0 + __ffsll((long long)m) - 1);
                    atomicMax(&sm.rng[2 * side + 1], e0 + 63 - __clzll((long long)m));
                  }
                }
              }
            }
            __syncthreads();
            const int f_lo = sm.rng[0], f_n = sm.rng[1] + 1 - sm.rng[0];
            const int g_lo = sm.rng[2], g_n = sm.rng[3] + 1 - sm.rng[2];
            if (f_n <= 0 || g_n <= 0) continue;  // no pixel pair of these forests is in the grid
            // G = R (1 / W, 1 / S) of the forest the lanes sweep (0 where the term is off)
            double gsc[2][2];
            {
              const EtaInfo ef = a.einfo[a.sorted[a.pair_p[q]]];
              const EtaInfo eg = a.einfo[a.sorted[a.nbr[q]]];
              gsc[0][0] = ef.active ? 1.0 / ef.W : 0.0;
              gsc[0][1] = ef.slope ? 1.0 / ef.S : 0.0;
              gsc[1][0] = eg.active ? 1.0 / eg.W : 0.0;
              gsc[1][1] = eg.slope ? 1.0 / eg.S : 0.0;
            }
            const T s = (T)s64, c = (T)c64;
            const T bsep = kF32 ? (T)(2.0 * a.glob->dc * s64) : (T)0;
            // sweep-1 rows give the pair histograms H^{kl}[x], Q^{kl}[x] (kl = 2k + l),
            // kept in registers: with 8 waves, thread tid - (BLOCK - 2 TW) (the last
            // waves, which own fewer tile blocks) keeps H (< TW) or Q of one x; with
            // 4 waves, thread tid < TW keeps both for x = tid
            constexpr bool kHQsplit = BLOCK >= 2 * TW;
            const int hq_t = kHQsplit ? tid - (BLOCK - 2 * TW) : tid;
            const bool hq_on = hq_t >= 0 && hq_t < (kHQsplit ? 2 * TW : TW);
            const bool hq_q = kHQsplit && hq_t >= TW;
            const int hq_x = hq_q ? hq_t - TW : hq_t;
            T hq0 = 0, hq1 = 0, hq2 = 0, hq3 = 0;
            T qq0 = 0, qq1 = 0, qq2 = 0, qq3 = 0;  // Q when not split

            // one sweep: rows of side RS, lanes over the pixels of the other side,
            // which are staged in LDS S at a time
            auto sweep = [&](auto rs_tag) {
              constexpr int RS = decltype(rs_tag)::value;
              const int nr = RS ? g_n : f_n, no = RS ? f_n : g_n;
              const int64_t prow0 = RS ? pg + g_lo : pf + f_lo, poth0 = RS ? pf + f_lo : pg + g_lo;
              const int nchunk = (no + S - 1) / S;
              auto stage = [&](int c0) {
                __syncthreads();
                for (int e = tid; e < min(S, no - c0); e += BLOCK) {
                  const Rec r = recs[poth0 + c0 + e];
                  sm.sd[e] = r.d;
                  sm.sw[e] = r.w;
                  sm.sa[e] = r.a;
                }
                __syncthreads();
              };
              if (nchunk == 1) stage(0);
              // lane qq < RPW of each wave holds the record of the wave's row qq of
              // the next group (loaded one group ahead)
              T pd = 0, pw = 0, pa = 0, pu = 0, pb = 0;
              auto fetch = [&](int gn) {
                const int row = gn + wave * RPW + lane;
                if (lane < RPW && row < nr) {
                  const Rec r = recs[prow0 + row];
                  pd = r.d; pw = r.w; pa = r.a; pu = r.u; pb = r.b;
                }
              };
              fetch(0);
              for (int g0 = 0; g0 < nr; g0 += NR) {
                // the group's row factors go to LDS right away (the previous group's
                // readers finished before the barrier that preceded its clearing)
                if (lane < RPW) {
                  const int slot = wave * RPW + lane;
                  const bool ok = g0 + slot < nr;
                  sm.rw[slot] = ok ? -pw : (T)0;
                  sm.rowc[slot][0] = ok ? pw : (T)0;
                  sm.rowc[slot][1] = ok ? pw * pa : (T)0;
                  sm.rowc[slot][2] = ok ? pu : (T)0;
                  sm.rowc[slot][3] = ok ? pb : (T)0;
                }
                T gd[RPW];
#pragma unroll
                for (int qq = 0; qq < RPW; ++qq) gd[qq] = lane_val(pd, qq);
                if (g0 + NR < nr) fetch(g0 + NR);
                uint32_t bx[RPW], by[RPW];
#pragma unroll
                for (int qq = 0; qq < RPW; ++qq) bx[qq] = by[qq] = 0;
                for (int ch = 0; ch < nchunk; ++ch) {
                  const int c0 = ch * S, cn = min(S, no - c0);
                  if (nchunk > 1) stage(c0);
                  // a lane takes every niter-th pixel, so the 64 pixels of one pass are
                  // spread over the forest and mostly fall in different bins; each pixel
                  // is paired with all RPW rows of the wave
                  const int niter = (cn + 63) >> 6;
                  for (int it = 0; it < niter; ++it) {
                    const int j = it + niter * lane;
                    if (j >= cn) continue;
                    const T od = sm.sd[j], ow = sm.sw[j], oa = sm.sa[j];
                    const T owa = ow * oa;
#pragma unroll
                    for (int qq = 0; qq < RPW; ++qq) {
                      const int slot = wave * RPW + qq;
                      if (g0 + slot >= nr) continue;
                      const T rd = gd[qq];
                      T rp, rt;
                      separations(rd, od, c, s, bsep, rp, rt);
                      if (!K.may_be_in(rp, rt)) continue;
                      const int L = K.bin_near(rp, rt, [&](double& rp64, double& rt64) {
                        if constexpr (kF32) {
                          separations64(recs[prow0 + g0 + slot].D, recs[poth0 + c0 + j].D, c64, s64, rp64, rt64);
                        } else {
                          rp64 = rp;
                          rt64 = rt;
                        }
                      });
                      if (L < 0) continue;
                      const int w = L - base_L;
                      if ((unsigned)w >= (unsigned)nwin) {
                        ++n_lost;
                        continue;
                      }
                      if (RS == 0 && first_pass) ++n_in;
                      const int x = w - a0, y = w - b0;
                      if ((unsigned)x < (unsigned)na) {
                        atomicAdd(&sm.rowR[slot][0][x], (double)ow);
                        atomicAdd(&sm.rowR[slot][1][x], (double)owa);
                        bx[qq] |= 1u << (x >> 4);
                      }
                      if (!diag && (unsigned)y < (unsigned)nbk) {
                        atomicAdd(&sm.rowG[slot][0][y], (double)ow);
                        atomicAdd(&sm.rowG[slot][1][y], (double)owa);
                        by[qq] |= 1u << (y >> 4);
                      }
                    }
                  }
                }
#pragma unroll
                for (int qq = 0; qq < RPW; ++qq) {
                  const int slot = wave * RPW + qq;
                  const uint32_t bxq = wave_or_blocks<Lay::NB>(bx[qq]);
                  const uint32_t byq = diag ? bxq : wave_or_blocks<Lay::NB>(by[qq]);
                  // block bits of every wave for this row
#pragma unroll
                  for (int h = 0; h < NWORD; ++h) {
                    const unsigned bl = sm.bal[h][lane];
                    const uint64_t wb = __ballot(((bxq >> (bl & 0xffu)) & (byq >> (bl >> 8)) & 1u) != 0u);
                    if (lane == 0) sm.act[slot][h] = wb;
                  }
                }
                __syncthreads();

                // MFMA steps on the wave's blocks, rows (2 st, 2 st + 1) per step
                {
                  const int slot_l = lk >> 1, comp = lk & 1;
                  const double* pa = &sm.rowR[slot_l][comp][wx * kBlk + lm];
                  const double* pb = diag ? &sm.rowR[slot_l][comp][wy * kBlk + lm] : &sm.rowG[slot_l][comp][wy * kBlk + lm];
                  const int cx = (4 * NFC + (wy & 1) - wy) * kBlk;  // extra column, relative to pb
                  const double gs = gsc[1 - RS][comp];
#pragma unroll 1
                  for (int st = 0; st < NR / 2; ++st) {
                    const uint32_t bits = __builtin_amdgcn_readfirstlane(
                        (uint32_t)((sm.act[2 * st][wave / WPW] | sm.act[2 * st + 1][wave / WPW]) >>
                                   (BPW * (wave % WPW))) &
                        ((1u << MB) - 1u));
                    if (bits == 0u) continue;
                    const int so = 2 * st * 2 * TW;  // two rows further per step
                    // A[x][k] B[k][y] = (-w_r R[x]) (g_l R[y]): both factors of the
                    // row and component k go on the A side
                    const double fa = (double)sm.rw[2 * st + slot_l] * gs;
                    T av[BI], bv[NFC + 1];
#pragma unroll
                    for (int i = 0; i < BI; ++i) av[i] = (T)(fa * pa[so + 2 * kBlk * i]);
#pragma unroll
                    for (int k = 0; k < NFC; ++k) bv[k] = (T)pb[so + 4 * kBlk * k];
                    bv[NFC] = (T)pb[so + cx];
#pragma unroll
                    for (int j = 0; j < MB; ++j)
                      if ((bits >> j) & 1u) {
                        const T aj = j < NF ? av[j / NFC] : (low ? av[j - NF] : av[j - NF + SP < BI ? j - NF + SP : BI - 1]);
                        cacc[j] = Tile::mfma(aj, bv[Lay::slot_k(j)], cacc[j]);
                      }
                  }
                }
                if (RS == 0 && hq_on) {
                  const double* hv = (hq_q && !diag) ? &sm.rowG[0][0][hq_x] : &sm.rowR[0][0][hq_x];
                  const int ck = hq_q ? 2 : 0;
#pragma unroll
                  for (int r = 0; r < NR; ++r) {
                    const T v0 = (T)hv[r * 2 * TW], v1 = (T)hv[r * 2 * TW + TW];
                    const T c0 = sm.rowc[r][ck], c1 = sm.rowc[r][ck + 1];
                    hq0 = fma(c0, v0, hq0);
                    hq1 = fma(c0, v1, hq1);
                    hq2 = fma(c1, v0, hq2);
                    hq3 = fma(c1, v1, hq3);
                    if constexpr (!kHQsplit) {
                      const double* gv = diag ? &sm.rowR[r][0][hq_x] : &sm.rowG[r][0][hq_x];
                      const T g0 = (T)gv[0], g1 = (T)gv[TW];
                      const T d0 = sm.rowc[r][2], d1 = sm.rowc[r][3];
                      qq0 = fma(d0, g0, qq0);
                      qq1 = fma(d0, g1, qq1);
                      qq2 = fma(d1, g0, qq2);
                      qq3 = fma(d1, g1, qq3);
                    }
                  }
                }
                __syncthreads();
                // clear the wave's rows; count the sparse outer-product work (statistics)
#pragma unroll
                for (int qq = 0; qq < RPW; ++qq) {
                  const int slot = wave * RPW + qq;
                  int cx = 0, cy = 0;
                  for (int x = lane; x < TW; x += 64) {
                    if (a.counters) {
                      cx += __popcll(__ballot((sm.rowR[slot][0][x] != 0.0) | (sm.rowR[slot][1][x] != 0.0)));
                      if (!diag) cy += __popcll(__ballot((sm.rowG[slot][0][x] != 0.0) | (sm.rowG[slot][1][x] != 0.0)));
                    }
                    sm.rowR[slot][0][x] = sm.rowR[slot][1][x] = 0;
                    sm.rowG[slot][0][x] = sm.rowG[slot][1][x] = 0;
                  }
                  if (diag) cy = cx;
                  if (a.counters && lane == 0) atomicAdd(&sm.nalg, 2ull * (unsigned long long)cx * (unsigned long long)cy);
                }
              }
            };

            // ---- sweep 1: rows i of f
            sweep(IC<0>{});
            if (hq_on) {
              // Q^{kl} = (1 / W_g, 1 / S_g)_l sum_r (u_r, b_r)_k R^l_r
              const T s0 = (T)gsc[1][0], s1 = (T)gsc[1][1];
              if (hq_q) {
                sm.Q[0][hq_x] = hq0 * s0;
                sm.Q[1][hq_x] = hq1 * s1;
                sm.Q[2][hq_x] = hq2 * s0;
                sm.Q[3][hq_x] = hq3 * s1;
              } else {
                sm.H[0][hq_x] = hq0;
                sm.H[1][hq_x] = hq1;
                sm.H[2][hq_x] = hq2;
                sm.H[3][hq_x] = hq3;
              }
              if constexpr (!kHQsplit) {
                sm.Q[0][hq_x] = qq0 * s0;
                sm.Q[1][hq_x] = qq1 * s1;
                sm.Q[2][hq_x] = qq2 * s0;
                sm.Q[3][hq_x] = qq3 * s1;
              }
            }
            __syncthreads();
            // ---- H (x) Q: one more step; the Kronecker term on the diagonal; w_A
            {
              T av[BI], bv[NFC + 1];
#pragma unroll
              for (int i = 0; i < BI; ++i) av[i] = sm.H[lk][(wx + 2 * i) * kBlk + lm];
#pragma unroll
              for (int k = 0; k <= NFC; ++k) bv[k] = sm.Q[lk][Lay::col(wy, k) * kBlk + lm];
#pragma unroll
              for (int j = 0; j < MB; ++j) {
                const int bx = Lay::bx(wx, low, j), by = Lay::by(wy, j);
                if (Lay::slot_ok(j, low) && bx < nbx && by < nby) {
                  const T aj = j < NF ? av[j / NFC] : (low ? av[j - NF] : av[j - NF + SP < BI ? j - NF + SP : BI - 1]);
                  cacc[j] = Tile::mfma(aj, bv[Lay::slot_k(j)], cacc[j]);
                }
              }
            }
            if (a.counters && wave == 0) {
              int hx = 0, qy = 0;
              for (int x = lane; x < TW; x += 64) {
                hx += __popcll(__ballot(x < na && sm.H[0][x] != (T)0));
                qy += __popcll(__ballot(x < nbk && ((sm.Q[0][x] != (T)0) | (sm.Q[3][x] != (T)0))));
              }
              if (lane == 0) atomicAdd(&sm.nalg, 4ull * (unsigned long long)hx * (unsigned long long)qy);
            }
            for (int x = tid; x < na; x += BLOCK) {
              if (bb == 0) sm.wdacc[x] += (double)sm.H[0][x];
              if (a0 == b0) sm.dacc[x] += (double)sm.H[0][x];
            }

            // ---- sweep 2: rows j of g
            sweep(IC<1>{});
          }
          __syncthreads();

          // ---- add the wave's blocks to the global numerator (and w_A)
#pragma unroll
          for (int j = 0; j < MB; ++j) {
            const int bx = Lay::bx(wx, low, j), by = Lay::by(wy, j);
            if (Lay::slot_ok(j, low) && bx < nbx && by < nby) {
              const int oy = sm.oy[by * kBlk + lm];
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int ox = sm.ox[bx * kBlk + Tile::row(lk, r)];
                const double v = (double)cacc[j][r];
                if (ox >= 0 && oy >= 0 && v != 0.0) atomicAdd(&a.dnum[(obase + ox) * nb + oy], v);
              }
            }
          }
          // the Kronecker term w_A [A = B] on the diagonal of diagonal passes, and w_A
          for (int x = tid; x < na; x += BLOCK) {
            const int ox = sm.ox[x];
            if (a0 == b0 && sm.dacc[x] != 0.0) atomicAdd(&a.dnum[(obase + ox) * nb + ox], sm.dacc[x]);
            if (bb == 0 && sm.wdacc[x] != 0.0) atomicAdd(&a.wd[obase + ox], sm.wdacc[x]);
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
      atomicAdd(&a.counters[2], nl);
    }
    __syncthreads();
    if (tid == 0) atomicAdd(&a.counters[1], sm.nalg);
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
      key = dmat_window_key(hi - lo + 1, fi.real, lo);
  }
  keys[q] = key;
  idx[q] = (int32_t)q;
}

__global__ void dmat_span_split_kernel(const uint64_t* keys, int64_t n, int max_span, int64_t* out) {
  const uint64_t bound = dmat_window_key(max_span, 0, 0);
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (keys[m] < bound) lo = m + 1; else hi = m;
  }
  *out = lo;
}

constexpr int kNumVariants = 1;
const char* const kNames[kNumVariants] = {"b512-mfma"};

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

// variants: this file's kernel, then the one- and two-wave kernels (k_dmat_wave.hip)
int dmat_num_variants() { return kNumVariants + dmat_wave_num_variants(); }
const char* dmat_variant_name(int v) {
  if (v >= kNumVariants) return dmat_wave_variant_name(v - kNumVariants);
  return v >= 0 ? kNames[v] : "?";
}

hipError_t launch_dmat_span_split(const uint64_t* keys, int64_t n, int max_span, int64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(dmat_span_split_kernel, dim3(1), dim3(1), 0, st, keys, n, max_span, out);
  return hipGetLastError();
}

hipError_t launch_dmat_keys(const DmatArgs& a, uint64_t* keys, int32_t* idx, hipStream_t st) {
  if (a.n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(dmat_keys_kernel, dim3((unsigned)((a.n_pairs + 255) / 256)), dim3(256), 0, st, a, keys, idx);
  return hipGetLastError();
}

hipError_t launch_dmat(int variant, int precision, const DmatArgs& a, int blocks, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  if (variant >= kNumVariants) return launch_dmat_wave(variant - kNumVariants, precision, a, blocks, st);
  return precision == LYA_FP64 ? launch_one<double, 512>(a, blocks, st) : launch_one<float, 512>(a, blocks, st);
}

int dmat_blocks_per_cu(int variant, int precision) {
  if (variant >= kNumVariants) return dmat_wave_blocks_per_cu(variant - kNumVariants, precision);
  return precision == LYA_FP64 ? occupancy<double, 512>() : occupancy<float, 512>();
}

size_t dmat_hsave_bytes_per_block(int variant, int precision, int run) {
  return variant >= kNumVariants ? dmat_wave_hsave_bytes_per_block(variant - kNumVariants, precision, run) : 0;
}

hipError_t launch_finalize_dmat(double* d, const double* wd, int64_t n_rows, int nb, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_dmat_kernel, dim3((unsigned)n_rows), dim3(256), 0, st, d, wd, n_rows, nb);
  return hipGetLastError();
}

}  // namespace lya
