// gwf_fisher_body.hpp -- the per-workgroup Fisher accumulation shared by the
// one-event-per-workgroup kernel and the batched work-item kernel.
//
// A workgroup of kBlock lanes sums the contributions of grid points
// [k0, k1) of one event: each lane takes points k0 + tid + kBlock*it,
// evaluates the derivative vectors of all interferometers at that point in
// registers and adds its share of the 8x8 block of (Mc, eta, dL, theta, phi,
// iota, psi, tc) to its kGramAcc register accumulators (the 5x5 block of the
// rows that are not pattern combinations, plus pattern moments; see
// accumulate_point).  The phase-only blocks Gamma_{b, 8+i} = sum U_b c_i and
// Gamma_{8+i, 8+j} = sum W c_i c_j split in two:
//   * the Phic column (c_0 = -1 at every point) needs only sums of U_b and of
//     W c_i; those of U_b and W are combinations of the pattern moments the
//     lanes already hold (U_b = c+ T_b,1 - cx T_b,2, U_dL = 0, U_iota and
//     U_psi and W from S), so a lane adds up only W c_i (i >= 1);
//   * the rest is a small dense contraction over frequency, X = sum_f a_f c_f^T
//     with a_f = (U_0, U_1, U_3, U_4, U_5, U_6, U_7, W c_1 .. W c_{NPI-1}) and
//     c_f = (c_1 .. c_{NPI-1}): every iteration each wavefront stages its 64
//     points' a_f and c_f in LDS and folds them into 4x4 output tiles of X
//     with the four-block FP64 MFMA 4x4x4 (k = frequency).  With tides
//     (NPI = 5) the 11 x 4 block fits three tiles, one MFMA per four points
//     (a fourth tile slot idle); with e0 as well six tiles, two MFMAs.
// The sums are then reduced in a fixed order (wavefront butterflies, then
// the waves in index order), so results are bitwise reproducible.
#pragma once

#include "gwf_kernels.hpp"

namespace gwf {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kRowsA = 16;        // 7 U rows, up to 5 W c rows, zero rows to a whole tile
constexpr int kRowsB = 8;         // up to 5 c rows, zero rows to a whole tile
constexpr int kZeroRowB = 7;      // a B row no point writes (operand of unused tile slots)
constexpr int kZeroRowA = 15;
// Row stride of the staged operands, in doubles.  The lanes of an MFMA
// operand read take rows 4 t + i (up to 16 rows: t the tile slot, i = 0..3)
// at points 4 s + k, and row r starts on four-byte bank 2 r LD mod 64.  With
// LD odd, r LD mod 32 differs for all 16 rows (an odd factor permutes the
// residues), so the rows of a read, and of the paired reads the compiler
// forms, fall on distinct banks.  Measured on the BNS catalogue: strides 68
// and 66 left 3.9e8 and 9.9e7 bank-conflict cycles per launch, 65 and 67 none
// (67 the fastest).
constexpr int kTileLd = 67;
constexpr int kNaccMax = 105;    // 36 + 8 NPI + NPI (NPI + 1)/2 at NPI = 6
constexpr int kURow[7] = {0, 1, 3, 4, 5, 6, 7};   // the U rows staged (U_dL = 0)

template <int NPI_>
struct FisherDims {
  static constexpr int NPI = NPI_;                   // phase-only parameters
  static constexpr bool TIDAL = NPI >= 5;
  static constexpr int P = 8 + NPI;
  static constexpr int NG = 36, NX = 8 * NPI, NY = NPI * (NPI + 1) / 2;
  static constexpr int NACC = NG + NX + NY;          // SNR^2 = Gamma_{Phic,Phic}
  // the staged contraction: NA rows of a_f (7 U rows, then W c_i for
  // i = 1..NPI-1), NB columns c_1..c_{NPI-1}; its 4x4 output tiles are those
  // holding a U row or an element of the upper triangle of W c_i c_j
  static constexpr int NA = 6 + NPI, NB = NPI - 1;
  static constexpr int RG = (NA + 3) / 4, CG = (NB + 3) / 4;
  __host__ __device__ static constexpr bool tile_used(int r, int c) {
    return 4 * r < 7 || 4 * c + 3 >= (4 * r > 7 ? 4 * r : 7) - 7;
  }
  __host__ __device__ static constexpr int count_tiles() {
    int n = 0;
    for (int r = 0; r < RG; ++r)
      for (int c = 0; c < CG; ++c) n += tile_used(r, c) ? 1 : 0;
    return n;
  }
  static constexpr int NT = count_tiles();
  static constexpr int NM = (NT + 3) / 4;            // MFMA accumulators (4 tiles each)
  // row group and column group of the t-th used tile (row-major order)
  __host__ __device__ static constexpr int tile_rc(int t, bool col) {
    for (int r = 0; r < RG; ++r)
      for (int c = 0; c < CG; ++c)
        if (tile_used(r, c) && t-- == 0) return col ? c : r;
    return 0;
  }
  __host__ __device__ static constexpr int tile_r(int t) { return tile_rc(t, false); }
  __host__ __device__ static constexpr int tile_c(int t) { return tile_rc(t, true); }
};
static_assert(FisherDims<5>::NM == 1 && FisherDims<3>::NM == 1 && FisherDims<4>::NM == 1 &&
              FisherDims<6>::NM == 2, "tile counts");

// LDS working set of one workgroup.
struct FisherLds {
  double red[kWaves][kNaccMax];
  double stA[kWaves][kRowsA][kTileLd];   // staged a_f, [row][point]
  double stB[kWaves][kRowsB][kTileLd];   // staged c_f
};

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Load an event's inputs: the 13 parameters (missing tidal rows read as
// zero), e0 and its reference frequency (zero without eccentricity; a NULL
// f_ref array means the grid's first frequency).
__device__ inline void load_par(const double* __restrict__ par, int64_t ld, int64_t e, bool tidal,
                                const double* ecc, const double* fref, double p[kNparIn]) {
  for (int r = 0; r < 13; ++r) p[r] = (r < 11 || tidal) ? par[r * ld + e] : 0.0;
  p[13] = ecc ? ecc[e] : 0.0;
  p[14] = fref ? fref[e] : 0.0;
}

// Sums of points [k0, k1) of the event whose constants are ec/sc.  On
// return (after a workgroup barrier), lane t < NACC holds accumulator slot t
// (see slot_position) in *tot.
template <int NPI_, bool ROT, bool MIXED = false, bool PSUM = true, bool EXPL = false, bool TAB = true>
__device__ inline void fisher_sums(const EventC& ec, const SiteC* sc, int n_site, int k0, int k1,
                                   FisherLds& L, double* tot) {
  using Dm = FisherDims<NPI_>;
  constexpr int NPI = Dm::NPI, NG = Dm::NG, NX = Dm::NX, NACC = Dm::NACC;
  const int tid = threadIdx.x;
  double G[kGramAcc];
#pragma unroll
  for (int i = 0; i < kGramAcc; ++i) G[i] = 0.0;
  // The 16 MFMAs of an iteration alternate between two independent chains
  // per accumulator (summed once at the end), so consecutive MFMAs do not wait
  // for each other's results.  Every instantiation sums in the same order, so
  // a tile holds the same bits whichever tile slot it occupies (e0 = 0 gives
  // the circular matrix exactly).
  constexpr int NC = 2;
  double acc[Dm::NM][NC];
  const int wave = tid >> 6, lane = tid & 63;
  // four-block MFMA 4x4x4 operand layout: lane 16 k + 4 q + i holds A[q][i][k]
  // and B[q][k][i]; the result D[q][i][j] is in lane 16 i + 4 q + j.  Block q
  // of accumulator m is tile 4 m + q; unused slots read zero rows.
  const int kk = lane >> 4, q4 = (lane >> 2) & 3, i4 = lane & 3;
  int arow[Dm::NM], bcol[Dm::NM];
#pragma unroll
  for (int m = 0; m < Dm::NM; ++m) {
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[m][c] = 0.0;
    const int t = 4 * m + q4;
    arow[m] = t < Dm::NT ? 4 * Dm::tile_r(t) + i4 : kZeroRowA;
    bcol[m] = t < Dm::NT ? 4 * Dm::tile_c(t) + i4 : kZeroRowB;
  }
  double(*A)[kTileLd] = L.stA[wave];
  double(*B)[kTileLd] = L.stB[wave];
  // rows no point ever writes stay zero
#pragma unroll
  for (int r = Dm::NA; r < kRowsA; ++r) A[r][lane] = 0.0;
#pragma unroll
  for (int r = Dm::NB; r < kRowsB; ++r) B[r][lane] = 0.0;
  double wc[NPI - 1];                      // this lane's sums of W c_i, i >= 1
#pragma unroll
  for (int i = 0; i < NPI - 1; ++i) wc[i] = 0.0;

  const int iters = (k1 - k0 + kBlock - 1) / kBlock;   // same trip count for every lane
  const int full = (k1 - k0) / kBlock;                  // iterations with every lane in range
  // on a log grid, v, 1/v and v^-12.42 walk from point to point (GridWalk)
  GridWalk gw;
  if (!EXPL) gw.start(ec, k0 + tid, kBlock);
  // One iteration: every lane's point, then the wavefront's MFMA phase.  The
  // iterations whose points are all in range run without the range test
  // (and without zeroing the point's outputs for lanes past the end); the
  // last, partial one, if any, runs with it.
  auto iteration = [&](int it, bool guard) {
    // The per-event constants are re-read every iteration (uniform reads);
    // hoisting them out of the loop would need more registers than a lane has.
    __asm__ volatile("" ::: "memory");
    const int k = k0 + it * kBlock + tid;
    double U[8], W, cph[NPI];
    if (guard) {
      W = 0.0;
#pragma unroll
      for (int b = 0; b < 8; ++b) U[b] = 0.0;
#pragma unroll
      for (int i = 0; i < NPI; ++i) cph[i] = 0.0;
    }
    if (!guard || k < k1)
      accumulate_point<NPI, ROT, MIXED, PSUM, EXPL, TAB>(ec, sc, n_site, k, G, U, W, cph,
                                                         EXPL ? nullptr : gw.val);
    if (!EXPL) gw.step();
    // stage this point's row (points past the range contribute zeros)
#pragma unroll
    for (int r = 0; r < 7; ++r) A[r][lane] = U[kURow[r]];
#pragma unroll
    for (int i = 1; i < NPI; ++i) {
      const double x = W * cph[i];
      wc[i - 1] += x;
      A[6 + i][lane] = x;
      B[i - 1][lane] = cph[i];
    }
    __builtin_amdgcn_wave_barrier();
    // The LDS-fed MFMA phase runs at raised issue priority, so it drains
    // quickly while the SIMD's other wave keeps the VALU busy.
    __builtin_amdgcn_s_setprio(1);
    // X += A^T B over this wavefront's 64 points, four points per step
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) {
#pragma unroll
      for (int m = 0; m < Dm::NM; ++m) {
        const double av = A[arow[m]][4 * s2 + kk];
        const double bv = B[bcol[m]][4 * s2 + kk];
        acc[m][s2 % NC] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bv, acc[m][s2 % NC], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_wave_barrier();
  };
  for (int it = 0; it < full; ++it) iteration(it, false);
  if (full < iters) iteration(full, true);

  // ---- deterministic reduction: wavefront butterflies, then the waves in order
  // The 8x8 block (NG values) and the Phic column (7 + NPI values: -sum U_b
  // from the pattern moments for the rows Mc, eta, theta, phi, tc, iota, psi,
  // then Gamma_{Phic,Phic} = sum W and Gamma_{Phic, 8+j} = -sum W c_j).
  constexpr int NR = NG + 7 + NPI;
  double rv[NR];
  gram_finish(ec, G, rv);
  {
    const AmpFactors am = amp_factors(ec);
    double* xc = rv + NG;
#pragma unroll
    for (int a = 0; a < 5; ++a)
      xc[a] = fma(am.ccross, G[17 + 4 * a], -am.cplus * G[16 + 4 * a]);   // rows Mc, eta, theta, phi, tc
    xc[5] = -(am.cplus * am.dcx - am.ccross * am.dcp) * G[36];               // iota
    xc[6] = 2.0 * am.cplus * am.ccross * (G[35] + G[37]);                    // psi
    xc[7] = fma(am.cplus * am.cplus, G[35], am.ccross * am.ccross * G[37]);   // Phic, Phic
#pragma unroll
    for (int i = 1; i < NPI; ++i) xc[7 + i] = -wc[i - 1];
  }
  // Each value is summed over the wavefront as wave_sum does (the same
  // additions in the same order), but step by step over all NR values, so
  // that a step's cross-lane reads are in flight together rather than one
  // value's six dependent exchanges after another's.
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int i = 0; i < NR; ++i) rv[i] += __shfl_xor(rv[i], off, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NG; ++i) L.red[wave][i] = rv[i];
    constexpr int rowof[5] = {0, 1, 3, 4, 7};
#pragma unroll
    for (int x = 0; x < 7 + NPI; ++x) {
      int slot;
      if (x < 5) slot = NG + rowof[x] * NPI;
      else if (x == 5) slot = NG + 5 * NPI;
      else if (x == 6) slot = NG + 6 * NPI;
      else slot = NG + NX + (x - 7);                 // row Phic: (8, 8 + x - 7)
      L.red[wave][slot] = rv[NG + x];
    }
  }
  // the dL row of the phase-only block is exactly zero (U_dL = 0)
  if (lane < NPI) L.red[wave][NG + 2 * NPI + lane] = 0.0;
  // lane 16 i + 4 q + j of accumulator m holds element (i, j) of tile 4 m + q:
  // rows 0..6 of X are U_0, U_1, U_3 .. U_7, rows 7.. the W c_i rows (i >= 1),
  // column c is c_{c+1}; the upper triangle of W c_i c_j is kept
#pragma unroll
  for (int m = 0; m < Dm::NM; ++m) {
    const int t = 4 * m + q4;
    if (t >= Dm::NT) continue;
    const int row = 4 * Dm::tile_r(t) + kk, col = 4 * Dm::tile_c(t) + i4;
    int slot = -1;
    if (col < Dm::NB) {
      const int j = col + 1;
      if (row < 7) {
        slot = NG + kURow[row] * NPI + j;
      } else if (row < Dm::NA) {
        const int i = row - 6;
        if (j >= i) slot = NG + NX + i * NPI - (i * (i - 1)) / 2 + (j - i);
      }
    }
    double x = acc[m][0];
#pragma unroll
    for (int c = 1; c < NC; ++c) x += acc[m][c];
    if (slot >= 0) L.red[wave][slot] = x;
  }
  __syncthreads();
  if (tid < NACC) {
    double t = L.red[0][tid];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) t += L.red[w][tid];
    *tot = t;
  }
}

}  // namespace gwf
