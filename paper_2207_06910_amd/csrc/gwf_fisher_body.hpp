// gwf_fisher_body.hpp -- the per-workgroup Fisher accumulation shared by the
// one-event-per-workgroup kernel and the batched work-item kernel.
//
// A workgroup of kBlock lanes sums the contributions of grid points
// [k0, k1) of one event: each lane takes points k0 + tid + kBlock*it,
// evaluates the derivative vectors of all interferometers at that point in
// registers and adds its share of the 8x8 block of (Mc, eta, dL, theta, phi,
// iota, psi, tc) to its kGramAcc register accumulators (the 5x5 block of the
// rows that are not pattern combinations, plus pattern moments; see
// accumulate_point).  The phase-only blocks are a small
// dense contraction over frequency, X = sum_f a_f c_f^T with
// a_f = (U_0..U_7, W c_0..W c_{NPI-1}) and c_f = (c_0..c_{NPI-1}): every
// iteration each wavefront stages its 64 points' a_f and c_f in LDS and
// folds them into 4x4 output tiles of X with the four-block FP64 MFMA
// 4x4x4 (k = frequency), which keeps those sums out of the lanes' registers.
// The 13 x 5 block (tides; 11 x 3 without; with e0 one more row and column,
// in the same tiles) needs seven tiles (three): two MFMAs (one) per four
// points, a quarter of the cycles of one 16x16x4 MFMA per four points, which
// computes mostly padding.
// The sums are then reduced in a fixed order (wavefront butterflies, then
// the waves in index order), so results are bitwise reproducible.
#pragma once

#include "gwf_kernels.hpp"

namespace gwf {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kRowsA = 16;        // 8 U rows, up to 6 W c rows, zero rows to a whole tile
constexpr int kRowsB = 8;         // up to 6 c rows, zero rows to a whole tile
constexpr int kZeroRowB = 7;      // a B row no point writes (operand of unused tile slots)
constexpr int kZeroRowA = 15;
constexpr int kTileLd = 64 + 4;   // row stride (doubles): an operand read touches 8 rows x
                                  // 4 points, 2 (8 row + k) mod 64 distinct dword banks
constexpr int kNaccMax = 105;    // 36 + 8 NPI + NPI (NPI + 1)/2 at NPI = 6

template <int NPI_>
struct FisherDims {
  static constexpr int NPI = NPI_;                   // phase-only parameters
  static constexpr bool TIDAL = NPI >= 5;
  static constexpr int P = 8 + NPI;
  static constexpr int NG = 36, NX = 8 * NPI, NY = NPI * (NPI + 1) / 2;
  static constexpr int NACC = NG + NX + NY;          // SNR^2 = Gamma_{Phic,Phic}
  // 4x4 output tiles (row group R of a_f, column group C of c_f) of the
  // phase-only blocks: every tile of the U rows, and of the W c rows those
  // holding an element of the upper triangle (4C + 3 >= 4R - 8)
  static constexpr int RG = (8 + NPI + 3) / 4, CG = (NPI + 3) / 4;
  static constexpr int NT = TIDAL ? 7 : 3;
  static constexpr int NM = (NT + 3) / 4;            // MFMA accumulators (4 tiles each)
  __host__ __device__ static constexpr int tile_r(int t) { return TIDAL ? (t < 4 ? t / 2 : t == 6 ? 3 : 2) : t; }
  __host__ __device__ static constexpr int tile_c(int t) { return TIDAL ? (t < 4 ? t % 2 : t == 6 ? 1 : t - 4) : 0; }
};

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
  double acc[Dm::NM];
  const int wave = tid >> 6, lane = tid & 63;
  // four-block MFMA 4x4x4 operand layout: lane 16 k + 4 q + i holds A[q][i][k]
  // and B[q][k][i]; the result D[q][i][j] is in lane 16 i + 4 q + j.  Block q
  // of accumulator m is tile 4 m + q; unused slots read zero rows.
  const int kk = lane >> 4, q4 = (lane >> 2) & 3, i4 = lane & 3;
  int arow[Dm::NM], bcol[Dm::NM];
#pragma unroll
  for (int m = 0; m < Dm::NM; ++m) {
    acc[m] = 0.0;
    const int t = 4 * m + q4;
    arow[m] = t < Dm::NT ? 4 * Dm::tile_r(t) + i4 : kZeroRowA;
    bcol[m] = t < Dm::NT ? 4 * Dm::tile_c(t) + i4 : kZeroRowB;
  }
  double(*A)[kTileLd] = L.stA[wave];
  double(*B)[kTileLd] = L.stB[wave];
  // rows no point ever writes stay zero
#pragma unroll
  for (int r = 8 + NPI; r < kRowsA; ++r) A[r][lane] = 0.0;
#pragma unroll
  for (int r = NPI; r < kRowsB; ++r) B[r][lane] = 0.0;

  const int iters = (k1 - k0 + kBlock - 1) / kBlock;   // same trip count for every lane
  // on a log grid, v, 1/v and v^-12.42 walk from point to point (GridWalk)
  GridWalk gw;
  if (!EXPL) gw.start(ec, k0 + tid, kBlock);
  for (int it = 0; it < iters; ++it) {
    // The per-event constants stay in LDS and are re-read every iteration
    // (uniform broadcast reads); hoisting them out of the loop would need
    // more registers than a lane has.
    __asm__ volatile("" ::: "memory");
    const int k = k0 + it * kBlock + tid;
    double U[8], W = 0.0, cph[NPI];
#pragma unroll
    for (int b = 0; b < 8; ++b) U[b] = 0.0;
#pragma unroll
    for (int i = 0; i < NPI; ++i) cph[i] = 0.0;
    if (k < k1)
      accumulate_point<NPI, ROT, MIXED, PSUM, EXPL, TAB>(ec, sc, n_site, k, G, U, W, cph,
                                                         EXPL ? nullptr : gw.val);
    if (!EXPL) gw.step();
    // stage this point's row (points past the range contribute zeros)
#pragma unroll
    for (int b = 0; b < 8; ++b) A[b][lane] = U[b];
#pragma unroll
    for (int i = 0; i < NPI; ++i) {
      A[8 + i][lane] = W * cph[i];
      B[i][lane] = cph[i];
    }
    __builtin_amdgcn_wave_barrier();
    // The LDS-fed MFMA phase runs at raised issue priority, so it drains
    // quickly while the SIMD's other wave keeps the VALU busy (measured:
    // items kernel 1.7% faster, sums unchanged).
    __builtin_amdgcn_s_setprio(1);
    // X += A^T B over this wavefront's 64 points, four points per step
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) {
#pragma unroll
      for (int m = 0; m < Dm::NM; ++m) {
        const double av = A[arow[m]][4 * s2 + kk];
        const double bv = B[bcol[m]][4 * s2 + kk];
        acc[m] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bv, acc[m], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_wave_barrier();
  }

  // ---- deterministic reduction: wavefront butterflies, then the waves in order
  double F[NG];
  gram_finish(ec, G, F);
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const double t = wave_sum(F[i]);
    if (lane == 0) L.red[wave][i] = t;
  }
  // lane 16 i + 4 q + j of accumulator m holds element (i, j) of tile 4 m + q:
  // X rows 0..7 are the U_b rows (columns 0..NPI-1), rows 8..8+NPI-1 the
  // W c_i rows (upper triangle kept)
#pragma unroll
  for (int m = 0; m < Dm::NM; ++m) {
    const int t = 4 * m + q4;
    if (t >= Dm::NT) continue;
    const int row = 4 * Dm::tile_r(t) + kk, col = 4 * Dm::tile_c(t) + i4;
    int slot = -1;
    if (row < 8 && col < NPI) slot = NG + row * NPI + col;
    else if (row >= 8 && row < 8 + NPI && col >= row - 8 && col < NPI) {
      const int i = row - 8;
      slot = NG + NX + i * NPI - (i * (i - 1)) / 2 + (col - i);
    }
    if (slot >= 0) L.red[wave][slot] = acc[m];
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
