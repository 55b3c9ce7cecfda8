// gwf_fisher_body.hpp -- the per-workgroup Fisher accumulation shared by the
// one-event-per-workgroup kernel and the batched work-item kernel.
//
// A workgroup of kBlock lanes sums the contributions of grid points
// [k0, k1) of one event: each lane takes points k0 + tid + kBlock*it,
// evaluates the derivative vectors of all interferometers at that point in
// registers and adds the 8x8 block of (Mc, eta, dL, theta, phi, iota, psi,
// tc) to its 36 register accumulators.  The phase-only blocks are a small
// dense contraction over frequency, X = sum_f a_f c_f^T with
// a_f = (U_0..U_7, W c_0..W c_{NPI-1}) and c_f = (c_0..c_{NPI-1}): every
// iteration each wavefront stages its 64 points' a_f and c_f in LDS and
// folds them into a 16x16 FP64 accumulator with 16 MFMA 16x16x4 steps
// (k = frequency), which keeps those 55 sums out of the lanes' registers.
// The sums are then reduced in a fixed order (wavefront butterflies, then
// the waves in index order), so results are bitwise reproducible.
#pragma once

#include "gwf_kernels.hpp"

namespace gwf {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kRowsA = 16;        // 8 U rows, up to 5 W c rows, zero rows up to the MFMA size
constexpr int kRowsB = 16;        // up to 5 c rows, zero rows up to the MFMA size
constexpr int kTileLd = 64 + 1;   // odd row stride (doubles): the 64 lanes of an operand
                                  // read (16 rows x 4 k-groups) fall in distinct banks
constexpr int kNaccMax = 91;

typedef double v4d __attribute__((ext_vector_type(4)));

template <bool TIDAL>
struct FisherDims {
  static constexpr int P = TIDAL ? 13 : 11;
  static constexpr int NPI = P - 8;                  // phase-only parameters
  static constexpr int NG = 36, NX = 8 * NPI, NY = NPI * (NPI + 1) / 2;
  static constexpr int NACC = NG + NX + NY;          // SNR^2 = Gamma_{Phic,Phic}
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

// Load an event's 13 parameters (missing tidal rows read as zero).
__device__ inline void load_par(const double* __restrict__ par, int64_t ld, int64_t e, bool tidal,
                                double p[13]) {
  for (int r = 0; r < 13; ++r) p[r] = (r < 11 || tidal) ? par[r * ld + e] : 0.0;
}

// Sums of points [k0, k1) of the event whose constants are ec/sc.  On
// return (after a workgroup barrier), lane t < NACC holds accumulator slot t
// (see slot_position) in *tot.
template <bool TIDAL, bool ROT, bool MIXED = false, bool PSUM = true>
__device__ inline void fisher_sums(const EventC& ec, const SiteC* sc, int n_site, int k0, int k1,
                                   FisherLds& L, double* tot) {
  using Dm = FisherDims<TIDAL>;
  constexpr int NPI = Dm::NPI, NG = Dm::NG, NX = Dm::NX, NACC = Dm::NACC;
  const int tid = threadIdx.x;
  double G[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) G[i] = 0.0;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  const int wave = tid >> 6, lane = tid & 63;
  const int mrow = lane & 15, mk = lane >> 4;      // MFMA operand position of this lane
  double(*A)[kTileLd] = L.stA[wave];
  double(*B)[kTileLd] = L.stB[wave];
  // rows no point ever writes stay zero
#pragma unroll
  for (int r = 8 + NPI; r < kRowsA; ++r) A[r][lane] = 0.0;
#pragma unroll
  for (int r = NPI; r < kRowsB; ++r) B[r][lane] = 0.0;

  const int iters = (k1 - k0 + kBlock - 1) / kBlock;   // same trip count for every lane
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
    if (k < k1) accumulate_point<TIDAL, ROT, MIXED, PSUM>(ec, sc, n_site, k, G, U, W, cph);
    // stage this point's row (points past the range contribute zeros)
#pragma unroll
    for (int b = 0; b < 8; ++b) A[b][lane] = U[b];
#pragma unroll
    for (int i = 0; i < NPI; ++i) {
      A[8 + i][lane] = W * cph[i];
      B[i][lane] = cph[i];
    }
    __builtin_amdgcn_wave_barrier();
    // X += A^T B over this wavefront's 64 points: k-step s takes points 16 mk + s
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) {
      const double av = A[mrow][16 * mk + s2];
      const double bv = B[mrow][16 * mk + s2];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
  }

  // ---- deterministic reduction: wavefront butterflies, then the waves in order
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const double t = wave_sum(G[i]);
    if (lane == 0) L.red[wave][i] = t;
  }
  // register r of lane (mk, mrow) holds accumulator element (4 r + mk, mrow):
  // rows 0..7 are the U_b rows (cols 0..NPI-1), rows 8..8+NPI-1 the W c_i
  // rows (upper triangle kept)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * r + mk, col = mrow;
    int slot = -1;
    if (row < 8 && col < NPI) slot = NG + row * NPI + col;
    else if (row >= 8 && row < 8 + NPI && col >= row - 8 && col < NPI) {
      const int i = row - 8;
      slot = NG + NX + i * NPI - (i * (i - 1)) / 2 + (col - i);
    }
    if (slot >= 0) L.red[wave][slot] = acc[r];
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
