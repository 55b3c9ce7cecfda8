// gwf_kernels.hpp -- kernel argument blocks and launchers of libgwf.
#pragma once

#include <algorithm>

#include "gwf_model.hpp"

namespace gwf {

// A launch counts its work-items in 32 bits, so kernels with one workgroup
// per event (or per work item, or per few matrices) go out in slices of at
// most 2^31 work-items; each slice's kernel adds its first unit, `base`.
template <class Args, class Launch>
hipError_t launch_slices(Args a, int64_t units, int64_t units_per_wg, unsigned block, Launch&& launch) {
  const int64_t max_wg = (int64_t(1) << 31) / block;
  const int64_t wgs = (units + units_per_wg - 1) / units_per_wg;
  for (int64_t b = 0; b < wgs; b += max_wg) {
    a.base = b * units_per_wg;
    launch(a, dim3((unsigned)std::min(max_wg, wgs - b)), dim3(block));
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

struct FisherArgs {
  const double* par;
  int64_t ld, n;
  const double* ecc;        // [n] or NULL: e0 (eccentric instantiations only)
  const double* fref;       // [n] or NULL: reference frequency of e0 (NULL: grid start)
  const double* fmin;
  const double* fmax;       // NULL: cut frequency
  const int32_t* npts;
  const int64_t* goff;      // explicit grid: [n] first frequency of each event in gf, or NULL (log grid)
  const double* gf;         // explicit grid frequencies, or NULL
  const uint8_t* active;    // [n_ifo][ld] or NULL: interferometers taking part (duty factor)
  const uint32_t* par_mask; // [n] or NULL: rows of each event's Fisher matrix (others 0)
  int32_t ifo_sel;          // 0: every interferometer; d + 1: interferometer d alone
  NetDesc net;
  double snr_th;
  const double* snr_pre;    // NULL, or SNRs of a previous pass for the threshold
  double* fisher;           // [P][P][n]
  double* snr;              // [n] or NULL
  int32_t* status;          // [n]
  int64_t base;             // first event of the launch (set by the launcher)
};

struct SnrArgs {
  const double* par;
  int64_t ld, n;
  const double* fmin;
  const double* fmax;
  const int32_t* npts;
  const int64_t* goff;      // explicit grid: [n] first frequency of each event in gf, or NULL (log grid)
  const double* gf;         // explicit grid frequencies, or NULL
  const uint8_t* active;    // [n_ifo][ld] or NULL
  NetDesc net;
  int32_t tidal;
  double* snr;              // [n]
  double* snr_ifo;          // [n_ifo][n] or NULL
  int32_t* status;          // [n] or NULL
  int64_t base;             // first event of the launch (set by the launcher)
};

struct InvertArgs {
  int64_t n;
  const double* fisher;     // [p_full][p_full][n]
  double cond_max;
  double* cov;              // [n_out][n_out][n] or NULL
  double* sigma;            // [n_out][n]
  double* cond;             // [n] or NULL
  double* inv_err;          // [n] or NULL
  double* logdet;           // [n] or NULL
  int32_t* status;          // [n]
  // Covariance manipulations (sec. 4.2).  p_full = 0: none, the stored matrix
  // is inverted whole (launch_invert fills the identity maps below).
  int32_t p_full;           // parameters of the stored matrix
  int32_t n_out;            // parameters of cov and sigma (after marginalisation)
  int8_t keep[kMaxPar];      // stored index of kept parameter i (fixed ones removed)
  int8_t out_pos[kMaxPar];   // output position of kept parameter i, -1 if marginalised
  double prior[kMaxPar];     // added to kept diagonal entry i before inversion
  int32_t i_theta, i_phi;   // kept positions of theta and phi, -1: no sky area
  double sky_fac;           // -2 pi ln(1 - X/100) [x (180/pi)^2 for square degrees]
  const double* theta;      // [n], the events' polar angles (sky area only)
  double* sky;              // [n] or NULL
  // Inversion method (sec. 4.1): 0 Cholesky, a failure flagged; 1 an SVD
  // where the Cholesky fails; 2 SVD, with truncate: singular values below
  // svals_thresh x max raised to that value; 3 SVD leaving them out;
  // 4 Cholesky in double-double arithmetic.
  int32_t method, truncate;
  double svals_thresh;
  double* eigval;           // [P][n] or NULL: eigenvalues of the normalised kept matrix
  double* eigvec;           // [P][P][n] or NULL: its eigenvectors (columns)
  // [n] or NULL: each event's parameter set, bit i for stored parameter i; a
  // kept parameter outside it is replaced by a unit row and column, and its
  // covariance row and column are written as 0, its sigma as NaN
  const uint32_t* par_mask;
  int64_t base;             // first matrix of the launch (set by the launcher)
};

struct BasisArgs {
  int64_t n;
  const double* fisher;     // [P][P][n] in the native basis
  double* out;              // [P][P][n], may equal fisher
  const double* par;        // [13][ld] native parameters
  int64_t ld;
  uint32_t basis;           // 1 chi_s/chi_a, 2 Lambda~/delta Lambda~, 4 m1/m2
  int32_t* status;          // [n] or NULL
};

struct WaveformArgs {
  const double* par;
  int64_t ld, n;
  const double* ecc;        // [n] or NULL: e0 (with kFlagEcc in the call's flags)
  const double* fref;       // [n] or NULL: reference frequency of e0
  uint32_t ecc_flag;        // kFlagEcc or 0
  const double* tc_s;       // [n] or NULL
  const double* fmin;
  const double* fmax;       // NULL: cut frequency
  const int32_t* npts;
  const int64_t* goff;      // explicit grid: [n] first frequency of each event in gf, or NULL (log grid)
  const double* gf;         // explicit grid frequencies, or NULL
  NetDesc net;
  const int64_t* offsets;   // [n]: event e writes columns [offsets[e], offsets[e] + npts[e])
  int64_t total;            // points per interferometer row of h
  double* h;                // [n_ifo][total] complex (re, im)
  int32_t* status;          // [n] or NULL
  double* dh;               // derivative kernel: [P][n_ifo][total] complex
  const uint32_t* par_mask; // derivative kernel: [n] or NULL, rows outside an event's set are 0
  int64_t base;             // first event of the launch (set by the launcher)
};

struct AdjointArgs {
  const double* par;
  int64_t ld, n;
  const double* ecc;        // [n] or NULL: e0 (eccentric instantiations only)
  const double* fref;       // [n] or NULL
  const double* fmin;
  const double* fmax;       // NULL: cut frequency
  const int32_t* npts;
  const uint8_t* active;    // [n_ifo][ld] or NULL
  const uint32_t* par_mask; // [n] or NULL: gbar entries outside an event's rows are ignored
  NetDesc net;
  const double* gbar;       // [P][P][n]
  const int32_t* status;    // [n] or NULL
  double w_snr, w_fisher;
  double* grad_event;       // [n][n_site][4]
  double* grad;             // [n_site][4]
  int64_t base;             // first event of the launch (set by the launcher)
};

// npi: phase-only parameters, 3 + 2 (tides) + 1 (eccentricity)
hipError_t launch_fisher(const FisherArgs& a, int npi, bool rot, hipStream_t stream);
hipError_t launch_snr(const SnrArgs& a, bool rot, hipStream_t stream);
hipError_t launch_invert(const InvertArgs& a, int P, hipStream_t stream);
hipError_t launch_basis(const BasisArgs& a, int P, hipStream_t stream);
hipError_t launch_waveform_deriv(const WaveformArgs& a, int npi, bool rot, hipStream_t stream);
hipError_t launch_waveform(const WaveformArgs& a, bool tidal, bool rot, bool mixed, hipStream_t stream);
hipError_t launch_adjoint(const AdjointArgs& a, int npi, bool rot, hipStream_t stream);

}  // namespace gwf
