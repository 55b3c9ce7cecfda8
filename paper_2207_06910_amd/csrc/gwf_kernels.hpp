// gwf_kernels.hpp -- kernel argument blocks and launchers of libgwf.
#pragma once

#include "gwf_model.hpp"

namespace gwf {

struct FisherArgs {
  const double* par;
  int64_t ld, n;
  const double* fmin;
  const double* fmax;       // NULL: cut frequency
  const int32_t* npts;
  NetDesc net;
  double snr_th;
  const double* snr_pre;    // NULL, or SNRs of a previous pass for the threshold
  double* fisher;           // [P][P][n]
  double* snr;              // [n]
  int32_t* status;          // [n]
};

struct SnrArgs {
  const double* par;
  int64_t ld, n;
  const double* fmin;
  const double* fmax;
  const int32_t* npts;
  NetDesc net;
  int32_t tidal;
  double* snr;              // [n]
  double* snr_ifo;          // [n_ifo][n] or NULL
  int32_t* status;          // [n] or NULL
};

struct InvertArgs {
  int64_t n;
  const double* fisher;     // [P][P][n]
  double cond_max;
  double* cov;              // [P][P][n] or NULL
  double* sigma;            // [P][n]
  double* cond;             // [n] or NULL
  double* inv_err;          // [n] or NULL
  double* logdet;           // [n] or NULL
  int32_t* status;          // [n]
};

struct WaveformArgs {
  const double* par;
  int64_t ld, n;
  const double* tc_s;       // [n] or NULL
  const double* fmin;
  const double* fmax;       // NULL: cut frequency
  const int32_t* npts;
  NetDesc net;
  const int64_t* offsets;   // [n]: event e writes columns [offsets[e], offsets[e] + npts[e])
  int64_t total;            // points per interferometer row of h
  double* h;                // [n_ifo][total] complex (re, im)
  int32_t* status;          // [n] or NULL
};

struct AdjointArgs {
  const double* par;
  int64_t ld, n;
  const double* fmin;
  const double* fmax;       // NULL: cut frequency
  const int32_t* npts;
  NetDesc net;
  const double* gbar;       // [P][P][n]
  const int32_t* status;    // [n] or NULL
  double w_snr, w_fisher;
  double* grad_event;       // [n][n_site][4]
  double* grad;             // [n_site][4]
};

hipError_t launch_fisher(const FisherArgs& a, bool tidal, bool rot, hipStream_t stream);
hipError_t launch_snr(const SnrArgs& a, bool rot, hipStream_t stream);
hipError_t launch_invert(const InvertArgs& a, int P, hipStream_t stream);
hipError_t launch_waveform(const WaveformArgs& a, bool tidal, bool rot, bool mixed, hipStream_t stream);
hipError_t launch_adjoint(const AdjointArgs& a, bool tidal, bool rot, hipStream_t stream);

}  // namespace gwf
