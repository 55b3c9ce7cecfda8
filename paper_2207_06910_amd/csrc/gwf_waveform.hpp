// gwf_waveform.hpp -- helpers shared by the strain kernel (gwf_waveform.hip)
// and the strain-derivative kernel (gwf_waveform_deriv.hip): the event's
// inputs and the phase's reduction in cycles.  The two kernels sit in
// separate sources because they are built with different code-generation
// options (see build.py).
#pragma once

#include "gwf_kernels.hpp"

namespace gwf {

constexpr int kWBlock = 256;

// Event e's inputs: the 13 parameters (no tidal rows without tides), e0 and
// its reference frequency (with the eccentric flag, else zero).
__device__ inline void load_event(const WaveformArgs& a, int64_t e, bool tidal, double* p) {
  for (int r = 0; r < 13; ++r) p[r] = (r < 11 || tidal) ? a.par[r * a.ld + e] : 0.0;
  p[13] = a.ecc_flag && a.ecc ? a.ecc[e] : 0.0;
  p[14] = a.ecc_flag && a.fref ? a.fref[e] : 0.0;
}

// x reduced to [-1/2, 1/2] by subtracting the nearest integer (exact).
__device__ inline double frac_center(double x) { return x - rint(x); }

// sin and cos of 2 pi x for |x| <= 1/2.  FP64: the quarter-turn q = rint(4x)
// and the rest r = x - q/4 are exact in cycles (|r| <= 1/8), so t = 2 pi r
// carries one rounding (|t| <= pi/4) and needs no Cody-Waite reduction; the
// Taylor series of sin to t^17 and cos to t^16 truncate below 1e-18.
// Mixed form: the quarter-turn q = rint(4x) and the rest
// r = x - q/4 (exact, |r| <= 1/8) are taken in FP64, then the Taylor series
// of sin (to the 9th power) and cos (to the 10th) of 2 pi r in FP32, whose
// truncation errors (< 2e-9, < 2e-10 on |2 pi r| <= pi/4) lie below the
// FP32 rounding; the absolute error is a few 1e-8 rad from rounding r and
// about 1e-7 from the FP32 arithmetic.
template <bool MIXED>
__device__ inline void sincos_cycles(double x, double* s, double* c) {
  if (MIXED) {
    const double q = rint(4.0 * x);
    const float t = (float)kTwoPi * (float)fma(-0.25, q, x);
    const float t2 = t * t;
    float ps = fmaf(t2, 1.0f / 362880.0f, -1.0f / 5040.0f);
    ps = fmaf(ps, t2, 1.0f / 120.0f);
    ps = fmaf(ps, t2, -1.0f / 6.0f);
    const float sr = fmaf(t * t2, ps, t);
    float pc = fmaf(t2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
    pc = fmaf(pc, t2, -1.0f / 720.0f);
    pc = fmaf(pc, t2, 1.0f / 24.0f);
    pc = fmaf(pc, t2, -0.5f);
    const float cr = fmaf(t2, pc, 1.0f);
    const int k = (int)q & 3;                  // angle = k quarter turns + t
    const float ss = (k & 1) ? cr : sr, cc = (k & 1) ? sr : cr;
    *s = (double)((k & 2) ? -ss : ss);
    *c = (double)(((k + 1) & 2) ? -cc : cc);
  } else {
    const double q = rint(4.0 * x);
    const double t = kTwoPi * fma(-0.25, q, x);
    const double t2 = t * t;
    double ps = -1.0 / 355687428096000.0;          // -1/17!
    ps = fma(ps, t2, 1.0 / 1307674368000.0);       //  1/15!
    ps = fma(ps, t2, -1.0 / 6227020800.0);         // -1/13!
    ps = fma(ps, t2, 1.0 / 39916800.0);            //  1/11!
    ps = fma(ps, t2, -1.0 / 362880.0);             // -1/9!
    ps = fma(ps, t2, 1.0 / 5040.0);                //  1/7!
    ps = fma(ps, t2, -1.0 / 120.0);                // -1/5!
    ps = fma(ps, t2, 1.0 / 6.0);                   //  1/3!
    const double sr = fma(-t * t2, ps, t);
    double pc = 1.0 / 20922789888000.0;            //  1/16!
    pc = fma(pc, t2, -1.0 / 87178291200.0);        // -1/14!
    pc = fma(pc, t2, 1.0 / 479001600.0);           //  1/12!
    pc = fma(pc, t2, -1.0 / 3628800.0);            // -1/10!
    pc = fma(pc, t2, 1.0 / 40320.0);               //  1/8!
    pc = fma(pc, t2, -1.0 / 720.0);                // -1/6!
    pc = fma(pc, t2, 1.0 / 24.0);                  //  1/4!
    pc = fma(pc, t2, -0.5);                        // -1/2!
    const double cr = fma(t2, pc, 1.0);
    const int k = (int)q & 3;                      // angle = k quarter turns + t
    const double ss = (k & 1) ? cr : sr, cc = (k & 1) ? sr : cr;
    *s = (k & 2) ? -ss : ss;
    *c = ((k + 1) & 2) ? -cc : cc;
  }
}

}  // namespace gwf
