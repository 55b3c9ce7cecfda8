/*
 * gwf.h -- C ABI of libgwf, the MI355X (gfx950) Fisher/SNR library.
 *
 * The library computes, for catalogues of compact-binary signals seen by a
 * network of ground-based interferometers, the matched-filter SNR and the
 * Fisher information matrix of the GWFAST method (arXiv:2207.06910), and
 * inverts the Fisher matrices into covariances:
 *
 *   SNR_i^2     = 4 int |h_i(f)|^2 / S_n,i(f) df                 (sec. 3.2)
 *   SNR^2       = sum_i SNR_i^2                                     (sec. 3.2)
 *   Gamma_ab    = sum_i 4 Re int d_a h_i d_b h_i^* / S_n,i df     (sec. 3.2)
 *   Cov         = Gamma^-1 by normalised Cholesky                  (sec. 4.1)
 *
 * with h_i the TaylorF2 restricted-PN strain (sec. 2.2, aligned spins,
 * optional tidal terms) projected on interferometer i with its antenna
 * patterns and arrival-time phase evaluated at the time t(f) = tc - tau*(f),
 * so that the Earth's rotation during the signal is included (sec. 3).
 * Integrals are trapezoid sums over log-spaced grids (sec. 2.2).
 *
 * Conventions
 *   - All array arguments are DEVICE pointers owned by the caller (for
 *     example the data of torch tensors on a ROCm device).  Descriptor
 *     structs (gwf_events, gwf_network, gwf_grid) live in host memory and are
 *     read only during the call.
 *   - Every compute call is asynchronous on `stream` (a hipStream_t; NULL is
 *     the null stream) and never synchronises it.  Outputs are valid once
 *     the stream has reached the call.
 *   - Structural argument errors (NULL pointers, sizes, descriptor fields,
 *     non-finite host-side geometry) are detected on the host before any
 *     launch and reported as GWF_E_INVALID_ARG; nothing is launched then.
 *     Per-event problems never fail a call: they are reported per event in
 *     the status[] array (bit flags GWF_EV_*), and the outputs of such an
 *     event are set to 0 (SNR/Fisher) or NaN (inversion outputs).
 *   - HIP failures at launch are reported as GWF_E_HIP; gwf_last_error()
 *     returns a message.  Device faults surface at the caller's next
 *     synchronisation.
 *   - The library holds no device memory of its own between calls except
 *     inside a plan (gwf_plan_*), and never frees caller memory.
 */
#ifndef GWF_H
#define GWF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GWF_VERSION 7

/* ------------------------------------------------------------- statuses */
typedef int32_t gwf_status;
enum {
  GWF_OK = 0,
  GWF_E_INVALID_ARG = 1,
  GWF_E_UNSUPPORTED = 2,
  GWF_E_HIP = 3,
  GWF_E_NOMEM = 4
};

/* per-event status bits */
enum {
  GWF_EV_OK = 0,
  GWF_EV_INVALID_PARAM = 1, /* Mc<=0, eta outside (0,1/4], dL<=0, |chi|>1,
                               Lambda<0, grid with n<2 or fmax<=fmin<=0     */
  GWF_EV_NOT_PD = 2,        /* Cholesky of the normalised Fisher failed     */
  GWF_EV_ILL_COND = 4,      /* condition number above cond_max: not inverted */
  GWF_EV_NONFINITE = 8,     /* a non-finite parameter or result            */
  GWF_EV_SKIPPED_SNR = 16,  /* SNR <= snr_th: Fisher not computed           */
  GWF_EV_SVD = 32           /* gwf_covariance with GWF_INV_CHO_SVD: the
                               Cholesky failed and the matrix was inverted
                               by SVD instead (outputs are set)              */
};

/* --------------------------------------------------------- parameters */
/* Row order of the parameter array and of the Fisher matrix (sec. 3.2,
 * with chi1z/chi2z as the spin basis and the two tidal deformabilities
 * last).  Units as in the paper's Table 1: Mc in solar masses (detector
 * frame), dL in Gpc, angles in radians, theta = pi/2 - dec, phi = RA.
 * Row GWF_TCOAL holds the GMST of coalescence in sidereal days (1 day =
 * 2 pi of Earth rotation); the matching Fisher row/column is the derivative
 * with respect to the coalescence time in SECONDS.  Masses are ordered
 * m1 >= m2 (chi1z, Lambda1 belong to the heavier body). */
enum {
  GWF_MC = 0, GWF_ETA, GWF_DL, GWF_THETA, GWF_PHI, GWF_IOTA, GWF_PSI,
  GWF_TCOAL, GWF_PHICOAL, GWF_CHI1Z, GWF_CHI2Z, GWF_LAMBDA1, GWF_LAMBDA2,
  GWF_NPAR_SRC = 13,  /* rows of gwf_events.par                               */
  GWF_NPAR_MAX = 14   /* rows of the largest Fisher matrix: the orbital
                         eccentricity e0 follows the spins and the tidal
                         deformabilities (sec. 3.2), so P = 11, 12 (e0),
                         13 (tides) or 14 (tides and e0)                     */
};

/* call flags */
enum {
  GWF_EARTH_ROT = 1, /* patterns and arrival-time phase at t(f); otherwise
                        frozen at the coalescence time (sec. 3, footnote)  */
  GWF_TIDAL = 2,     /* 5PN/6PN tidal phase; Fisher has 13 rows instead of 11 */
  GWF_ECCENTRIC = 8, /* moderate eccentricity (sec. 2.2, e0 <~ 0.1): the
                        leading-order e0^2 correction to the TaylorF2 phase,
                        e0 given at a reference frequency (gwf_events ecc,
                        f_ref_ecc); one more Fisher row, last              */
  GWF_MIXED = 4      /* mixed-precision form, accepted by gwf_plan_create and
                        gwf_waveform (gwf_snr and gwf_fisher return
                        GWF_E_UNSUPPORTED).  Plans: the noise weight
                        4 w A^2 / S_n(f) is evaluated with the PSD shape in
                        FP32; being a positive factor per grid point, its
                        relative error e (about 1e-6) moves SNR^2 by at most e
                        and each sigma_i by at most about e/2 at any condition
                        number.  Derivatives, sums and the inversion stay FP64
                        (FP32 products or sums would move the sigmas of
                        Fisher matrices with condition numbers of 1e10-1e17 by
                        far more than their size).  gwf_waveform: amplitude
                        and the sin/cos of the reduced phase in FP32 (the
                        phase itself, including the hour angle that sets the
                        arrival-time term, is assembled and reduced in FP64):
                        strain error below 1e-6 of the point's largest |h|.   */
};

typedef struct gwf_events {
  int64_t n;           /* number of events, >= 1                              */
  int64_t ld;          /* row stride of par in elements, >= n                 */
  const double* par;   /* device [GWF_NPAR_SRC][ld]: row r, event e at par[r*ld+e].
                          Rows LAMBDA1/LAMBDA2 are read only with GWF_TIDAL.   */
  const double* tc_s;  /* device [n] or NULL: coalescence time in seconds used
                          only in the 2 pi f tc term of the waveform phase     */
  const uint8_t* active; /* device [n_ifo][ld] or NULL (all on): interferometer d
                          (numbered site by site, three for a triangle) takes
                          part in event e's SNR, Fisher and adjoint only where
                          active[d*ld + e] != 0 -- the paper's duty factor
                          (sec. 3.1), the random draws being the caller's; its
                          per-interferometer SNR is then 0.  The strain
                          (gwf_waveform) is not affected.                      */
  const uint32_t* par_mask; /* device [n] or NULL (every row): the parameters of
                          event e's Fisher matrix, bit r for row r (GWF_MC ...
                          order; bits at or beyond the call's P are ignored),
                          so that one launch serves a mixed population (black
                          holes without their deformabilities).  A row outside
                          the set is left out: its row and column of the Fisher
                          output are 0, the inversions of a plan invert the rest
                          (its covariance row and column 0, its sigma NaN), and
                          the adjoint ignores gbar there.  SNR and strain are
                          not affected.                                       */
  const double* ecc;   /* device [n], required with GWF_ECCENTRIC (else not read):
                          the orbital eccentricity e0 >= 0 at the reference
                          frequency (sec. 2.1; e0 <~ 0.1 for the model to hold)  */
  const double* f_ref_ecc; /* device [n] or NULL: the reference frequency of e0 in
                          Hz, > 0; NULL means each event's grid starts there
                          (the paper's default fRef_ecc = None, sec. 2.1)      */
} gwf_events;

/* ------------------------------------------------------------ detectors */
enum { GWF_SHAPE_L = 0, GWF_SHAPE_T = 1 };
enum { GWF_PSD_ANALYTIC = 0, GWF_PSD_TABLE = 1, GWF_ASD_TABLE = 2 };

/* One detector site (sec. 3.1, Table 2), angles in radians.  An L site is
 * one interferometer whose arm bisector makes the angle gamma with local
 * East (counted towards North) and whose arms open by zeta.  A T site is
 * three co-located interferometers with 60-degree arms in a closed loop;
 * gamma is its first arm's angle, so the three bisectors are at
 * gamma + 30 deg + k 120 deg (zeta is ignored).  The three arms of a T
 * share its noise curve.
 * PSD (GWF_PSD_ANALYTIC): S_n(f) = S0 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 +
 * x^4/2)/(1 + x^2/2)] with x = f/f0.
 * PSD (GWF_PSD_TABLE, GWF_ASD_TABLE): a sampled noise curve, the paper's
 * psd_path file with its is_ASD flag (sec. 3.1): psd_n >= 2 frequencies
 * psd_f [Hz], strictly increasing and > 0, and the values psd_S there, the
 * PSD [1/Hz] or (GWF_ASD_TABLE) the ASD [1/sqrt(Hz)], squared into a PSD;
 * S_n(f) = S0 x (the PSD linearly interpolated in f), S0 a scale (1 for the
 * curve as given).  A grid point outside [psd_f[0], psd_f[psd_n-1]] gets
 * zero weight (the detector is blind there).  Both arrays are DEVICE
 * memory owned by the caller; their ordering and positivity are the
 * caller's (not checked: a value <= 0 inside the range makes that site's
 * weights infinite or negative, or NaN in the Fisher kernels, which take the
 * weight's square root; flagged GWF_EV_NONFINITE where it shows). */
typedef struct gwf_site {
  double lat, lon, gamma, zeta;
  int32_t shape;
  int32_t psd_kind;    /* GWF_PSD_ANALYTIC, GWF_PSD_TABLE or GWF_ASD_TABLE */
  double S0;           /* > 0: 1/Hz (analytic), a dimensionless scale (tables) */
  double f0;           /* > 0, Hz (analytic; not read for tables)            */
  const double* psd_f; /* device [psd_n] (tables; NULL for the analytic PSD)   */
  const double* psd_S; /* device [psd_n] (tables)                              */
  int64_t psd_n;       /* 2 <= psd_n <= 2^31 - 1 (tables)                      */
} gwf_site;

#define GWF_MAX_SITES 8
#define GWF_MAX_IFO 16

typedef struct gwf_network {
  int32_t n_site;          /* 1..GWF_MAX_SITES; at most GWF_MAX_IFO interferometers */
  const gwf_site* site;    /* host [n_site] */
} gwf_network;

/* ----------------------------------------------------------------- grids */
enum { GWF_GRID_LOG = 0, GWF_GRID_EXPLICIT = 1 };

/* Per-event log-spaced grid (sec. 2.2: geomspace from fmin to fmax):
 * f_k = fmin exp(k D), D = ln(fmax/fmin)/(n-1), k = 0..n-1, trapezoid
 * weights.  fmax == NULL means every grid ends at the event's cut frequency
 * 1/(6^{3/2} pi G M/c^3) (twice the ISCO orbital frequency, sec. 2.2). */
/* GWF_GRID_EXPLICIT: the frequencies themselves, event e's npts[e] values
 * at f[off[e]] .. f[off[e] + npts[e] - 1] (increasing and positive: the
 * first and last are checked, GWF_EV_INVALID_PARAM otherwise), with the
 * trapezoid weights of their differences; fmin and fmax are not read and
 * no cut frequency is applied.  Accepted by gwf_snr, gwf_fisher,
 * gwf_fisher_ifo, gwf_waveform and gwf_waveform_deriv; plans and the
 * adjoint return GWF_E_UNSUPPORTED (they generate log grids in registers). */
typedef struct gwf_grid {
  int32_t kind;            /* GWF_GRID_LOG or GWF_GRID_EXPLICIT */
  const double* fmin;      /* device [n], Hz (log)             */
  const double* fmax;      /* device [n] or NULL (log)         */
  const int32_t* npts;     /* device [n], 2 <= npts <= 2^30    */
  const int64_t* off;      /* device [n] (explicit)            */
  const double* f;         /* device, Hz (explicit)            */
} gwf_grid;

/* -------------------------------------------------------------- calls */

/* Detector strain h_i(f) of every event at every interferometer (sec. 3.1,
 * the full strain of the detector class, with the amplitude and phase of
 * sec. 2.2):
 *   h_i(f) = A(f) [F+_i (1 + cos^2 iota)/2 + i Fx_i cos iota] exp(i Psi_i)
 *   Psi_i  = 2 pi f (tc_s + Delta_i) - Phic - pi/4 + Psi_PN(f)
 * with the patterns F+/Fx and the geocentre delay Delta_i at t(f) under
 * GWF_EARTH_ROT, on the same log grids as gwf_fisher.  The phase is formed
 * in cycles and every term is reduced modulo one exactly before sin/cos, so
 * the result is limited by the FP64 evaluation of Psi_PN (relative error a
 * few 1e-16 of |Psi_PN|) and by how exactly f itself is known (the 2 pi f
 * tc_s term moves by 2 pi tc_s df).
 *   offsets device int64 [n]: event e writes columns offsets[e] ..
 *           offsets[e] + npts[e] - 1 of every row (packed grids: the
 *           exclusive prefix sum of npts; gaps between events are allowed
 *           and left untouched).  An event whose range does not lie in
 *           [0, total) gets GWF_EV_INVALID_PARAM and writes nothing.  The
 *           ranges of different events must not overlap (not checked).
 *   total   points per row, >= 1
 *   h       device [n_ifo][total][2] (re, im), required; a T site gives
 *           its three arms in order.  Points of events with a status
 *           are not written.
 *   status  device int32 [n] or NULL */
gwf_status gwf_waveform(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                        uint32_t flags, const int64_t* offsets, int64_t total, double* h,
                        int32_t* status, void* stream);

/* Derivatives of the detector strain with respect to the P parameters
 * (P = 13 with GWF_TIDAL, else 11), the vectors whose noise-weighted
 * products make the Fisher matrix (sec. 3.2):
 *   Gamma_ab = 4 Re sum_i int d_a h_i(f) d_b h_i(f)^* / S_n,i(f) df,
 * in the rows and units of gwf_fisher (GWF_MC ... order, dL in Gpc, the
 * GWF_TCOAL row per second), analytic and evaluated with the strain's phase
 * as in gwf_waveform.  Same events, network, grids, offsets and total as
 * gwf_waveform (no GWF_MIXED: GWF_E_UNSUPPORTED).
 *   dh      device [P][n_ifo][total][2] (re, im), required: row a * n_ifo + i
 *           holds d h_i / d parameter a; rows of parameters outside an
 *           event's set (ev->par_mask) are 0 over its columns.  Points of
 *           events with a status are not written.
 *   status  device int32 [n] or NULL
 * The output holds P times the strain's bytes (about 101 GB for 10^4
 * neutron-star binaries with 13 parameters on five interferometers). */
gwf_status gwf_waveform_deriv(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                              uint32_t flags, const int64_t* offsets, int64_t total, double* dh,
                              int32_t* status, void* stream);

/* Network SNR (sec. 3.2) of every event.
 *   snr     device [n], required
 *   snr_ifo device [n_ifo][n] or NULL: SNR of each interferometer (a T site
 *           contributes its three arms in order), the `return_all` output
 *   status  device int32 [n] or NULL
 * Same definitions and grids as gwf_fisher. */
gwf_status gwf_snr(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                   uint32_t flags, double* snr, double* snr_ifo, int32_t* status,
                   void* stream);

/* Network Fisher matrix (sec. 3.2) and SNR of every event, fused.
 *   fisher  device [P][P][n], required, P = 13 with GWF_TIDAL else 11, the
 *           the event index last, as the paper stacks its matrices
 *           (sec. 3.2); both triangles are written
 *   snr, snr_ifo, status as in gwf_snr (snr required, status required)
 *   snr_th  <= 0: every event; > 0: the Fisher is computed only where the
 *           network SNR exceeds snr_th (decided by a first SNR pass), other
 *           events get GWF_EV_SKIPPED_SNR and a zero Fisher.
 * Derivatives are exact partial derivatives of the model with the grid held
 * fixed (the cut frequency is not differentiated); they include the
 * dependence of the patterns and of the arrival-time phase on tc and, with
 * GWF_EARTH_ROT, on Mc and eta through tau*(f). */
gwf_status gwf_fisher(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                      uint32_t flags, double snr_th, double* fisher, double* snr,
                      double* snr_ifo, int32_t* status, void* stream);

/* The Fisher matrix of every interferometer on its own (the paper's
 * per-detector matrices, return_all in sec. 3.2), whose sum over the
 * interferometers is gwf_fisher's network matrix; a T site gives its three
 * arms in order, each with its own pattern map.  Same events (the duty
 * factor's active flags and par_mask included), network, grids and flags as
 * gwf_fisher, no SNR threshold and no GWF_MIXED (GWF_E_UNSUPPORTED).  One
 * launch per interferometer.
 *   fisher_ifo device [n_ifo][P][P][n], required; an interferometer that is
 *              off for an event (active) gives zeros there
 *   status     device int32 [n], required: the parameter status, as for
 *              gwf_fisher (GWF_EV_NONFINITE if any matrix is not finite)
 * Per-interferometer SNRs come from gwf_snr (snr_ifo). */
gwf_status gwf_fisher_ifo(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                          uint32_t flags, double* fisher_ifo, int32_t* status, void* stream);

/* Adjoint (reverse mode) of the Fisher/SNR map with respect to the detector
 * parameters: the gradient of a network figure of merit
 *   J = sum_e [ w_snr ln SNR_e + w_fisher sum_ij Gbar_e,ij Gamma_e,ij ]
 * along xi[s] = (latitude, longitude, gamma [rad], ln S0) of every site s,
 * with Gbar held fixed.  Passing Gbar = Gamma^-1 (the cov output of
 * gwf_invert) makes the second term the gradient of sum_e ln det Gamma_e;
 * any other Gbar = dJ/dGamma chains an arbitrary function of the Fisher
 * matrices.  The strain derivatives are recomputed at every grid point and
 * contracted on the fly (no Jacobian is stored); the SNR^2 that divides the
 * first term is recomputed too.  Triangle sites move as one (all three
 * arms).  Same definitions, grids and flags as gwf_fisher (no GWF_MIXED).
 *   gbar       device [P][P][n]; only its symmetric part enters
 *   status     device int32 [n] or NULL: events with a nonzero status (and
 *              events whose parameters are invalid or whose gbar holds a
 *              non-finite value) contribute zero
 *   grad_event device [n][n_site][4], required: each event's terms
 *   grad       device [n_site][4], required: their sum over events, taken in
 *              a fixed order (bitwise reproducible) */
gwf_status gwf_fisher_adjoint(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                              uint32_t flags, const double* gbar, const int32_t* status,
                              double w_snr, double w_fisher, double* grad_event, double* grad,
                              void* stream);

/* Batched FP64 inversion (sec. 4.1) of n Fisher matrices of size P
 * (1 <= P <= 13) in the [P][P][n] layout: each matrix is normalised by the
 * square root of its diagonal (skipped when a diagonal entry is not > 0),
 * Cholesky-factorised and inverted, and the normalisation is undone.
 *   cov      device [P][P][n] or NULL     covariance
 *   sigma    device [P][n], required      sqrt of the covariance diagonal
 *   cond     device [n] or NULL           condition number of the normalised
 *                                         matrix (ratio of extreme |eigenvalues|,
 *                                         one-sided Jacobi)
 *   inv_err  device [n] or NULL           max_ij |(Gamma Cov - 1)_ij| (sec. 4.1)
 *   logdet   device [n] or NULL           ln det Gamma from the Cholesky factor of
 *                                         the normalised matrix and the diagonal
 *   status   device int32 [n], required   bits are OR-ed into what is there
 *                                         (pass the gwf_fisher status through, or
 *                                         zeros)
 *   cond_max matrices with cond > cond_max are not inverted (GWF_EV_ILL_COND);
 *            the paper's default is 1e50.
 * Events with GWF_EV_INVALID_PARAM or GWF_EV_SKIPPED_SNR already set are
 * skipped.  Failed or skipped events get NaN cov/sigma/inv_err/logdet.
 * Every matrix is inverted whole; per-event parameter sets (gwf_events
 * par_mask) are honoured by gwf_covariance (gwf_cov_opts par_mask) and by
 * the inversion of a plan. */
gwf_status gwf_invert(int32_t P, int64_t n, const double* fisher, double cond_max,
                      double* cov, double* sigma, double* cond, double* inv_err,
                      double* logdet, int32_t* status, void* stream);

/* Covariance manipulations (sec. 4.2) and the sky localisation region
 * (sec. 4.1), around the inversion of gwf_invert, in this order:
 *   1. parameters in fixed_mask are held at their fiducial values: their rows
 *      and columns are removed from each Fisher matrix;
 *   2. prior[i] (the inverse variance of a Gaussian prior on parameter i,
 *      >= 0; 0 = none) is added to the diagonal of every kept parameter;
 *   3. that matrix is inverted as by gwf_invert (cond, inv_err, logdet and
 *      the status bits refer to it);
 *   4. with sky_level > 0, the region holding sky_level percent of the
 *      probability, -2 pi |sin theta| sqrt(C_tt C_pp - C_tp^2)
 *      ln(1 - sky_level/100), from the covariance entries of parameters
 *      i_theta and i_phi (NaN where that 2 x 2 determinant is negative);
 *   5. parameters in marg_mask are marginalised over: their rows and
 *      columns are left out of cov and sigma.
 * Bit i of a mask is parameter i of the stored matrix (GWF_MC ... order for
 * the Fisher output); fixed_mask and marg_mask must be disjoint and leave at
 * least one parameter; theta and phi must not be fixed when the sky area is
 * requested. */
enum { GWF_SKY_STERAD = 0, GWF_SKY_SQDEG = 1 };

/* Inversion methods (sec. 4.1; the paper's 'cho' with its SVD fallback,
 * 'svd', 'svd_reg'), applied to the normalised matrix:
 *   GWF_INV_CHO      Cholesky; a failure is flagged GWF_EV_NOT_PD (gwf_invert)
 *   GWF_INV_CHO_SVD  Cholesky, and an SVD where it fails (GWF_EV_SVD)
 *   GWF_INV_SVD      SVD, H^-1 = V diag(1/s) U^T; with truncate, singular
 *                    values below svals_thresh x max(s) are raised to it
 *   GWF_INV_SVD_REG  SVD, singular values below svals_thresh x max(s) left out
 *   GWF_INV_CHO_DD   Cholesky, L^-1 and L^-T L^-1 in double-double arithmetic
 *                    (about 106 bits): the covariance of the stored FP64 matrix
 *                    to about kappa 2^-104 before its rounding to FP64, the
 *                    GPU's counterpart of the paper's mpmath inversion
 * The SVD is the one-sided Jacobi of the condition number, run again with
 * the rotations accumulated; it also gives the eigen-decomposition. */
enum { GWF_INV_CHO = 0, GWF_INV_CHO_SVD = 1, GWF_INV_SVD = 2, GWF_INV_SVD_REG = 3, GWF_INV_CHO_DD = 4 };

typedef struct gwf_cov_opts {
  uint32_t fixed_mask;              /* parameters held fixed (step 1)            */
  uint32_t marg_mask;               /* parameters marginalised over (step 5)     */
  double prior[GWF_NPAR_MAX];       /* inverse prior variances (step 2), host    */
  double cond_max;                  /* as for gwf_invert; the paper's default 1e50 */
  double sky_level;                 /* percent, 0 < level < 100; <= 0: no sky area */
  int32_t i_theta, i_phi;           /* parameter indices of theta and phi
                                       (GWF_THETA, GWF_PHI for Fisher output)    */
  int32_t sky_units;                /* GWF_SKY_STERAD or GWF_SKY_SQDEG           */
  int32_t method;                   /* GWF_INV_*                                 */
  int32_t truncate;                 /* GWF_INV_SVD: raise small singular values  */
  int32_t pad;
  double svals_thresh;              /* ratio to the largest singular value; the
                                       paper's default is 1e-15                  */
  const uint32_t* par_mask;         /* device [n] or NULL: each event's parameter
                                       set, bit i for parameter i of the stored
                                       matrix (gwf_events par_mask); a parameter
                                       outside it is left out of steps 2-4 (a unit
                                       row and column stand in for it, so cond,
                                       inv_err and logdet are those of the rest),
                                       and its row and column of cov are 0, its
                                       sigma NaN; the sky area is NaN for an event
                                       without theta or phi; its eigenvalue is 1
                                       with eigenvector e_i                      */
} gwf_cov_opts;

/* P, n, fisher, status: as for gwf_invert (fisher is [P][P][n]).  With Po the
 * number of parameters neither fixed nor marginalised, in their stored order:
 *   cov      device [Po][Po][n] or NULL   covariance after marginalisation
 *   sigma    device [Po][n], required
 *   cond, inv_err, logdet   device [n] or NULL, of the matrix of step 3
 *   theta    device [n], the events' polar angles; required with sky_level > 0
 *   sky      device [n]; required with sky_level > 0, ignored otherwise
 *   eigval   device [Pk][n] or NULL, eigvec device [Pk][Pk][n] or NULL: the
 *            eigen-decomposition (the paper's CheckFisher) of the normalised
 *            matrix of step 3 (Pk parameters, fixed ones removed): eigenvalues
 *            ascending, eigvec[i][r] component i of eigenvector r, signed so
 *            that its largest-magnitude component is positive; NaN for events
 *            not processed (invalid, skipped or non-finite)
 * opts is host memory read during the call.  Invalid masks, priors, levels,
 * indices or methods return GWF_E_INVALID_ARG before any launch.  ln det is
 * NaN where the SVD inverts a matrix with a non-positive eigenvalue. */
gwf_status gwf_covariance(int32_t P, int64_t n, const double* fisher, const gwf_cov_opts* opts,
                          const double* theta, double* cov, double* sigma, double* cond,
                          double* inv_err, double* logdet, double* sky, double* eigval,
                          double* eigvec, int32_t* status, void* stream);

/* The Fisher matrix in other parameter bases: chi_s = (chi1z + chi2z)/2,
 * chi_a = (chi1z - chi2z)/2 in rows GWF_CHI1Z, GWF_CHI2Z; the paper's
 * tidal combinations Lambda~, delta Lambda~ (sec. 2.1) in rows GWF_LAMBDA1,
 * GWF_LAMBDA2; the component masses m1 >= m2 [solar masses] in rows GWF_MC,
 * GWF_ETA (sec. 3.2, use_m1m2).  Gamma' = J^T Gamma J with J = d native /
 * d new at each event's parameters; at fixed Lambda~, delta Lambda~ the
 * Lambdas move with eta, so in that basis the eta row (or the m1, m2 rows)
 * picks up the tidal rows.
 *   P        11 or 13 (GWF_BASIS_LAMBDA_TILDE needs 13)
 *   fisher   device [P][P][n] in the native basis (the gwf_fisher output)
 *   ev       the events the matrices belong to (par rows read on the device)
 *   basis    OR of GWF_BASIS_*; 0 copies
 *   out      device [P][P][n]; may equal fisher (in place)
 *   status   device int32 [n] or NULL: GWF_EV_NONFINITE is OR-ed in where the
 *            result is not finite (e.g. the tidal basis at eta = 1/4, where
 *            the map is singular)
 * ev->par_mask is not read: a matrix with rows left out of its event's
 * parameter set keeps zeros there when each pair of rows a basis mixes is
 * wholly in or out of the set (a black-hole pair's 11 rows in any basis); a
 * set holding one row of a pair (an NS-BH pair's Lambda2 without Lambda1)
 * gives a singular matrix in the basis that mixes them. */
enum { GWF_BASIS_CHI_SA = 1, GWF_BASIS_LAMBDA_TILDE = 2, GWF_BASIS_M1M2 = 4 };

gwf_status gwf_fisher_basis(int32_t P, int64_t n, const double* fisher, const gwf_events* ev,
                            uint32_t basis, double* out, int32_t* status, void* stream);

/* ------------------------------------------------------ batched form */
/* A plan runs the Fisher (and optionally the inversion) of one catalogue
 * repeatedly: the work is cut into items of at most `chunk` grid points
 * (events with long grids give several items), one workgroup takes each
 * item (longest items first), and each event's item sums are combined in
 * item order, so results are deterministic and independent of scheduling.
 * The set-up, item, combine and inversion kernels are captured once into a
 * HIP graph and replayed.  This is the batched form of the path
 * for catalogues with uneven grid lengths (the paper's counterpart is its
 * batch/process parallelism over catalogues, sec. 5).
 *
 * gwf_plan_create reads the grid lengths (npts) back to the host and
 * synchronises `stream`; with chunk left at 0 it also times the candidate
 * item lengths on the given events (autotuning).  The event,
 * grid and network descriptors are captured: later runs read the device
 * arrays at the same addresses, whose values (parameters, fmin, fmax) may
 * change, but the grid lengths may not (an event whose npts differs from
 * the plan's gets GWF_EV_INVALID_PARAM).  The plan owns its workspace
 * (about 2 KB per event plus 0.75 KB per work item) until gwf_plan_destroy. */
typedef struct gwf_plan gwf_plan;

typedef struct gwf_plan_options {
  int32_t chunk;       /* points per work item, a multiple of 256; 0 = autotune     */
  int32_t use_graph;   /* nonzero: capture and replay a HIP graph                     */
  int32_t profile;     /* nonzero (with use_graph = 0): time the work-item kernel of
                          each run with HIP events on its stream                     */
  int32_t inv_method;  /* inversion of gwf_plan_fisher: GWF_INV_CHO (0, flags a failed
                          Cholesky NOT_PD), GWF_INV_CHO_SVD (the paper's default: an
                          SVD where the Cholesky fails, status GWF_EV_SVD) or
                          GWF_INV_CHO_DD (double-double Cholesky); see gwf_covariance */
} gwf_plan_options;

typedef struct gwf_plan_info {
  int32_t chunk, n_items, use_graph, pad;
  int64_t workspace_bytes;
  double tuned_ms;     /* time of the chosen configuration during autotuning, or 0 */
  double items_ms;     /* with profile: work-item kernel time of the last run (this
                          call waits for that run to finish), else 0               */
} gwf_plan_info;

/* opt NULL: autotune both knobs, use a graph.  Sampled noise curves of the
 * network (gwf_site psd_f, psd_S) are read at their addresses on every run:
 * they must stay allocated, at the same addresses, for the plan's life. */
gwf_status gwf_plan_create(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                           uint32_t flags, const gwf_plan_options* opt, gwf_plan** plan,
                           void* stream);

/* Fisher, SNR and status of the plan's catalogue (same layouts and meaning
 * as gwf_fisher with snr_th = 0).  With sigma non-NULL the inversion of
 * gwf_invert follows in the same graph (cov, cond, inv_err optional), by the
 * plan's inv_method (gwf_plan_options). */
gwf_status gwf_plan_fisher(gwf_plan* plan, double* fisher, double* snr, int32_t* status,
                           double cond_max, double* cov, double* sigma, double* cond,
                           double* inv_err, void* stream);

/* The adjoint of gwf_fisher_adjoint over the plan's work items: the same
 * gradient (sec. 3.3 derivatives, reverse mode; the detector gradient is the
 * batched form of the adjoint) along every site's (latitude, longitude,
 * gamma, ln S0) of
 *   J = sum_e [ w_snr ln SNR_e + w_fisher sum_ij Gbar_e,ij Gamma_e,ij ],
 * for the plan's events, grids and current network (gwf_plan_set_network),
 * one workgroup per work item (longest first), each item's per-site sums
 * combined per event in item order and the events summed in a fixed order
 * (bitwise reproducible).  gbar, status, grad_event and grad as for
 * gwf_fisher_adjoint (grad_event [n][n_site][4], grad [n_site][4]).  Plans
 * created with GWF_MIXED return GWF_E_UNSUPPORTED.  The adjoint shares the
 * plan's workspace with gwf_plan_fisher: calls on one plan must be ordered
 * (one stream, or synchronised).  The first call on a plan allocates the
 * adjoint's constants (the contractions of each event's Gbar, about 1 KB per
 * event, and each site's pattern-derivative polynomials, about 0.7 KB per
 * event and site), kept with the plan until gwf_plan_destroy and counted in
 * gwf_plan_info's workspace_bytes; later calls allocate nothing.  Returns
 * GWF_E_NOMEM if that allocation fails. */
gwf_status gwf_plan_adjoint(gwf_plan* plan, const double* gbar, const int32_t* status, double w_snr,
                            double w_fisher, double* grad_event, double* grad, void* stream);

/* Replace the plan's network (any valid network of at most as many sites as
 * the plan was created with; grid lengths and items do not depend on it):
 * the detector positions, orientations and
 * noise curves of the next gwf_plan_fisher and gwf_plan_adjoint calls, e.g.
 * for gradient steps on the detector parameters.  A captured graph is
 * rebuilt at the next gwf_plan_fisher. */
gwf_status gwf_plan_set_network(gwf_plan* plan, const gwf_network* net);

gwf_status gwf_plan_get_info(const gwf_plan* plan, gwf_plan_info* info);

/* Frees the plan and its workspace (NULL is allowed). */
gwf_status gwf_plan_destroy(gwf_plan* plan);

/* ------------------------------------------- no device allocation */
/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * batched form of gwf_plan_fisher (work items of at most `chunk` points,
 * one workgroup each, each event's item sums combined in item order)
 * with its workspace in one fixed device array of GWF_STATIC_SCRATCH_BYTES
 * per device, which the library holds from its load until the process ends.
 * The work items are built on the device from the grid lengths, so the call
 * allocates nothing, reads nothing back and never synchronises; there is no
 * autotuning (chunk is the caller's) and no graph.  Outputs as for
 * gwf_fisher with snr_th = 0 (the same kernels as a plan: for the same chunk
 * the results equal gwf_plan_fisher's bit for bit).
 *   chunk     points per work item, a positive multiple of 256
 *   npts_max  an upper bound of the catalogue's grid lengths; an event with a
 *             longer grid gets GWF_EV_INVALID_PARAM and a zero Fisher matrix
 * The workspace needs, in 256-byte aligned parts, n x 1048 bytes of event
 * constants, n x n_site x 512 of site constants, 4 (n + 1) of item offsets,
 * and 16 + 8 NACC bytes per work item (NACC = 91 with GWF_TIDAL, else 69)
 * for n ceil(npts_max / chunk) items, plus 256; a call needing more than
 * GWF_STATIC_SCRATCH_BYTES returns GWF_E_INVALID_ARG before any launch (the
 * 10^4 neutron-star binaries of 2000-20000 points on three sites need
 * about 41 MB with chunk 16384).  Every call on a device uses the same
 * array: calls that overlap on one device (different streams, or threads)
 * race and must be serialised by the caller; each call rewrites everything
 * it reads. */
#define GWF_STATIC_SCRATCH_BYTES (64ll << 20)

gwf_status gwf_fisher_static(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                             uint32_t flags, int32_t chunk, int32_t npts_max, double* fisher, double* snr,
                             int32_t* status, void* stream);

/* Number of interferometers of a network (T sites count 3); -1 if invalid. */
int32_t gwf_network_n_ifo(const gwf_network* net);

/* Human-readable text of the last error of this thread. */
const char* gwf_last_error(void);

int32_t gwf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GWF_H */
