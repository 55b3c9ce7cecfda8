"""TEST INFRASTRUCTURE ONLY -- the CPU oracle of the Fisher/SNR path.

A plain, slow, FP64 reference written from the paper (arXiv:2207.06910):
``gwf_oracle.cpp`` evaluates the strain, SNR and Fisher matrices literally
(tensor-form antenna patterns, full complex phase, dual-number derivatives,
compensated trapezoid sums); ``invert.py`` inverts Fisher matrices with
mpmath, the arbitrary-precision library the paper itself uses (sec. 4.1),
and applies the covariance manipulations of sec. 4.2 and the sky area.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library shares no code with
it and never calls it.
"""
from .core import (build, load, fisher, fisher_tangent, restrict_rows, waveform, waveform_derivs, strain, strain_cstep, strain_plain, phase_tau,
                   phase_dpsi_df_cstep, phase_cstep_par, n_params, antenna, delay, cut_frequency, psd, noise_weight, grid, constants,
                   ifos, n_ifo)
from .basis import fisher_basis, jacobian as basis_jacobian, CHI_SA, LAMBDA_TILDE, M1M2
from .invert import covariance, eigen, fix_params, add_prior, marginalise, sky_area, covariance_epilogue

__all__ = ["build", "load", "fisher", "fisher_tangent", "restrict_rows", "waveform", "waveform_derivs", "strain", "strain_cstep", "strain_plain", "phase_tau",
           "phase_dpsi_df_cstep", "phase_cstep_par", "n_params", "antenna", "delay", "cut_frequency", "psd", "noise_weight", "grid",
           "constants", "ifos", "n_ifo", "covariance", "eigen", "fix_params", "add_prior", "marginalise",
           "sky_area", "covariance_epilogue", "fisher_basis", "basis_jacobian", "CHI_SA",
           "LAMBDA_TILDE", "M1M2"]
