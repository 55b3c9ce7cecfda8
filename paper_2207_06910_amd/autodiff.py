"""Differentiable network figure of merit over the detector parameters.

    J(xi) = w_snr * sum_e ln SNR_e + w_logdet * sum_e ln det Gamma_e[A, A]

as a function of xi [n_site, 4] = (latitude, longitude, arm angle gamma,
ln S0) of every site, for the events whose Fisher matrix (restricted to the
parameter rows A, all of them by default) inverts with a condition number
below cond_max (default 1e13).  The gradient of ln det Gamma is
tr(Gamma^-1 dGamma), a sum whose terms cancel by up to the condition number;
in FP64 it keeps about 1e-16 kappa relative accuracy per event, so events
with larger kappa would add noise rather than signal.  An event's own
parameter set (the workload's par_mask) further restricts A for that event.
The forward pass runs gwf_fisher (or a plan's gwf_plan_fisher) and
gwf_covariance (which returns ln det Gamma and Gamma^-1); the backward pass
runs the hand-written adjoint gwf_fisher_adjoint (or gwf_plan_adjoint) with
Gbar = Gamma^-1 embedded in the full matrix, recomputing the strain
derivatives at every grid point instead of storing them.  Every per-point
and per-event step runs in the library's kernels; this module only moves
tensors and adds the per-event values.
"""
from __future__ import annotations

import dataclasses
import math

from . import binding


def _sites_at(sites, xi):
    x = xi.detach().to("cpu", dtype=__import__("torch").float64).numpy()
    if x.shape != (len(sites), 4):
        raise binding.GwfError(f"xi must have shape ({len(sites)}, 4)")
    return [dataclasses.replace(s, lat=float(r[0]), lon=float(r[1]), gamma=float(r[2]),
                                S0=math.exp(float(r[3]))) for s, r in zip(sites, x)]


def site_parameters(dw):
    """xi [n_site, 4] of a workload's network, float64 on the CPU."""
    import torch
    return torch.tensor([[s.lat, s.lon, s.gamma, math.log(s.S0)] for s in dw.sites],
                        dtype=torch.float64)


def _forward(dw, xi, w_snr, w_logdet, rows, cond_max, plan=None):
    import torch
    dwx = dw.with_sites(_sites_at(dw.sites, xi))
    if plan is not None:              # the batched form: the plan's work items, network replaced
        plan.set_sites(dwx.sites)
        r = plan.run()
    else:
        r = binding.fisher(dwx)
    F = r["fisher"]
    P = F.shape[0]
    # restriction to the rows A by fixing the others; each event's own
    # parameter set (par_mask) is honoured by the inversion
    fixed = () if rows is None else [i for i in range(P) if i not in set(int(k) for k in rows)]
    inv = binding.covariance(F, r["status"], fixed=fixed, cond_max=cond_max, par_mask=dwx.par_mask)
    ok = inv["status"] == 0
    J = (w_snr * torch.log(r["snr"][ok]).sum() + w_logdet * inv["logdet"][ok].sum()).to(torch.float64)
    return dwx, r, inv, ok, J


class NetworkFoM(__import__("torch").autograd.Function):
    """J(xi); see the module docstring.  Use network_fom()."""

    @staticmethod
    def forward(ctx, xi, dw, w_snr, w_logdet, rows, cond_max, plan):
        import torch
        dwx, r, inv, ok, J = _forward(dw, xi, w_snr, w_logdet, rows, cond_max, plan)
        P = r["fisher"].shape[0]
        gbar = inv["cov"]
        if len(inv["out"]) != P:
            full = torch.zeros((P, P, dw.n), dtype=torch.float64, device=gbar.device)
            idx = torch.as_tensor(list(inv["out"]), dtype=torch.long, device=gbar.device)
            full[idx.view(-1, 1), idx.view(1, -1)] = gbar
            gbar = full
        ctx.dwx, ctx.gbar, ctx.status, ctx.plan = dwx, gbar, inv["status"], plan
        ctx.w = (float(w_snr), float(w_logdet))
        ctx.xi_device, ctx.xi_dtype = xi.device, xi.dtype
        return J.to(device=xi.device, dtype=xi.dtype)

    @staticmethod
    def backward(ctx, gJ):
        if ctx.plan is not None:
            g = ctx.plan.adjoint(ctx.gbar, status=ctx.status, w_snr=ctx.w[0], w_fisher=ctx.w[1])["grad"]
        else:
            g = binding.fisher_adjoint(ctx.dwx, ctx.gbar, status=ctx.status, w_snr=ctx.w[0],
                                       w_fisher=ctx.w[1])["grad"]
        g = g.to(device=ctx.xi_device, dtype=ctx.xi_dtype)
        return gJ * g, None, None, None, None, None, None


def network_fom(xi, dw, w_snr=1.0, w_logdet=1.0, rows=None, cond_max=1e13, plan=None):
    """J(xi) as a differentiable scalar (see the module docstring); rows
    selects the Fisher rows whose ln det enters (None: all).  With a plan
    (binding.Plan of the same workload, FP64) the forward and backward passes
    run over its work items (gwf_plan_fisher, gwf_plan_adjoint), the plan's
    network replaced by the sites at xi."""
    return NetworkFoM.apply(xi, dw, float(w_snr), float(w_logdet), None if rows is None else tuple(rows),
                            float(cond_max), plan)


def network_fom_value(xi, dw, w_snr=1.0, w_logdet=1.0, rows=None, cond_max=1e13):
    """J(xi) without gradient bookkeeping, and the mask of events that entered."""
    dwx, r, inv, ok, J = _forward(dw, xi, w_snr, w_logdet, None if rows is None else tuple(rows),
                                  float(cond_max))
    return J, ok
