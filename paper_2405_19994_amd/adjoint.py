"""Probe-voltage misfit of serial hybrid SDC as a torch.autograd.Function.

The loss L = sum_s sum_q (V(probe_q, t_s) - target_{s,q})^2 of a run of
nsteps serial HSDC steps and its gradient with respect to the per-node
conductivity field and the G_Na, G_CaL, G_Kr scalings come from the library
(hsdc_misfit_forward / hsdc_misfit_backward: per-step checkpoints, the
transposed sweep on the device); this module only marshals the arguments.
"""
import torch

from . import hsdc as H


class ProbeMisfit(torch.autograd.Function):
    """forward(sigma_node [N] float64 device, g_scale [3] float64, spec) -> L.

    spec: dict with dims, dx, chi, Cm, stim_w (device tensor or None),
    stim_amp, stim_t0, stim_dur, method (an hsdc_method), probes (int64 device
    [Q]), targets (float64 device [nsteps // sample_every, Q]), nsteps,
    sample_every and optionally y0 (device [19, N])."""

    @staticmethod
    def forward(ctx, sigma_node, g_scale, spec):
        gs = tuple(float(v) for v in g_scale.detach().cpu().tolist())
        prob = H.make_problem(spec["dims"], spec["dx"], (1.0, 1.0, 1.0),
                              sigma_node.detach().contiguous(), spec["chi"], spec["Cm"], gs,
                              spec.get("stim_w"), spec["stim_amp"], spec["stim_t0"],
                              spec["stim_dur"])
        m = H.Misfit(prob, spec["method"], spec["probes"], spec["targets"], spec["nsteps"],
                     spec["sample_every"], spec.get("y0"))
        ctx.misfit = m
        ctx.gdev, ctx.gdtype = g_scale.device, g_scale.dtype
        return torch.tensor(m.loss, dtype=torch.float64, device=sigma_node.device)

    @staticmethod
    def backward(ctx, grad_out):
        ds, dg, _ = ctx.misfit.backward(sigma=True)
        ctx.misfit.destroy()
        g = torch.tensor(dg, dtype=ctx.gdtype, device=ctx.gdev)
        return grad_out * ds, grad_out.to(ctx.gdev) * g, None


def probe_misfit(sigma_node, g_scale, spec):
    return ProbeMisfit.apply(sigma_node, g_scale, spec)
