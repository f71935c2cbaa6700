"""Differentiable unrolled PnP-MS2G iterations (Sec. 2.1, Algorithm 1).

``UnrolledPnP`` runs T iterations of ``pnp_step`` forward and, in the backward pass,
walks them in reverse with ``pnp_step_vjp``: the matched projector pair is its own
adjoint, the TV-prox is differentiated through its dual iterations, and each
iteration's internals are recomputed from a per-iteration checkpoint of its inputs
(x_{t-1}, y_{t-1}) and of its coarse gradient, which the forward step stores (so the
reverse step needs no forward projection of its own). Gradients are returned for the
initial image x_0 (= y_0) and for every step size eta_t. Batches of slices share the step sizes; their eta gradients
add up. All arithmetic runs in the library's kernels; this module only orders the
calls and keeps the checkpoints.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import fbpnp


@dataclass
class StepSpec:
    """One iteration: plan stage, optional device view list, minibatch scale, momentum,
    relaxation and denoiser parameters."""
    stage: int
    views: torch.Tensor | None = None
    sigma: float = 1.0
    a_t: float = 0.0
    alpha: float = 1.0
    lam: float = 0.01
    tau: float = 0.125
    tv_iters: int = 5


class UnrolledPnP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0: torch.Tensor, eta: torch.Tensor, plan: fbpnp.Plan, b: torch.Tensor, steps: list):
        """x0: [B, ny, nx] (or [ny, nx]); eta: [T]; b: [B, n_views * n_bins] (or flat)."""
        single = x0.dim() == 2
        x0b = x0.unsqueeze(0) if single else x0
        bb = b.reshape(x0b.shape[0], -1)
        T = len(steps)
        assert eta.numel() == T
        etas = [float(v) for v in eta.detach().cpu().tolist()]
        npix = plan.geom.nx * plan.geom.ny
        ckpt_x, ckpt_y, ckpt_g, outs = [], [], [], []
        for s in range(x0b.shape[0]):
            x = x0b[s].reshape(-1).contiguous().clone()
            y = x.clone()
            xs, ys, gs = [], [], []
            for t, st in enumerate(steps):
                xs.append(x)
                ys.append(y)
                nys, nxs = plan.coarse_shape(st.stage)
                g = torch.empty(nys * nxs, device=x.device)
                gs.append(g)
                xn = torch.empty(npix, device=x.device)
                yn = torch.empty(npix, device=x.device)
                args = fbpnp.pnp_args(plan, st.stage, bb[s].contiguous(), y, x, xn, yn, etas[t], st.a_t, st.views,
                                      st.sigma, st.alpha, st.lam, st.tau, st.tv_iters, grad=g)
                fbpnp.pnp_step(plan, args)
                x, y = xn, yn
            ckpt_x.append(xs)
            ckpt_y.append(ys)
            ckpt_g.append(gs)
            outs.append(x.reshape(plan.geom.ny, plan.geom.nx))
        ctx.plan, ctx.steps, ctx.etas, ctx.single = plan, steps, etas, single
        ctx.ckpt_x, ctx.ckpt_y, ctx.ckpt_g = ckpt_x, ckpt_y, ckpt_g
        ctx.b = bb
        out = torch.stack(outs)
        return out[0] if single else out

    @staticmethod
    def backward(ctx, gx):
        plan, steps, etas = ctx.plan, ctx.steps, ctx.etas
        gxb = gx.unsqueeze(0) if ctx.single else gx
        npix = plan.geom.nx * plan.geom.ny
        T = len(steps)
        tv_max = max(st.tv_iters for st in steps)
        ws = fbpnp.pnp_vjp_workspace(plan, tv_max, gx.device)
        eta_bar = torch.zeros((gxb.shape[0], T), device=gx.device)
        grads = []
        for s in range(gxb.shape[0]):
            xbar = gxb[s].reshape(-1).contiguous()
            ybar = None
            for t in range(T - 1, -1, -1):
                st = steps[t]
                y_prev, x_prev = ctx.ckpt_y[s][t], ctx.ckpt_x[s][t]
                args = fbpnp.pnp_args(plan, st.stage, ctx.b[s].contiguous(), y_prev, x_prev, x_prev, y_prev,
                                      etas[t], st.a_t, st.views, st.sigma, st.alpha, st.lam, st.tau, st.tv_iters,
                                      grad=ctx.ckpt_g[s][t])
                combine = t == 0
                xbar_prev = None if combine else torch.empty(npix, device=gx.device)
                ybar_prev = torch.empty(npix, device=gx.device)
                fbpnp.pnp_step_vjp(plan, args, xbar, ybar, xbar_prev, ybar_prev, eta_bar[s, t:t + 1], ws, combine)
                xbar, ybar = xbar_prev, ybar_prev
            grads.append(ybar.reshape(plan.geom.ny, plan.geom.nx))
        gx0 = torch.stack(grads)
        return (gx0[0] if ctx.single else gx0), eta_bar.sum(dim=0), None, None, None


def unrolled_pnp(plan: fbpnp.Plan, b: torch.Tensor, steps: list, x0: torch.Tensor, eta: torch.Tensor) -> torch.Tensor:
    """x_T as a differentiable function of x0 and eta (see UnrolledPnP)."""
    return UnrolledPnP.apply(x0, eta, plan, b, steps)
