"""Differentiable rollout of the cascaded D2Q9 LBM with a hand-written adjoint.

    rho_T, u_T = rollout(params, force, u0, steps, checkpoint_every=100)

maps a per-node body-force field F [2, ny, nx] and an initial velocity u0
[2, ny, nx] to the density and velocity after `steps` steps (Sec. II
hydrodynamic fields of the state at time T).  Gradients of any scalar loss of
rho_T, u_T with respect to F and u0 are computed by the library's adjoint
kernels: the loss cotangent is pulled back through the macroscopic map, then
through each step in reverse (transposed per-node Jacobian of the cascaded
collision and forcing, then reverse streaming), then through the
initial-state map.

Memory: the forward keeps a lattice snapshot every `checkpoint_every` steps;
the backward recomputes each segment from its snapshot into a buffer of
`checkpoint_every + 1` lattices and runs the adjoint over it newest-first.
Work per step of the backward: one recomputed step and one adjoint step.
"""
from __future__ import annotations

from typing import Optional

import torch

from .lattice import Lattice, Params


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, force: torch.Tensor, u0: torch.Tensor, params: Params, steps: int,
                every: int, rho_init: Optional[torch.Tensor]):
        if params.storage not in ("fp64", "fp32"):
            raise ValueError("the adjoint needs fp64 or fp32 storage")
        if steps < 0 or every < 1:
            raise ValueError("steps >= 0 and checkpoint_every >= 1 required")
        ny, nx = params.ny, params.nx
        dev = force.device
        real = params.real_dtype
        lat = Lattice(params, device=dev, force=force.detach())
        f64 = torch.float64
        rho = (torch.full((ny, nx), params.rho0, dtype=f64, device=dev) if rho_init is None
               else rho_init.detach().to(dtype=f64).contiguous())
        ux0 = u0[0].detach().to(dtype=f64).contiguous()
        uy0 = u0[1].detach().to(dtype=f64).contiguous()
        lat.init_equilibrium(rho, ux0, uy0)
        snaps = []
        t = 0
        while True:
            snaps.append(lat.snapshot())
            n = min(every, steps - t)
            if n <= 0:
                break
            lat.step(n)
            t += n
            if t >= steps:
                break
        m = lat.macroscopic(strain=False)
        ctx.lat, ctx.snaps, ctx.steps, ctx.every = lat, snaps, steps, every
        ctx.init_fields = (rho, ux0, uy0)
        return m["rho"], torch.stack([m["ux"], m["uy"]])

    @staticmethod
    def backward(ctx, g_rho, g_u):
        lat: Lattice = ctx.lat
        steps, every = ctx.steps, ctx.every
        p = lat.params
        dev, real = lat.device, lat.real
        grad_force = torch.zeros((2, p.ny, p.nx), dtype=real, device=dev)
        g_rho = None if g_rho is None else g_rho.to(real).contiguous()
        g_ux = None if g_u is None else g_u[0].to(real).contiguous()
        g_uy = None if g_u is None else g_u[1].to(real).contiguous()
        mu, mu2 = lat.new_cotangent(), lat.new_cotangent()
        nseg = len(ctx.snaps)
        seg_len = [min(every, steps - s * every) for s in range(nseg)]
        # Segment buffers: every node of seg[i] is written by the recompute
        # before any read (row padding is never read), so no clearing.
        bufs = [torch.empty_like(lat.lat[0]) for _ in range(min(every, max(steps, 0)))]
        for s in range(nseg - 1, -1, -1):
            n = max(seg_len[s], 0)
            seg = [ctx.snaps[s]] + bufs[:n]
            for i in range(1, n + 1):
                lat.step_between(seg[i - 1], seg[i])
            if s == nseg - 1:
                lat.adjoint_macroscopic(seg[n], g_rho, g_ux, g_uy, mu, grad_force)
            for i in range(n, 0, -1):
                lat.adjoint_step(seg[i - 1], mu, mu2, grad_force)
                mu, mu2 = mu2, mu
        rho, ux0, uy0 = ctx.init_fields
        g_ux0 = torch.empty_like(ux0, dtype=real)
        g_uy0 = torch.empty_like(uy0, dtype=real)
        lat.adjoint_init(rho, ux0, uy0, mu, None, g_ux0, g_uy0, grad_force)
        ctx.lat = ctx.snaps = None
        return grad_force, torch.stack([g_ux0, g_uy0]), None, None, None, None


def rollout(params: Params, force: torch.Tensor, u0: torch.Tensor, steps: int,
            checkpoint_every: int = 100, rho_init: Optional[torch.Tensor] = None):
    """(rho_T [ny, nx], u_T [2, ny, nx]) after `steps` steps from the
    equilibrium state with velocity u0 and density rho_init (default rho0),
    driven by the force field `force`; differentiable in force and u0."""
    return Rollout.apply(force, u0, params, int(steps), int(checkpoint_every), rho_init)
