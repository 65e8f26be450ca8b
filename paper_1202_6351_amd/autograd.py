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

Memory: the forward keeps a lattice snapshot every `checkpoint_every` steps,
and, when a gradient is wanted, every state of the last segment (it runs
that segment as one state-keeping sequence, so the backward can start its
adjoint at once).  The backward recomputes each older segment's states from
its snapshot and runs the adjoint over them newest-first.  The recompute of
the next (older) segment runs on one stream while the adjoint of the current
one runs on another, so the two kernels share the GPU; they alternate
between two sets of lattice buffers (the forward's set and one more of
`checkpoint_every - 1`), each set one allocation.  Both streams are ordinary streams
kept per device (not the legacy default stream, whose implicit
synchronisation with other streams serialised the two).  Work per step of
the backward: one recomputed step and one adjoint step.
"""
from __future__ import annotations

from typing import Optional

import torch

from .lattice import Lattice, Params


_BACKWARD_STREAMS = {}


def _lattice_set(lat: Lattice, count: int):
    """(base tensor, list of `count` lattice buffers): views of one
    allocation, each at a multiple of the lattice size (a multiple of 256
    bytes, since the pitch is a multiple of 64 nodes)."""
    if count <= 0:
        return None, []
    base = torch.empty((count, lat.lat[0].numel()), dtype=lat.lat[0].dtype, device=lat.device)
    return base, [base[i] for i in range(count)]


def _backward_streams(dev: torch.device):
    """(adjoint stream, recompute stream) of a device, created once."""
    key = dev.index if dev.index is not None else torch.cuda.current_device()
    if key not in _BACKWARD_STREAMS:
        _BACKWARD_STREAMS[key] = (torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev))
    return _BACKWARD_STREAMS[key]


def _backward_setup(lat: Lattice, width: int, nseg: int):
    """What the backward needs besides the forward's results: the two
    streams and a library context on each, the cotangent pair, the force
    gradient, the initial-velocity gradient and the second set of segment
    buffers.  Made at the end of the forward when a gradient is wanted, while
    the GPU still runs the forward's steps, so that the host work of the
    backward's start is hidden."""
    p, dev, real = lat.params, lat.device, lat.real
    main, side = _backward_streams(dev)
    set1_base, set1 = _lattice_set(lat, width if nseg > 1 else 0)
    return dict(main=main, side=side, adj=lat.on_stream(main), rec=lat.on_stream(side),
                mu=lat.new_cotangent(), mu2=lat.new_cotangent(),
                grad_force=torch.zeros((2, p.ny, p.nx), dtype=real, device=dev),
                g_u0=torch.empty((2, p.ny, p.nx), dtype=real, device=dev),
                set1_base=set1_base, set1=set1)


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
        # a copy: the backward works with the force field of the forward, even
        # if the caller changes its tensor in place in between
        lat = Lattice(params, device=dev, force=force.detach().to(device=dev, dtype=real, copy=True))
        f64 = torch.float64
        rho = (torch.full((ny, nx), params.rho0, dtype=f64, device=dev) if rho_init is None
               else rho_init.detach().to(dtype=f64).contiguous())
        ux0 = u0[0].detach().to(dtype=f64).contiguous()
        uy0 = u0[1].detach().to(dtype=f64).contiguous()
        lat.init_equilibrium(rho, ux0, uy0)
        nseg = max(1, -(-steps // every))
        snap_base, snaps = _lattice_set(lat, nseg)
        keep_base, keep = None, []
        for s in range(nseg):
            lat.snapshot(snaps[s])
            n = min(every, steps - s * every)
            if n <= 0:
                break
            if s == nseg - 1 and any(ctx.needs_input_grad[:2]):
                # the last segment keeps its states for the backward; its
                # final state becomes the lattice's current state.  The set
                # later serves the backward's recomputes of older segments
                # (every - 1 states each).
                keep_base, keep = _lattice_set(lat, n if nseg == 1 else max(n, every - 1))
                lat.step_sequence(snaps[s], keep[:n])
                lat.restore(keep[n - 1], steps)
            else:
                lat.step(n)
        m = lat.macroscopic(strain=False)
        ctx.lat, ctx.snaps, ctx.steps, ctx.every = lat, snaps, steps, every
        ctx.bases = (snap_base, keep_base)
        ctx.keep = keep
        ctx.init_fields = (rho, ux0, uy0)
        ctx.prep = (_backward_setup(lat, max(min(every, steps) - 1, 0), nseg)
                    if any(ctx.needs_input_grad[:2]) else None)
        return m["rho"], torch.stack([m["ux"], m["uy"]])

    @staticmethod
    def backward(ctx, g_rho, g_u):
        lat: Lattice = ctx.lat
        steps, every = ctx.steps, ctx.every
        dev, real = lat.device, lat.real
        snaps = ctx.snaps
        nseg = len(snaps)
        seg_len = [max(min(every, steps - s * every), 0) for s in range(nseg)]
        width = max(min(every, max(steps, 0)) - 1, 0)
        prep = ctx.prep if ctx.prep is not None else _backward_setup(lat, width, nseg)
        g_rho = None if g_rho is None else g_rho.to(real).contiguous()
        g_ux = None if g_u is None else g_u[0].to(real).contiguous()
        g_uy = None if g_u is None else g_u[1].to(real).contiguous()
        mu, mu2, grad_force, g_u0 = prep["mu"], prep["mu2"], prep["grad_force"], prep["g_u0"]
        # set 0: the forward's kept states of the last segment; set 1: new
        sets = [ctx.keep, prep["set1"]]
        rho, ux0, uy0 = ctx.init_fields
        # Adjoint calls run on `main`, recomputes on `side`, each through a
        # context of its own over the forward's buffers and force field.  A
        # segment of n steps needs its snapshot and the n - 1 states after
        # it; the state after the last step of the last segment is the
        # forward lattice's current state.  Both streams start after the
        # forward's stream (snapshots, final state) and the caller's (the
        # loss cotangents and every buffer allocated above).
        caller = torch.cuda.current_stream(dev)
        main, side, adj, rec = prep["main"], prep["side"], prep["adj"], prep["rec"]
        for st in (main, side):
            st.wait_stream(lat.stream)
            st.wait_stream(caller)
        for t in (*ctx.bases, prep["set1_base"], lat.force, lat.current, grad_force, mu, mu2, g_rho, g_ux, g_uy,
                  g_u0, rho, ux0, uy0):
            if t is not None:
                t.record_stream(side)
                t.record_stream(main)
        ready = [torch.cuda.Event(), torch.cuda.Event()]
        free = [None, None]

        def recompute(s, b):
            # issued with `side` current, so the call orders itself by these
            # events only and does not make the main stream wait for it
            with torch.cuda.stream(side):
                if free[b] is not None:
                    side.wait_event(free[b])  # the adjoint that read this set is done
                rec.step_sequence(snaps[s], sets[b][:max(seg_len[s] - 1, 0)])
                ready[b].record(side)

        # the last segment's states were kept by the forward
        with torch.cuda.stream(main):
            for k, s in enumerate(range(nseg - 1, -1, -1)):
                b = k % 2
                if s > 0:
                    recompute(s - 1, 1 - b)
                if k > 0:  # set 0 of the first segment: ordered by the forward's stream
                    main.wait_event(ready[b])
                n = seg_len[s]
                states = [snaps[s]] + sets[b][:max(n - 1, 0)]
                if s == nseg - 1:
                    adj.adjoint_macroscopic(lat.current, g_rho, g_ux, g_uy, mu, grad_force)
                if adj.adjoint_sequence(states[:n], mu, mu2, grad_force) is mu2:
                    mu, mu2 = mu2, mu
                free[b] = torch.cuda.Event()
                free[b].record(main)
            main.wait_stream(side)
            adj.adjoint_init(rho, ux0, uy0, mu, None, g_u0[0], g_u0[1], grad_force)
        caller.wait_stream(main)
        ctx.lat = ctx.snaps = ctx.keep = ctx.bases = ctx.prep = None
        return grad_force, g_u0, None, None, None, None


def rollout(params: Params, force: torch.Tensor, u0: torch.Tensor, steps: int,
            checkpoint_every: int = 100, rho_init: Optional[torch.Tensor] = None):
    """(rho_T [ny, nx], u_T [2, ny, nx]) after `steps` steps from the
    equilibrium state with velocity u0 and density rho_init (default rho0),
    driven by the force field `force`; differentiable in force and u0."""
    return Rollout.apply(force, u0, params, int(steps), int(checkpoint_every), rho_init)
