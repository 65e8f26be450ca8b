"""The kernels never read a lattice row's padding (x = nx .. pitch - 1).

Both ping-pong buffers get NaN in every padding element after the state is
set; the run must then equal, bit for bit, a run whose padding holds zeros,
through every launch form (four-, three-, two- and single-step launches, the
state-keeping sequence, the macroscopic and diagnostics kernels).  A read of
one padding element anywhere would carry a NaN into the state or the sums.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

BCS = [
    (("periodic",) * 4, (0, 0, 0, 0)),
    (("wall",) * 4, (0.01, -0.02, 0.03, 0.1)),
]


def _lattice(nx, ny, storage, bc, wu, force):
    from paper_1202_6351_amd import Lattice, Params
    return Lattice(Params(nx, ny, tau=0.62, omega3=1.1, storage=storage, bc=bc, wall_u=wu), device=DEV,
                   force=None if force is None else torch.from_numpy(force))


def _poison(lat, value):
    for buf in lat.lat:
        v = buf.view(9, lat.params.ny, lat.pitch)
        v[:, :, lat.params.nx:] = value


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("bci", range(len(BCS)))
@pytest.mark.parametrize("shape", [(100, 70), (1000, 1100)])
def test_nan_in_row_padding_is_never_read(storage, bci, shape):
    nx, ny = shape
    bc, wu = BCS[bci]
    frc = W.force_field(nx, ny, 1e-4, seed=3) if storage in ("fp64", "fp32") else None
    f0 = W.random_populations(nx, ny, seed=11, amp=0.05)
    runs = []
    for pad in (0.0, math.nan):
        lat = _lattice(nx, ny, storage, bc, wu, frc)
        assert lat.pitch > nx
        lat.set_populations(f0)
        _poison(lat, pad)
        out = {}
        for n in (4, 3, 2, 1, 7):  # every launch form
            lat.step(n)
            out[f"f{n}"] = lat.populations()
        m = lat.macroscopic()
        out.update(m)
        out["diag"] = torch.from_numpy(lat.diagnostics())
        if storage in ("fp64", "fp32"):
            src = lat.snapshot()
            seq = [lat.new_lattice() for _ in range(5)]
            for s in seq:
                s.view(9, ny, lat.pitch)[:, :, nx:] = pad
            lat.step_sequence(src, seq)
            out["seq"] = torch.stack([s.view(9, ny, lat.pitch)[:, :, :nx].double() for s in seq])
        torch.cuda.synchronize()
        runs.append({k: v.cpu() for k, v in out.items()})
    clean, poisoned = runs
    for k in clean:
        assert torch.isfinite(poisoned[k]).all(), k
        assert torch.equal(clean[k], poisoned[k]), k
