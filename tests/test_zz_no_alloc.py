"""lbm_diagnostics_noalloc, the allocation-free variant of lbm_diagnostics
(its reduction scratch is a static device array of the library), called
through the C ABI: equal to lbm_diagnostics bit for bit on two calls in a
row, the second on a smaller lattice, and allocating no device memory."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _lattice(nx, ny, storage, bc, wu, steps):
    from paper_1202_6351_amd import Lattice, Params
    lat = Lattice(Params(nx, ny, tau=0.7, storage=storage, bc=bc, wall_u=wu), device=DEV)
    lat.set_populations(W.random_populations(nx, ny, seed=nx + ny, amp=0.05)).step(steps)
    return lat


def _noalloc(lat, out):
    from paper_1202_6351_amd import _lib
    lib = _lib.lib()
    st = lib.lbm_diagnostics_noalloc(lat._ctx, ctypes.c_void_p(out.data_ptr()))
    assert st == _lib.LBM_OK, lib.lbm_last_error(lat._ctx)
    lat.stream.synchronize()
    return out.cpu().numpy().copy()


def test_noalloc_diagnostics_equal_the_allocating_call():
    """Two calls in a row, the second on a smaller lattice (and the other
    storage), each equal to lbm_diagnostics bit for bit.  The first call on
    the device looks up the static array's address (set-up; the HIP runtime
    may reserve memory for it then); after that the calls change the
    device's free memory by nothing."""
    out = torch.full((4,), float("nan"), dtype=torch.float64, device=DEV)
    setup = _lattice(64, 64, "fp32", ("periodic",) * 4, (0, 0, 0, 0), 1)
    _noalloc(setup, out)
    cases = [(1000, 900, "fp32", ("wall",) * 4, (0.01, -0.02, 0.03, 0.1), 9),
             (70, 33, "fp64", ("periodic",) * 4, (0, 0, 0, 0), 5)]  # second call: a smaller lattice
    lats = [_lattice(*c) for c in cases]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = [_noalloc(lat, out) for lat in lats]
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0  # no device allocation
    for lat, g, c in zip(lats, got, cases):
        ref = lat.diagnostics()  # the allocating entry point (its own scratch)
        assert np.array_equal(g, ref), (c, g, ref)
        # a repeated call over the scratch the previous one left
        assert np.array_equal(_noalloc(lat, out), ref)


def test_noalloc_diagnostics_errors():
    from paper_1202_6351_amd import Lattice, Params, _lib
    lib = _lib.lib()
    lat = Lattice(Params(64, 64, tau=0.8, storage="fp32"), device=DEV)
    out = torch.zeros(4, dtype=torch.float64, device=DEV)
    assert lib.lbm_diagnostics_noalloc(lat._ctx, ctypes.c_void_p(out.data_ptr())) == _lib.LBM_ESTATE
    lat.init_equilibrium(*W.at_rest(64, 64))
    assert lib.lbm_diagnostics_noalloc(lat._ctx, None) == _lib.LBM_EINVAL
    assert lib.lbm_diagnostics_noalloc(lat._ctx, ctypes.c_void_p(out.data_ptr() + 4)) == _lib.LBM_EINVAL
    got = lat.diagnostics_noalloc(out)
    torch.cuda.synchronize()
    assert got[0].item() == 64 * 64 and got[1].item() == 0 and got[3].item() == 0
