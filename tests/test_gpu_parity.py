"""GPU parity of the HIP step (through the C ABI) against the FP64 oracle.

Tolerances: velocity relative global error (the Sec. III norm) <= 1e-12 for
FP64 and <= 1e-5 for FP32; populations element by element where the state is
arbitrary.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests import analytic as A

pytestmark = pytest.mark.gpu

BCMAP = {"periodic": 0, "wall": 1}


def _lattice(nx, ny, storage="fp64", force=None, **kw):
    from paper_1202_6351_amd import Lattice, Params
    return Lattice(Params(nx, ny, storage=storage, **kw), device="cuda:0",
                   force=None if force is None else torch.from_numpy(force))


def _oracle_params(nx, ny, force=None, **kw):
    kw = dict(kw)
    kw.pop("storage", None)
    bc = kw.pop("bc", ("periodic",) * 4)
    return oracle.Params(nx, ny, force=force, bc=tuple(BCMAP[b] for b in bc), **kw)


def _np(d):
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in d.items()}


def _vel_err(g, o):
    return A.rel_error_vec(g["ux"], g["uy"], o["ux"], o["uy"])


# --------------------------------------------------------------- Taylor-Green

@pytest.mark.parametrize("storage,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_taylor_green_64(storage, tol):
    """64x64 periodic, tau 0.8, U0 0.01, noise 1e-5 (seed 0), 1000 steps."""
    n, tau, steps = 64, 0.8, 1000
    rho, ux, uy = W.taylor_green(n, 0.01, noise=1e-5, seed=0)
    lat = _lattice(n, n, storage, tau=tau)
    g = _np(lat.init_equilibrium(rho, ux, uy).step(steps).macroscopic())
    p = _oracle_params(n, n, tau=tau)
    o = oracle.macroscopic(p, oracle.step(p, oracle.init_state(p, rho, ux, uy), steps))
    err = _vel_err(g, o)
    print(f"taylor-green 64 {storage}: velocity rel err {err:.3e}")
    assert err <= tol
    assert A.rel_error_scalar(g["sxx"], o["sxx"]) <= 100 * tol
    assert lat.time == steps


# --------------------------------------------------- arbitrary states, shapes

SHAPES = [(64, 64), (67, 33), (2, 2), (3, 200), (300, 5), (129, 130), (256, 3)]
BCS = [
    (("periodic",) * 4, (0, 0, 0, 0)),
    (("periodic", "periodic", "wall", "wall"), (0, 0, 0.02, 0.1)),
    (("wall", "wall", "periodic", "periodic"), (-0.05, 0.03, 0, 0)),
    (("wall",) * 4, (0.01, -0.02, 0.03, 0.1)),
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bci", range(len(BCS)))
def test_random_state_fp64_populations(shape, bci):
    """Arbitrary non-equilibrium state, per-node force field, every boundary
    kind: populations after 1 and 5 steps equal the oracle's to round-off."""
    nx, ny = shape
    bc, wu = BCS[bci]
    frc = W.force_field(nx, ny, 1e-3, seed=nx * 7 + ny)
    kw = dict(tau=0.62, omega3=1.1, omega6=0.9, omega7=1.3, omega8=1.2, bc=bc, wall_u=wu)
    f0 = W.random_populations(nx, ny, seed=nx + 1000 * ny + bci)
    lat = _lattice(nx, ny, "fp64", force=frc, **kw)
    lat.set_populations(f0)
    back = lat.populations().cpu().numpy()
    np.testing.assert_allclose(back, f0, rtol=0, atol=1e-16)
    p = _oracle_params(nx, ny, force=frc, **kw)
    for steps in (1, 4):
        lat.step(steps)
        got = lat.populations().cpu().numpy()
        f0 = oracle.step(p, f0, steps)
        np.testing.assert_allclose(got, f0, rtol=0, atol=2e-15)


@pytest.mark.parametrize("shape", [(64, 64), (67, 33), (3, 200), (129, 130)])
def test_random_state_fp32_populations(shape):
    nx, ny = shape
    bc, wu = BCS[3]
    frc = W.force_field(nx, ny, 1e-3, seed=3)
    kw = dict(tau=0.7, omega3=1.0, bc=bc, wall_u=wu)
    f0 = W.random_populations(nx, ny, seed=11, amp=0.05)
    lat = _lattice(nx, ny, "fp32", force=frc, **kw)
    lat.set_populations(f0).step(3)
    got = lat.populations().cpu().numpy()
    want = oracle.step(_oracle_params(nx, ny, force=frc, **kw), f0, 3)
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-7)


# ------------------------------------------------------- Poiseuille and cavity

@pytest.mark.parametrize("storage,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0])
def test_poiseuille_256x64(storage, tol, tau):
    """Channel 256x64, halfway bounce-back at y, periodic x, F_x for centre
    speed 0.05, from rest, 4000 steps."""
    nx, ny, steps = 256, 64, 4000
    F = W.poiseuille_force(tau, 0.05, ny)
    kw = dict(tau=tau, fx=F, bc=("periodic", "periodic", "wall", "wall"))
    rho, ux, uy = W.at_rest(nx, ny)
    g = _np(_lattice(nx, ny, storage, **kw).init_equilibrium(rho, ux, uy).step(steps).macroscopic())
    p = _oracle_params(nx, ny, **kw)
    o = oracle.macroscopic(p, oracle.step(p, oracle.init_state(p, rho, ux, uy), steps))
    err = _vel_err(g, o)
    print(f"poiseuille tau {tau} {storage}: velocity rel err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("shape", [(64, 64), (96, 80)])
def test_cavity(storage, tol, shape):
    """Lid-driven cavity, lid 0.1, walls elsewhere, density noise 1e-6."""
    nx, ny = shape
    steps = 2000
    kw = dict(tau=W.cavity_tau(nx, 0.1, 100.0), bc=("wall",) * 4, wall_u=(0, 0, 0, 0.1))
    rho, ux, uy = W.at_rest(nx, ny, density_noise=1e-6, seed=2)
    lat = _lattice(nx, ny, storage, **kw).init_equilibrium(rho, ux, uy).step(steps)
    g = _np(lat.macroscopic())
    p = _oracle_params(nx, ny, **kw)
    f = oracle.step(p, oracle.init_state(p, rho, ux, uy), steps)
    o = oracle.macroscopic(p, f)
    err = _vel_err(g, o)
    print(f"cavity {shape} {storage}: velocity rel err {err:.3e}")
    assert err <= tol
    for k in ("sxx", "syy", "sxy"):
        assert A.rel_error_scalar(g[k], o[k]) <= 100 * tol
    d = lat.diagnostics()
    do = oracle.diagnostics(p, f)
    assert abs(d[0] - do[0]) <= 1e-13 * do[0] if storage == "fp64" else abs(d[0] - do[0]) <= 1e-6 * do[0]
    np.testing.assert_allclose(d[1:], do[1:], rtol=100 * tol, atol=1e-12 * nx * ny)


# ------------------------------------------------------------- state handling

@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
def test_restart_is_bit_exact(storage):
    """2n steps equal n steps, snapshot, restore into a fresh lattice, n steps."""
    n = 40
    rho, ux, uy = W.taylor_green(96, 0.03, noise=1e-4, seed=1, ny=72)
    kw = dict(tau=0.7, bc=("periodic", "periodic", "wall", "wall"), wall_u=(0, 0, 0, 0.05))
    a = _lattice(96, 72, storage, **kw).init_equilibrium(rho, ux, uy).step(2 * n)
    b = _lattice(96, 72, storage, **kw).init_equilibrium(rho, ux, uy).step(n)
    snap = b.snapshot()
    c = _lattice(96, 72, storage, **kw)
    c.restore(snap, n)
    c.step(n)
    assert c.time == 2 * n
    assert torch.equal(a.populations(), c.populations())


def test_errors_reported():
    from paper_1202_6351_amd import _lib
    lat = _lattice(32, 32, "fp16", tau=0.8)
    with pytest.raises(_lib.LbmError) as ei:
        lat.step(1)
    assert ei.value.status == _lib.LBM_ESTATE
    lat.init_equilibrium(*W.at_rest(32, 32))
    mu = torch.zeros(9 * 32 * lat.pitch, dtype=torch.float32, device="cuda:0")
    with pytest.raises(_lib.LbmError) as ei:
        lat.adjoint_step(lat.current, mu, mu.clone())
    assert ei.value.status == _lib.LBM_EUNSUPPORTED


def test_diagnostics_detect_instability():
    """A NaN planted in the lattice makes lbm_diagnostics return
    LBM_EUNSTABLE."""
    from paper_1202_6351_amd import _lib
    lat = _lattice(64, 64, "fp32", tau=0.8).init_equilibrium(*W.at_rest(64, 64))
    lat.current[1000] = float("nan")
    with pytest.raises(_lib.LbmError) as ei:
        lat.diagnostics()
    assert ei.value.status == _lib.LBM_EUNSTABLE


# ------------------------------------------- multi-step (temporal) kernels

@pytest.mark.parametrize("storage,rounding", [("fp64", "nearest"), ("fp32", "nearest"), ("fp16", "nearest"),
                                              ("bf16", "nearest"), ("fp16", "stochastic"),
                                              ("bf16", "stochastic")])
@pytest.mark.parametrize("shape", [(2, 2), (3, 200), (300, 5), (67, 33), (130, 70), (200, 131)])
@pytest.mark.parametrize("bci", [0, 1, 3])
@pytest.mark.parametrize("force", ["none", "uniform", "field"])
@pytest.mark.parametrize("n", [5, 7])
def test_multi_step_launch_equals_single_steps(storage, rounding, shape, bci, force, n):
    """lbm_step(n) fuses steps in launches of four (FP64, FP32: 5 = 4 + 1,
    7 = 4 + 3) or two (16-bit: 5 = 2 + 2 + 1, 7 = 2 + 2 + 2 + 1), the
    intermediate states kept in LDS; it must give bit-for-bit the state of n
    single-step launches.  The rates omega_6, omega_7 differ from 1, so the
    fused kernels take their general collision (the default rates take the
    variant without those multiplies, covered by the full-size tests)."""
    from paper_1202_6351_amd import Lattice, Params
    nx, ny = shape
    bc, wu = BCS[bci]
    frc = W.force_field(nx, ny, 1e-4, seed=3) if force == "field" else None
    kw = dict(tau=0.7, omega3=1.1, omega6=0.9, omega7=1.2, bc=bc, wall_u=wu, storage=storage,
              rounding=rounding, seed=5)
    if force == "uniform":
        kw.update(fx=2e-5, fy=-1e-5)
    f0 = W.random_populations(nx, ny, seed=nx * 3 + ny, amp=0.05)
    a = Lattice(Params(nx, ny, **kw), device="cuda:0", force=None if frc is None else torch.from_numpy(frc))
    a.set_populations(f0).step(n)
    b = Lattice(Params(nx, ny, **kw), device="cuda:0", force=None if frc is None else torch.from_numpy(frc))
    b.set_populations(f0)
    for _ in range(n):
        b.step(1)  # a count of one always runs the single-step kernel
    assert a.time == n and b.time == n
    assert torch.equal(a.populations(), b.populations())


@pytest.mark.parametrize("storage,rounding", [("fp64", "nearest"), ("fp32", "nearest"), ("fp16", "nearest"),
                                              ("bf16", "stochastic")])
@pytest.mark.parametrize("shape", [(200, 131), (1030, 1030), (1500, 1000)])
@pytest.mark.parametrize("bci", [0, 3])
def test_force_field_fused_default_rates(storage, rounding, shape, bci):
    """A force field with the default rates (omega_6 = omega_7 = omega_8 = 1,
    the collision variant without those multiplies).  Interior tiles read the
    field in every stage through a buffer descriptor, edge tiles through the
    general path; the shapes give FP32 its 64 x 8, 64 x 12 and 64 x 24
    four-step tiles.  lbm_step(7) equals seven single steps bit for bit."""
    from paper_1202_6351_amd import Lattice, Params
    nx, ny = shape
    bc, wu = BCS[bci]
    frc = torch.from_numpy(W.force_field(nx, ny, 1e-4, seed=21))
    kw = dict(tau=0.6, bc=bc, wall_u=wu, storage=storage, rounding=rounding, seed=3)
    f0 = W.random_populations(nx, ny, seed=17, amp=0.05)
    a = Lattice(Params(nx, ny, **kw), device="cuda:0", force=frc)
    a.set_populations(f0).step(7)
    b = Lattice(Params(nx, ny, **kw), device="cuda:0", force=frc)
    b.set_populations(f0)
    for _ in range(7):
        b.step(1)
    assert torch.equal(a.populations(), b.populations())


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("bci", [0, 1, 3])
@pytest.mark.parametrize("force", ["none", "field"])
def test_multi_step_launch_large_shape(storage, bci, force):
    """1030 x 1030 (ragged against every tile size; above a million nodes,
    where FP64 takes its large three-step shape and FP32 its 64 x 12
    four-step tiles): seven steps (a four-step and a three-step launch),
    bit-for-bit seven single steps."""
    from paper_1202_6351_amd import Lattice, Params
    nx = ny = 1030
    bc, wu = BCS[bci]
    frc = W.force_field(nx, ny, 1e-4, seed=4) if force == "field" else None
    kw = dict(tau=0.6, omega3=1.1, omega6=0.9, omega7=1.2, bc=bc, wall_u=wu, storage=storage)
    f0 = W.random_populations(nx, ny, seed=11, amp=0.05)
    mk = lambda: Lattice(Params(nx, ny, **kw), device="cuda:0",
                         force=None if frc is None else torch.from_numpy(frc)).set_populations(f0)
    a = mk().step(7)
    b = mk()
    for _ in range(7):
        b.step(1)
    assert torch.equal(a.populations(), b.populations())



def test_lattice_on_its_own_stream():
    """A Lattice bound to a stream other than the caller's: its outputs are
    ordered before the caller's stream reads them, and the caller's inputs
    before the library reads them."""
    from paper_1202_6351_amd import Lattice, Params
    n = 256
    p = Params(n, n, tau=0.7, bc=("wall",) * 4, wall_u=(0, 0, 0, 0.05), storage="fp32")
    ref = Lattice(p, device="cuda:0").init_equilibrium(*W.at_rest(n, n, density_noise=1e-4, seed=1)).step(200)
    side = torch.cuda.Stream()
    lat = Lattice(p, device="cuda:0", stream=side)
    rho, ux, uy = (torch.from_numpy(a).cuda() for a in W.at_rest(n, n, density_noise=1e-4, seed=1))
    lat.init_equilibrium(rho, ux, uy).step(200)
    m, mr = lat.macroscopic(), ref.macroscopic()
    for k in mr:
        assert torch.equal(m[k], mr[k]), k
    assert torch.equal(lat.populations(), ref.populations())
