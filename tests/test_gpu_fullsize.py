"""Full-size GPU parity on sampled nodes, at the sizes the benchmark runs
(the library picks tiles and paths by lattice size).

After a few hundred steps from the benchmark's initial state, the state f(n)
is read back, one more step is taken on the GPU (the single-step kernel), and
the oracle recomputes that step at sampled nodes (random interior nodes,
every corner, nodes on every wall and wrap edge) from the same f(n).  The
oracle works in FP64 from the values the GPU actually stored, so the
difference is the GPU's own arithmetic and storage rounding for one step:
  FP64   <= 2e-15 absolute,
  FP32   <= 1e-7 absolute (FP32 arithmetic on deviations of order 1e-2),
  16-bit <= half an ulp of the stored deviation + 1e-7 (round to nearest).

The launch the benchmark times fuses steps (four per launch in FP32 and
FP64, two in 16-bit).  At the same sizes, one fused launch is checked against
single steps bit for bit on the raw lattice buffers, and for FP32/FP64 a
four- or three-step launch from a read-back state against as many full
oracle steps.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
BCMAP = {"periodic": 0, "wall": 1}
WGT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _sample_nodes(nx, ny, count, seed):
    rng = np.random.default_rng(seed)
    xs = list(rng.integers(0, nx, count))
    ys = list(rng.integers(0, ny, count))
    for x, y in [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]:
        xs.append(x)
        ys.append(y)
    for k in range(16):  # along every edge
        t = int(rng.integers(0, nx))
        u = int(rng.integers(0, ny))
        xs += [t, t, 0, nx - 1, 1, nx - 2]
        ys += [0, ny - 1, u, u, u, u]
    return np.array(xs, dtype=np.int32), np.array(ys, dtype=np.int32)


def _check_one_step(lat, p_oracle, storage, warm, seed):
    from paper_1202_6351_amd import Lattice  # noqa: F401
    lat.step(warm)
    f_n = lat.populations().cpu().numpy()
    lat.step(1)
    nx, ny = lat.params.nx, lat.params.ny
    xs, ys = _sample_nodes(nx, ny, 3000, seed)
    got_dev = lat.populations()
    got = got_dev[:, torch.from_numpy(ys).long().cuda(), torch.from_numpy(xs).long().cuda()].cpu().numpy().T
    del got_dev
    want = oracle.step_at(p_oracle, f_n, xs, ys)
    err = np.abs(got - want)
    if storage == "fp64":
        tol = 2e-15
    elif storage == "fp32":
        tol = 1e-7
    else:
        dev = np.abs(want - WGT[None, :] * p_oracle.rho0)
        half_ulp = (2.0 ** -11 if storage == "fp16" else 2.0 ** -8) * dev
        tol = half_ulp * (1 + 1e-3) + 1e-7
    bad = err > tol
    print(f"{storage} {nx}x{ny}: max one-step error {err.max():.3e} over {len(xs)} nodes")
    assert not bad.any(), (err[bad].max(), np.argwhere(bad)[:5])


@pytest.mark.parametrize("storage", ["fp32", "fp64"])
def test_cavity_4096_sampled(storage):
    from paper_1202_6351_amd import Lattice, Params
    n = 4096
    tau = W.cavity_tau(n, 0.1, 1000.0)
    lat = Lattice(Params(n, n, tau=tau, bc=("wall",) * 4, wall_u=(0, 0, 0, 0.1), storage=storage),
                  device="cuda:0")
    lat.init_equilibrium(*W.at_rest(n, n, density_noise=1e-6, seed=2))
    p = oracle.Params(n, n, tau=tau, bc=(1, 1, 1, 1), wall_u=(0, 0, 0, 0.1))
    _check_one_step(lat, p, storage, 200, seed=1)


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_taylor_green_8192_sampled(storage):
    from paper_1202_6351_amd import Lattice, Params
    n = 8192
    lat = Lattice(Params(n, n, tau=0.8, storage=storage), device="cuda:0")
    lat.init_equilibrium(*W.taylor_green(n, 0.05, noise=1e-5, seed=0))
    p = oracle.Params(n, n, tau=0.8)
    _check_one_step(lat, p, storage, 100, seed=2)


def test_beyond_fast_path_limit_sampled():
    """FP32 16384 x 8192 (lattice 4.8 GB > 4 GiB: every wavefront takes the
    general gather), walls on y, periodic x, uniform force."""
    from paper_1202_6351_amd import Lattice, Params
    nx, ny = 16384, 8192
    kw = dict(tau=0.7, fx=1e-6, bc=("periodic", "periodic", "wall", "wall"), wall_u=(0, 0, 0, 0.05))
    lat = Lattice(Params(nx, ny, storage="fp32", **kw), device="cuda:0")
    assert lat.nbytes > (1 << 32)
    lat.init_equilibrium(*W.at_rest(nx, ny, density_noise=1e-6, seed=3))
    p = oracle.Params(nx, ny, tau=0.7, fx=1e-6, bc=(0, 0, 1, 1), wall_u=(0, 0, 0, 0.05))
    _check_one_step(lat, p, "fp32", 20, seed=3)


def _fused_equals_single(lat, group):
    """One fused launch of `group` steps = `group` single-step launches, bit
    for bit, on the raw lattice buffer."""
    snap = lat.snapshot()
    t = lat.time
    lat.step(group)
    fused = lat.current.clone()
    lat.restore(snap, t)
    for _ in range(group):
        lat.step(1)
    assert torch.equal(fused, lat.current)


@pytest.mark.parametrize("shape", [(1500, 1000), (1408, 1000), (1300, 1250), (4200, 480), (600, 2400),
                                   (150000, 9), (9, 150000)])
@pytest.mark.parametrize("case", ["cavity", "periodic", "periodic_force", "channel"])
def test_fp32_four_step_tiles_shapes(shape, case):
    """FP32 lattices above 1.2 M nodes take four steps per launch on 64 x 24
    tiles.  Shapes with ragged edges, a pitch equal to the width (1408), few
    tile rows (4200 x 480) and few tile columns (600 x 2400), and strips
    narrower than a tile's window (150000 x 9, 9 x 150000: every tile an
    edge tile, both walls of a pair inside one window, periodic sides
    wrapping several times); walls, periodic sides, uniform force: every
    launch equals four single steps bit for bit, twice in a row."""
    from paper_1202_6351_amd import Lattice, Params
    nx, ny = shape
    kw = {"cavity": dict(bc=("wall",) * 4, wall_u=(0, 0, 0, 0.1)),
          "periodic": dict(),
          "periodic_force": dict(fx=2e-6, fy=-1e-6),
          "channel": dict(bc=("periodic", "periodic", "wall", "wall"), fx=1e-6)}[case]
    lat = Lattice(Params(nx, ny, tau=0.6, storage="fp32", **kw), device="cuda:0")
    lat.init_equilibrium(*W.random_flow(nx, ny, seed=11, u_amp=0.04))
    lat.step(9)
    _fused_equals_single(lat, 4)
    lat.step(5)
    _fused_equals_single(lat, 4)


@pytest.mark.parametrize("storage,group,tol", [("fp32", 4, 4e-7), ("fp32", 3, 4e-7), ("fp64", 4, 6e-15),
                                               ("fp64", 3, 6e-15)])
def test_cavity_4096_fused_launch(storage, group, tol):
    """The benchmark's launch: cavity 4096^2, Re 1000, four steps in one
    launch after 300 warm-up steps, and the three-step launch of a
    remainder.  Bit-exact against single steps; at sampled nodes within tol
    of as many FP64 oracle steps from the same read-back state (FP32: the
    steps' FP32 rounding)."""
    from paper_1202_6351_amd import Lattice, Params
    n = 4096
    tau = W.cavity_tau(n, 0.1, 1000.0)
    lat = Lattice(Params(n, n, tau=tau, bc=("wall",) * 4, wall_u=(0, 0, 0, 0.1), storage=storage),
                  device="cuda:0")
    lat.init_equilibrium(*W.at_rest(n, n, density_noise=1e-6, seed=2))
    lat.step(300)
    _fused_equals_single(lat, group)
    f_n = lat.populations().cpu().numpy()
    lat.step(group)
    p = oracle.Params(n, n, tau=tau, bc=(1, 1, 1, 1), wall_u=(0, 0, 0, 0.1))
    want_all = oracle.step(p, f_n, group)
    del f_n
    xs, ys = _sample_nodes(n, n, 3000, seed=5)
    got = lat.populations()[:, torch.from_numpy(ys).long().cuda(), torch.from_numpy(xs).long().cuda()].cpu().numpy()
    want = want_all[:, ys, xs]
    err = np.abs(got - want)
    print(f"{storage} 4096x4096: max {group}-step error {err.max():.3e} over {len(xs)} nodes")
    assert err.max() <= tol


@pytest.mark.parametrize("shape", [(1000, 1045), (1024, 1024), (1021, 1031), (2600, 2597)])
@pytest.mark.parametrize("case", ["cavity", "periodic_force"])
def test_fp32_fused_kernels_ragged(shape, case):
    """FP32 four-, three- and two-step launches on 1000 x 1045, 1024 x 1024,
    1021 x 1031 and 2600 x 2597 (ragged in x and y but 1024^2), each
    bit-exact against single steps; the cavity case also within 4e-7 of four
    FP64 oracle steps at sampled nodes."""
    from paper_1202_6351_amd import Lattice, Params
    nx, ny = shape
    if case == "cavity":
        tau = W.cavity_tau(nx, 0.1, 1000.0)
        kw = dict(bc=("wall",) * 4, wall_u=(0, 0, 0, 0.1))
        fields = W.at_rest(nx, ny, density_noise=1e-6, seed=2)
    else:
        tau = 0.7
        kw = dict(fx=2e-6, fy=-1e-6)
        fields = W.at_rest(nx, ny, density_noise=1e-4, seed=3)
    lat = Lattice(Params(nx, ny, tau=tau, storage="fp32", **kw), device="cuda:0")
    lat.init_equilibrium(*fields)
    lat.step(30)
    _fused_equals_single(lat, 4)  # above the switch: the four-step tile launch
    _fused_equals_single(lat, 3)
    _fused_equals_single(lat, 2)  # the two-step launch of a remainder
    if case != "cavity":
        return
    group = 4
    f_n = lat.populations().cpu().numpy()
    lat.step(group)
    p = oracle.Params(nx, ny, tau=tau, bc=(1, 1, 1, 1), wall_u=(0, 0, 0, 0.1))
    want_all = oracle.step(p, f_n, group)
    del f_n
    xs, ys = _sample_nodes(nx, ny, 2000, seed=7)
    got = lat.populations()[:, torch.from_numpy(ys).long().cuda(), torch.from_numpy(xs).long().cuda()].cpu().numpy()
    err = np.abs(got - want_all[:, ys, xs])
    print(f"fp32 {nx}x{ny}: max {group}-step error {err.max():.3e} over {len(xs)} nodes")
    assert err.max() <= 4e-7


@pytest.mark.parametrize("storage,rounding", [("fp16", "nearest"), ("bf16", "stochastic")])
def test_taylor_green_8192_two_step_launch(storage, rounding):
    """The 16-bit forms' launch (two steps, Taylor-Green 8192^2) equals two
    single steps bit for bit, stochastic keys included."""
    from paper_1202_6351_amd import Lattice, Params
    n = 8192
    lat = Lattice(Params(n, n, tau=0.8, storage=storage, rounding=rounding, seed=1), device="cuda:0")
    lat.init_equilibrium(*W.taylor_green(n, 0.05, noise=1e-5, seed=0))
    lat.step(20)
    _fused_equals_single(lat, 2)

