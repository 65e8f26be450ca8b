"""GPU checks of the hand-written adjoint (through the C ABI).

* per-step dot-product tests <J v, w> = <v, J^T w> with J v from central
  finite differences of the forward step (FP64);
* the macroscopic and initial-state adjoints the same way;
* full checkpointed rollouts: directional central differences on 32x32, and
  agreement with float64 torch autograd of the independent dense-matrix
  formulation in oracle/ref_torch.py on 16x14 and 136x24 (FP64 and FP32).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import ref_torch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BCMAP = {"periodic": 0, "wall": 1}

BCS = [
    (("periodic",) * 4, (0, 0, 0, 0)),
    (("periodic", "periodic", "wall", "wall"), (0, 0, 0.0, 0.1)),
    (("wall",) * 4, (0.01, -0.02, 0.03, 0.1)),
]


def _lattice(nx, ny, force, storage="fp64", **kw):
    from paper_1202_6351_amd import Lattice, Params
    return Lattice(Params(nx, ny, storage=storage, **kw), device=DEV,
                   force=torch.from_numpy(force))


def _lattice_noise(lat, seed):
    """Random lattice-layout tensor, zero in the row padding."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    ny, nx, pitch = lat.params.ny, lat.params.nx, lat.pitch
    v = torch.zeros(9, ny, pitch, dtype=torch.float64)
    v[:, :, :nx] = torch.randn(9, ny, nx, generator=g, dtype=torch.float64)
    return v.reshape(-1).to(DEV)


def _step(lat, src):
    out = torch.zeros_like(src)
    lat.step_between(src, out)
    return out


@pytest.mark.parametrize("bci", range(len(BCS)))
@pytest.mark.parametrize("shape", [(16, 12), (67, 33)])
def test_step_adjoint_dot_product(bci, shape):
    nx, ny = shape
    bc, wu = BCS[bci]
    frc = W.force_field(nx, ny, 1e-3, seed=5)
    lat = _lattice(nx, ny, frc, tau=0.6, omega3=1.2, omega6=0.8, omega7=1.4, omega8=1.1,
                   bc=bc, wall_u=wu)
    lat.set_populations(W.random_populations(nx, ny, seed=9))
    L = lat.current.clone()
    v, w = _lattice_noise(lat, 1), _lattice_noise(lat, 2)
    eps = 1e-6
    jv = (_step(lat, L + eps * v) - _step(lat, L - eps * v)) / (2 * eps)
    mu_out = torch.zeros_like(w)
    gF = torch.zeros_like(lat.force)
    lat.adjoint_step(L, w, mu_out, gF)
    lhs, rhs = torch.dot(jv, w).item(), torch.dot(v, mu_out).item()
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs), (lhs, rhs)
    # force direction
    dF = torch.randn(lat.force.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(3)).to(DEV)
    f0 = lat.force.clone()
    lat.force.copy_(f0 + eps * dF)
    up = _step(lat, L)
    lat.force.copy_(f0 - eps * dF)
    dn = _step(lat, L)
    lat.force.copy_(f0)
    lhs = torch.dot((up - dn) / (2 * eps), w).item()
    rhs = torch.dot(dF.reshape(-1), gF.reshape(-1)).item()
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs), (lhs, rhs)


def test_step_adjoint_support():
    """With w nonzero on one element of the new lattice (node x, direction
    a), J^T w is supported exactly on the nine elements of the old lattice
    that stream into node x."""
    nx, ny = 8, 6
    frc = np.zeros((2, ny, nx))
    lat = _lattice(nx, ny, frc, tau=1.0)
    lat.init_equilibrium(*W.at_rest(nx, ny))
    L = lat.current.clone()
    w = torch.zeros_like(L)
    pitch = lat.pitch
    a, y, x = 5, 2, 3
    w[(a * ny + y) * pitch + x] = 1.0
    mu_out = torch.zeros_like(w)
    lat.adjoint_step(L, w, mu_out, None)
    nz = torch.nonzero(mu_out.reshape(9, ny, pitch)).cpu().numpy()
    # the node's populations all stream in from its 9 neighbours (x - e_a)
    ex = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    ey = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    allowed = {(b, (y - ey[b]) % ny, (x - ex[b]) % nx) for b in range(9)}
    assert {tuple(r) for r in nz} <= allowed and len(nz) > 0


def test_macroscopic_adjoint():
    nx, ny = 20, 14
    bc, wu = BCS[2]
    frc = W.force_field(nx, ny, 1e-3, seed=6)
    lat = _lattice(nx, ny, frc, tau=0.7, bc=bc, wall_u=wu)
    lat.set_populations(W.random_populations(nx, ny, seed=4))
    L = lat.current.clone()
    g = torch.Generator().manual_seed(8)
    gr, gx, gy = (torch.randn(ny, nx, dtype=torch.float64, generator=g).to(DEV) for _ in range(3))

    def J(buf):
        lat.restore(buf, 0)
        m = lat.macroscopic(strain=False)
        return (gr * m["rho"] + gx * m["ux"] + gy * m["uy"]).sum().item()

    v = _lattice_noise(lat, 3)
    eps = 1e-6
    fd = (J(L + eps * v) - J(L - eps * v)) / (2 * eps)
    mu = torch.zeros_like(L)
    gF = torch.zeros_like(lat.force)
    lat.adjoint_macroscopic(L, gr, gx, gy, mu, gF)
    assert abs(fd - torch.dot(v, mu).item()) <= 1e-8 * abs(fd)
    dF = torch.randn(lat.force.shape, dtype=torch.float64, generator=g).to(DEV)
    f0 = lat.force.clone()
    lat.force.copy_(f0 + eps * dF)
    up = J(L)
    lat.force.copy_(f0 - eps * dF)
    dn = J(L)
    lat.force.copy_(f0)
    fd = (up - dn) / (2 * eps)
    assert abs(fd - torch.dot(dF.reshape(-1), gF.reshape(-1)).item()) <= 1e-8 * abs(fd)


def test_init_adjoint():
    nx, ny = 18, 10
    bc, wu = BCS[1]
    frc = W.force_field(nx, ny, 1e-3, seed=2)
    lat = _lattice(nx, ny, frc, tau=0.7, bc=bc, wall_u=wu)
    rho, ux, uy = (torch.from_numpy(a).to(DEV) for a in W.random_flow(nx, ny, seed=3))
    w = _lattice_noise(lat, 5)

    def J(r, vx, vy):
        lat.init_equilibrium(r, vx, vy)
        return torch.dot(lat.current, w).item()

    gr, gx, gy = (torch.empty_like(rho) for _ in range(3))
    gF = torch.zeros_like(lat.force)
    lat.adjoint_init(rho, ux, uy, w, gr, gx, gy, gF)
    g = torch.Generator().manual_seed(1)
    eps = 1e-6
    for k, grad in ((0, gr), (1, gx), (2, gy)):
        d = torch.randn(ny, nx, dtype=torch.float64, generator=g).to(DEV)
        args_p = [rho, ux, uy]
        args_m = [rho, ux, uy]
        args_p = [a + eps * d if i == k else a for i, a in enumerate(args_p)]
        args_m = [a - eps * d if i == k else a for i, a in enumerate(args_m)]
        fd = (J(*args_p) - J(*args_m)) / (2 * eps)
        assert abs(fd - torch.dot(d.reshape(-1), grad.reshape(-1)).item()) <= 1e-8 * abs(fd)
    dF = torch.randn(lat.force.shape, dtype=torch.float64, generator=g).to(DEV)
    f0 = lat.force.clone()
    lat.force.copy_(f0 + eps * dF)
    up = J(rho, ux, uy)
    lat.force.copy_(f0 - eps * dF)
    dn = J(rho, ux, uy)
    lat.force.copy_(f0)
    fd = (up - dn) / (2 * eps)
    assert abs(fd - torch.dot(dF.reshape(-1), gF.reshape(-1)).item()) <= 1e-8 * abs(fd)


# ------------------------------------------------------------------ rollouts

def _tg_target(n, t, tau, u0=0.02):
    """Analytic Taylor-Green velocity at time t (the flow-matching target)."""
    import math
    k = 2 * math.pi / n
    nu = (tau - 0.5) / 3
    x = np.arange(n)[None, :]
    y = np.arange(n)[:, None]
    dec = math.exp(-2 * nu * k * k * t)
    return np.stack([-u0 * np.cos(k * x) * np.sin(k * y) * dec, u0 * np.sin(k * x) * np.cos(k * y) * dec])


def _loss_fn(target):
    def loss(u):
        return ((u - target) ** 2).sum(dim=0).mean()
    return loss


def test_rollout_finite_differences_32():
    """32x32 periodic FP64, learnable force field (N(0, 1e-6^2), seed 4) and
    initial velocity (0), Taylor-Green target at U0 = 0.02, T = 200 with a
    checkpoint every 50 steps: directional central differences."""
    from paper_1202_6351_amd import Params, rollout
    n, tau, T = 32, 0.8, 200
    p = Params(n, n, tau=tau, storage="fp64")
    target = torch.from_numpy(_tg_target(n, T, tau)).to(DEV)
    loss = _loss_fn(target)
    F = torch.from_numpy(W.force_field(n, n, 1e-6, seed=4)).to(DEV).requires_grad_(True)
    u0 = torch.zeros(2, n, n, dtype=torch.float64, device=DEV, requires_grad=True)
    _, u = rollout(p, F, u0, T, checkpoint_every=50)
    loss(u).backward()
    gF, gu0 = F.grad.clone(), u0.grad.clone()
    gen = torch.Generator().manual_seed(12)

    def L(Fv, uv):
        with torch.no_grad():
            return loss(rollout(p, Fv, uv, T, checkpoint_every=50)[1]).item()

    for which in ("F", "u0"):
        d = torch.randn(2, n, n, dtype=torch.float64, generator=gen).to(DEV)
        eps = 1e-8 if which == "F" else 1e-6
        if which == "F":
            fd = (L(F.detach() + eps * d, u0.detach()) - L(F.detach() - eps * d, u0.detach())) / (2 * eps)
            an = torch.dot(d.reshape(-1), gF.reshape(-1)).item()
        else:
            fd = (L(F.detach(), u0.detach() + eps * d) - L(F.detach(), u0.detach() - eps * d)) / (2 * eps)
            an = torch.dot(d.reshape(-1), gu0.reshape(-1)).item()
        print(f"rollout FD {which}: fd {fd:.10e} adjoint {an:.10e}")
        assert abs(fd - an) <= 1e-6 * abs(fd)
    # 20 random single entries of dL/dF
    idx = torch.randint(0, 2 * n * n, (20,), generator=gen)
    for i in idx.tolist():
        e = torch.zeros(2 * n * n, dtype=torch.float64, device=DEV)
        e[i] = 1.0
        e = e.reshape(2, n, n)
        eps = 1e-7
        fd = (L(F.detach() + eps * e, u0.detach()) - L(F.detach() - eps * e, u0.detach())) / (2 * eps)
        an = gF.reshape(-1)[i].item()
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-12 * gF.abs().max().item(), (i, fd, an)


# (nx, ny, T, checkpoint interval, storage, tolerance relative to the largest
# reference gradient entry).  16 x 14 has no tile away from the domain's
# edges; on 136 x 24 the adjoint pairs run their wall-free form on the tiles
# at x0 = 64, y0 = 4 .. 16 in FP64 (64 x 4 tiles) and at x0 = 64, y0 = 8 in
# FP32 (64 x 8), and the forward its four-step tiles (64 x 8).  FP32 bound: the FP32 forward and adjoint accumulate
# rounding of order 1e-7 per step over T = 20 steps; measured errors are
# about 1e-6 of the largest entry.
AUTOGRAD_CASES = [
    (16, 14, 30, 7, "fp64", 1e-10),
    (136, 24, 20, 7, "fp64", 1e-10),
    (136, 24, 20, 7, "fp32", 1e-4),
]


@pytest.mark.parametrize("case", range(len(AUTOGRAD_CASES)))
@pytest.mark.parametrize("bci", range(len(BCS)))
def test_rollout_matches_torch_autograd(bci, case):
    """Checkpointed rollouts (FP64, and the FP32 the benchmark runs): the
    loss and the gradients with respect to the force field and the initial
    velocity equal float64 torch autograd of the independent dense-matrix
    step on the same (storage-rounded) inputs."""
    from paper_1202_6351_amd import Params, rollout
    nx, ny, T, every, storage, tol = AUTOGRAD_CASES[case]
    tau = 0.7
    bc, wu = BCS[bci]
    kw = dict(tau=tau, omega3=1.1, omega6=0.9, omega7=1.2, omega8=1.3, bc=bc, wall_u=wu)
    p = Params(nx, ny, storage=storage, **kw)
    real = p.real_dtype
    Fn = W.force_field(nx, ny, 1e-4, seed=7)
    rho_n, ux_n, uy_n = W.random_flow(nx, ny, seed=2, u_amp=0.03, rho_amp=0.0)
    tgt = np.stack(W.random_flow(nx, ny, seed=3, u_amp=0.03)[1:])
    F = torch.from_numpy(Fn).to(DEV, real).requires_grad_(True)
    u0 = torch.from_numpy(np.stack([ux_n, uy_n])).to(DEV, real).requires_grad_(True)
    rho_T, u = rollout(p, F, u0, T, checkpoint_every=every)
    target = torch.from_numpy(tgt).to(DEV, real)
    L = ((u - target) ** 2).sum(dim=0).mean() + 0.3 * (rho_T ** 2).mean()
    L.backward()

    # reference: torch autograd on the CPU, from the inputs as the GPU saw
    # them (rounded to the compute real)
    Fq = F.detach().double().cpu().numpy()
    u0q = u0.detach().double().cpu().numpy()
    tq = target.double().cpu().numpy()
    Ft = torch.from_numpy(Fq.reshape(2, -1).T.copy()).requires_grad_(True)
    u0t = torch.from_numpy(u0q.reshape(2, -1).copy()).requires_grad_(True)
    tab = ref_torch.stream_tables(nx, ny, [BCMAP[b] for b in bc], wu)
    om = p.c()
    omega = [0, 0, 0, om.omega3, om.omega_nu, om.omega_nu, om.omega6, om.omega7, om.omega8]
    f = ref_torch.init_state(torch.ones(nx * ny, dtype=torch.float64), u0t[0], u0t[1], Ft)
    for _ in range(T):
        f = ref_torch.step(f, Ft, omega, tab)
    r, vx, vy = ref_torch.velocity(f, Ft)
    tt = torch.from_numpy(tq.reshape(2, -1))
    Lr = ((vx - tt[0]) ** 2 + (vy - tt[1]) ** 2).mean() + 0.3 * (r ** 2).mean()
    Lr.backward()
    assert abs(L.item() - Lr.item()) <= tol * abs(Lr.item())
    gF_ref = Ft.grad.T.reshape(2, ny, nx).numpy()
    gu_ref = u0t.grad.reshape(2, ny, nx).numpy()
    gF, gu = F.grad.double().cpu().numpy(), u0.grad.double().cpu().numpy()
    eF = np.abs(gF - gF_ref).max() / np.abs(gF_ref).max()
    eu = np.abs(gu - gu_ref).max() / np.abs(gu_ref).max()
    print(f"{storage} {nx}x{ny} T={T}: grad F {eF:.2e}, grad u0 {eu:.2e} (max-norm, relative)")
    assert eF <= tol and eu <= tol


@pytest.mark.parametrize("n,T", [(64, 300), (512, 60)])
def test_rollout_fp32_gradient_close_to_fp64(n, T):
    """The FP32 adjoint agrees with the FP64 one to FP32 accuracy (checkpoint
    every 100; at 512 x 512 the FP32 adjoint runs four steps per launch, the
    FP64 one pairs, so the two launch forms are tied together)."""
    from paper_1202_6351_amd import Params, rollout
    tau = 0.8
    target = _tg_target(n, T, tau)
    grads = {}
    for storage in ("fp64", "fp32"):
        real = torch.float64 if storage == "fp64" else torch.float32
        p = Params(n, n, tau=tau, storage=storage)
        F = torch.from_numpy(W.force_field(n, n, 1e-6, seed=4)).to(DEV, real).requires_grad_(True)
        u0 = torch.zeros(2, n, n, dtype=real, device=DEV, requires_grad=True)
        _, u = rollout(p, F, u0, T, checkpoint_every=100)
        ((u - torch.from_numpy(target).to(DEV)) ** 2).sum(dim=0).mean().backward()
        grads[storage] = (F.grad.double().cpu().numpy(), u0.grad.double().cpu().numpy())
    for k in range(2):
        a, b = grads["fp32"][k], grads["fp64"][k]
        rel = np.abs(a - b).sum() / np.abs(b).sum()
        print(f"fp32 vs fp64 gradient {k}: rel {rel:.3e}")
        assert rel < 1e-4


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [0, 1, 4, 6, 7])
@pytest.mark.parametrize("bci", range(len(BCS)))
@pytest.mark.parametrize("shape", [(67, 33), (200, 131), (5, 7)])
def test_sequences_equal_single_calls(storage, n, bci, shape):
    """lbm_step_sequence = n lbm_step_between calls, and lbm_adjoint_sequence
    (pairs of adjoint steps fused in one launch) = n lbm_adjoint_step calls
    newest-first, grad_force included, bit for bit.  The 5 x 7 shape puts
    wrapped copies of the same nodes into one tile window."""
    nx, ny = shape
    bc, wu = BCS[bci]
    frc = W.force_field(nx, ny, 1e-4, seed=6)
    lat = _lattice(nx, ny, frc, storage=storage, tau=0.7, omega3=1.1, bc=bc, wall_u=wu)
    lat.set_populations(W.random_populations(nx, ny, seed=8, amp=0.05))
    src = lat.snapshot()
    seq = [lat.new_lattice() for _ in range(n)]
    lat.step_sequence(src, seq)
    prev = src
    for i in range(n):
        one = _step(lat, prev)
        assert torch.equal(one, seq[i])
        prev = one
    states = [src] + seq[:-1] if n else []
    mu0 = _lattice_noise(lat, 3).to(lat.real)
    gf_a = torch.from_numpy(W.force_field(nx, ny, 1.0, seed=7)).to(DEV, lat.real)
    gf_b = gf_a.clone()
    a, b = mu0.clone(), lat.new_cotangent()
    res = lat.adjoint_sequence(states, a, b, gf_a)
    assert res is a or res is b
    mu, tmp = mu0.clone(), lat.new_cotangent()
    for i in range(n - 1, -1, -1):
        lat.adjoint_step(states[i], mu, tmp, gf_b)
        mu, tmp = tmp, mu
    assert torch.equal(res, mu)
    assert torch.equal(gf_a, gf_b)


@pytest.mark.parametrize("shape", [(801, 800), (512, 512), (700, 511)])
@pytest.mark.parametrize("bci", range(len(BCS)))
def test_adjoint_pairs_large_tiles(bci, shape):
    """FP32 adjoint pairs on 64 x 8 tiles, with 256 threads on lattices above
    600 000 nodes (801 x 800, ragged in x) and 512 threads below (512 x 512,
    the rollout benchmark's launch; 700 x 511, ragged in x and y).  These
    lattices run groups of four steps as one four-step launch (64 x 16 tiles
    above 600 000 nodes, 64 x 8 below), so seven steps are a four-step
    launch, a pair and a single step: equal to seven single adjoint steps,
    grad_force included, bit for bit."""
    (nx, ny), n = shape, 7
    bc, wu = BCS[bci]
    frc = W.force_field(nx, ny, 1e-4, seed=6)
    lat = _lattice(nx, ny, frc, storage="fp32", tau=0.7, omega3=1.1, bc=bc, wall_u=wu)
    lat.set_populations(W.random_populations(nx, ny, seed=8, amp=0.05))
    src = lat.snapshot()
    seq = [lat.new_lattice() for _ in range(n)]
    lat.step_sequence(src, seq)
    states = [src] + seq[:-1]
    mu0 = _lattice_noise(lat, 3).to(lat.real)
    gf_a = torch.from_numpy(W.force_field(nx, ny, 1.0, seed=7)).to(DEV, lat.real)
    gf_b = gf_a.clone()
    res = lat.adjoint_sequence(states, mu0.clone(), lat.new_cotangent(), gf_a)
    mu, tmp = mu0.clone(), lat.new_cotangent()
    for i in range(n - 1, -1, -1):
        lat.adjoint_step(states[i], mu, tmp, gf_b)
        mu, tmp = tmp, mu
    assert torch.equal(res, mu)
    assert torch.equal(gf_a, gf_b)


@pytest.mark.parametrize("n", [6, 9])
@pytest.mark.parametrize("shape", [(1100, 1100), (1500, 1000), (20000, 70), (700, 511), (4000, 64)])
@pytest.mark.parametrize("bci", range(len(BCS)))
def test_adjoint_quads(bci, shape, n):
    """FP32 lattices of at least 200 000 nodes (and at least 128 x 64) run
    groups of four adjoint steps as one launch (a four-node ring, three
    in-place stages in LDS), then a pair or a single step: n = 6 is a quad
    and a pair, n = 9 two quads and a single step.  64 x 16 tiles above
    600 000 nodes: ragged in x and y (1100 x 1100, 1500 x 1000) and a strip
    20000 x 70; 64 x 8 tiles below: 700 x 511 and a strip 4000 x 64.  Equal
    to n single adjoint steps, grad_force included, bit for bit."""
    (nx, ny) = shape
    bc, wu = BCS[bci]
    frc = W.force_field(nx, ny, 1e-4, seed=6)
    lat = _lattice(nx, ny, frc, storage="fp32", tau=0.7, omega3=1.1, bc=bc, wall_u=wu)
    lat.set_populations(W.random_populations(nx, ny, seed=8, amp=0.05))
    src = lat.snapshot()
    seq = [lat.new_lattice() for _ in range(n)]
    lat.step_sequence(src, seq)
    states = [src] + seq[:-1]
    mu0 = _lattice_noise(lat, 3).to(lat.real)
    gf_a = torch.from_numpy(W.force_field(nx, ny, 1.0, seed=7)).to(DEV, lat.real)
    gf_b = gf_a.clone()
    res = lat.adjoint_sequence(states, mu0.clone(), lat.new_cotangent(), gf_a)
    mu, tmp = mu0.clone(), lat.new_cotangent()
    for i in range(n - 1, -1, -1):
        lat.adjoint_step(states[i], mu, tmp, gf_b)
        mu, tmp = tmp, mu
    assert torch.equal(res, mu)
    assert torch.equal(gf_a, gf_b)


def test_handle_on_another_stream():
    """Lattice.on_stream: a context of its own over the same buffers, whose
    calls run on the given stream.  Its kept states equal the original's; it
    has no state of its own (state calls fail with LBM_ESTATE); making many
    of them allocates no device memory (the diagnostics scratch is made on
    first use)."""
    from paper_1202_6351_amd import _lib
    nx, ny = 130, 70
    bc, wu = BCS[1]
    lat = _lattice(nx, ny, W.force_field(nx, ny, 1e-4, seed=16), storage="fp32", tau=0.7, bc=bc, wall_u=wu)
    lat.set_populations(W.random_populations(nx, ny, seed=17, amp=0.05))
    src = lat.snapshot()
    ref = [lat.new_lattice() for _ in range(5)]
    lat.step_sequence(src, ref)
    side = torch.cuda.Stream()
    v = lat.on_stream(side)
    got = [lat.new_lattice() for _ in range(5)]
    torch.cuda.current_stream().synchronize()
    with torch.cuda.stream(side):
        v.step_sequence(src, got)
    side.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    with pytest.raises(_lib.LbmError) as e:
        v.step(1)
    assert e.value.status == _lib.LBM_ESTATE
    torch.cuda.synchronize()
    before = torch.cuda.mem_get_info()[0]
    views = [lat.on_stream(side) for _ in range(50)]
    assert torch.cuda.mem_get_info()[0] == before
    del views
    assert lat.diagnostics()[0] > 0  # the original's first diagnostics call makes its scratch


@pytest.mark.parametrize("pattern", ["pingpong", "cycle3", "cycle4", "cycle5"])
@pytest.mark.parametrize("storage", ["fp32", "fp64"])
def test_step_sequence_with_reused_buffers(pattern, storage):
    """lbm_step_sequence may reuse a buffer once its state has been read.  In
    FP32 lattices of up to 1.2 M nodes the library fuses groups of four steps
    (storing the three intermediate states) only when the group's five
    buffers are distinct and falls back to single steps otherwise: ping-pong
    buffers and a cycle of three never fuse, a cycle of four fuses once (the
    next group's input is its own output buffer), a cycle of five twice.
    Every buffer ends holding the state last written into it, as with single
    steps."""
    nx, ny = 130, 70
    bc, wu = BCS[2]
    lat = _lattice(nx, ny, W.force_field(nx, ny, 1e-4, seed=14), storage=storage, tau=0.65, bc=bc, wall_u=wu)
    lat.set_populations(W.random_populations(nx, ny, seed=15, amp=0.05))
    src = lat.snapshot()
    n = 8
    bufs = [lat.new_lattice() for _ in range(5)]
    idx = {"pingpong": [0, 1] * 4, "cycle3": [0, 1, 2] * 3, "cycle4": [0, 1, 2, 3] * 2,
           "cycle5": [0, 1, 2, 3, 4] * 2}[pattern][:n]
    lat.step_sequence(src, [bufs[j] for j in idx])
    prev, ref = src, []
    for _ in range(n):
        prev = _step(lat, prev)
        ref.append(prev)
    for j in set(idx):
        last = max(i for i, jj in enumerate(idx) if jj == j)
        assert torch.equal(bufs[j], ref[last]), (j, last)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("T", [0, 1, 10, 23])
def test_rollout_gradient_independent_of_checkpointing(storage, T):
    """The backward pipeline (segment recompute on a second stream, two
    alternating buffer sets) gives bit-for-bit the same gradients for every
    checkpoint interval, ragged last segments included."""
    from paper_1202_6351_amd import Params, rollout
    nx, ny = 40, 24
    bc, wu = BCS[1]
    p = Params(nx, ny, tau=0.7, bc=bc, wall_u=wu, storage=storage)
    real = p.real_dtype
    F0 = torch.from_numpy(W.force_field(nx, ny, 1e-4, seed=9)).to(DEV, real)
    u00 = torch.from_numpy(np.stack(W.random_flow(nx, ny, seed=5, u_amp=0.03)[1:])).to(DEV, real)
    w = torch.from_numpy(np.random.default_rng(2).normal(size=(2, ny, nx))).to(DEV, real)
    grads = []
    for every in (1, 2, 3, 7, 10, 11, 40):
        F = F0.clone().requires_grad_(True)
        u0 = u00.clone().requires_grad_(True)
        rho, u = rollout(p, F, u0, T, checkpoint_every=every)
        ((u * w).sum() + rho.sum()).backward()
        grads.append((F.grad.clone(), u0.grad.clone()))
    for gF, gu in grads[1:]:
        assert torch.equal(gF, grads[0][0]) and torch.equal(gu, grads[0][1])


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("T,every", [(23, 10), (20, 10), (5, 40)])
def test_rollout_forward_same_with_and_without_gradient(storage, T, every):
    """With a gradient wanted, the forward runs its last segment as a
    state-keeping sequence and restores the final state; the outputs equal
    those of the plain stepping forward bit for bit."""
    from paper_1202_6351_amd import Params, rollout
    nx, ny = 40, 24
    bc, wu = BCS[1]
    p = Params(nx, ny, tau=0.7, bc=bc, wall_u=wu, storage=storage)
    real = p.real_dtype
    F = torch.from_numpy(W.force_field(nx, ny, 1e-4, seed=9)).to(DEV, real)
    u0 = torch.from_numpy(np.stack(W.random_flow(nx, ny, seed=5, u_amp=0.03)[1:])).to(DEV, real)
    rho_a, u_a = rollout(p, F, u0, T, checkpoint_every=every)
    rho_b, u_b = rollout(p, F.clone().requires_grad_(True), u0, T, checkpoint_every=every)
    assert torch.equal(rho_a, rho_b) and torch.equal(u_a, u_b.detach())


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("bci", [0, 2])
@pytest.mark.parametrize("n", [6, 7])
@pytest.mark.parametrize("shape", [(300, 200), (1030, 1030), (1500, 1000)])
@pytest.mark.parametrize("force", ["field", "none"])
def test_step_sequence_large_shape(storage, bci, n, shape, force):
    """lbm_step_sequence on 300 x 200, 1030 x 1030 and 1500 x 1000 (FP32
    takes its 64 x 8, 64 x 12 and 64 x 24 four-step tiles that keep their
    states, interior tiles included: a group of four, then one launch cut
    short after two or three steps; FP64 runs single steps), periodic or
    walls and lid, with a force field or none: the kept states equal as many
    lbm_step_between calls bit for bit."""
    from paper_1202_6351_amd import Lattice, Params
    nx, ny = shape
    bc, wu = BCS[bci]
    if force == "field":
        lat = _lattice(nx, ny, W.force_field(nx, ny, 1e-4, seed=12), storage=storage, tau=0.6, bc=bc, wall_u=wu)
    else:
        lat = Lattice(Params(nx, ny, storage=storage, tau=0.6, bc=bc, wall_u=wu), device=DEV)
    lat.set_populations(W.random_populations(nx, ny, seed=13, amp=0.05))
    src = lat.snapshot()
    seq = [lat.new_lattice() for _ in range(n)]
    lat.step_sequence(src, seq)
    prev = src
    for i in range(n):
        one = _step(lat, prev)
        assert torch.equal(one, seq[i]), i
        prev = one



def test_rollout_backward_uses_the_forward_force():
    """The forward copies the force field: changing the caller's tensor in
    place between forward and backward leaves the gradient unchanged."""
    from paper_1202_6351_amd import Params, rollout
    nx, ny, T = 40, 24, 9
    p = Params(nx, ny, tau=0.7, storage="fp32")
    F0 = torch.from_numpy(W.force_field(nx, ny, 1e-4, seed=9)).to(DEV, torch.float32)
    u0 = torch.from_numpy(np.stack(W.random_flow(nx, ny, seed=5, u_amp=0.03)[1:])).to(DEV, torch.float32)
    w = torch.from_numpy(np.random.default_rng(2).normal(size=(2, ny, nx))).to(DEV, torch.float32)
    grads = []
    for touch in (False, True):
        F = F0.clone().requires_grad_(True)
        _, u = rollout(p, F, u0, T, checkpoint_every=4)
        if touch:
            with torch.no_grad():
                F.mul_(3.0).add_(1e-3)
        (u * w).sum().backward()
        grads.append(F.grad.clone())
    assert torch.equal(grads[0], grads[1])
