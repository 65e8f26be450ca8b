"""Pins of the oracle's lattice-level behaviour (no GPU).

Analytic flows of Sec. III (Taylor-Green decay, Poiseuille parabola), the
paper's grid-convergence slopes, conservation laws, the lattice symmetries
and agreement with the independent plain-definition torch formulation.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import ref_torch
from tests import analytic as A

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper_slopes():
    out = {}
    with open(os.path.join(GOLDEN, "convergence_slopes.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            prob, qty, val = line.split()[:3]
            out[(prob, qty)] = float(val)
    return out


# ----------------------------------------------------------- Taylor-Green

def test_taylor_green_64_decay():
    """Taylor-Green 64x64, tau = 0.8, u0 = 0.01, noise 1e-5, 1000 steps
    against u = -u0 cos kx sin ky exp(-2 nu k^2 t) (Sec. III).  The relative
    global error is second order in 1/N; at N = 64 it is about 1e-3."""
    n, tau = 64, 0.8
    p = oracle.Params(n, n, tau=tau)
    rho, ux, uy = W.taylor_green(n, 0.01, noise=1e-5, seed=0)
    f0 = oracle.init_state(p, rho, ux, uy)
    m0 = oracle.macroscopic(p, f0)
    # the initial state reproduces the prescribed velocity exactly
    assert np.abs(m0["ux"] - ux).max() < 1e-16 and np.abs(m0["uy"] - uy).max() < 1e-16
    m = oracle.macroscopic(p, oracle.step(p, f0, 1000))
    uxa, uya, sxxa = A.taylor_green(n, 0.01, 1000, tau)
    assert A.rel_error_vec(m["ux"], m["uy"], uxa, uya) < 2e-3
    assert A.rel_error_scalar(m["sxx"], sxxa) < 1e-3
    # kinetic energy decays as exp(-4 nu k^2 t)
    k = 2 * math.pi / n
    e0 = (m0["ux"] ** 2 + m0["uy"] ** 2).sum()
    e1 = (m["ux"] ** 2 + m["uy"] ** 2).sum()
    assert abs(e1 / e0 / math.exp(-4 * A.nu_of(tau) * k * k * 1000) - 1) < 5e-3


@pytest.mark.parametrize("mode", [1, 2])
def test_taylor_green_second_order_convergence(mode):
    """Diffusive scaling (u0 ~ 1/N, tau = 0.55 fixed, t ~ N^2) on 24^2, 48^2,
    96^2: slopes of the velocity and S_xx errors match the paper's
    (Sec. III.B: 1.99 for k = 1, 1.98 for k = 2) within 0.05."""
    gold = _paper_slopes()
    ns, eu, es = [24, 48, 96], [], []
    for n in ns:
        tau, u0 = 0.55, 0.01 * 24 / n
        k = 2 * math.pi * mode / n
        t = int(round(1.0 / (2 * k * k * A.nu_of(tau))))  # one decay time T
        p = oracle.Params(n, n, tau=tau)
        rho, ux, uy = W.taylor_green(n, u0, mode=mode)
        m = oracle.macroscopic(p, oracle.step(p, oracle.init_state(p, rho, ux, uy), t))
        uxa, uya, sxxa = A.taylor_green(n, u0, t, tau, mode)
        eu.append(A.rel_error_vec(m["ux"], m["uy"], uxa, uya))
        es.append(A.rel_error_scalar(m["sxx"], sxxa))
    key = f"taylor_green_k{mode}"
    assert abs(A.slope(ns, eu) - gold[(key, "u")]) < 0.05
    assert abs(A.slope(ns, es) - gold[(key, "sxx")]) < 0.05


# ------------------------------------------------------------- Poiseuille

def _poiseuille_steady(ny, tau, uc, nx=3, tol=1e-13, chunk=500, max_chunks=2000):
    F = W.poiseuille_force(tau, uc, ny)
    p = oracle.Params(nx, ny, tau=tau, fx=F, bc=(oracle.lbmref.PERIODIC,) * 2 + (oracle.lbmref.WALL,) * 2)
    ua = A.poiseuille(ny, F, tau)
    rho = np.ones((ny, nx))
    f = oracle.init_state(p, rho, np.repeat(ua[:, None], nx, 1), np.zeros((ny, nx)))
    prev = None
    for _ in range(max_chunks):
        f = oracle.step(p, f, chunk)
        u = oracle.macroscopic(p, f)["ux"]
        if prev is not None and np.abs(u - prev).sum() / np.abs(u).sum() < tol:
            break
        prev = u.copy()
    return u, ua, f, p


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_poiseuille_second_order_convergence(tau):
    """Poiseuille channel, halfway bounce-back walls, under diffusive scaling:
    the error against the parabola falls with slope 2.00 (Sec. III.A)."""
    gold = _paper_slopes()[("poiseuille", "u")]
    ns, errs = [16, 32, 64], []
    for ny in ns:
        u, ua, _, _ = _poiseuille_steady(ny, tau, 0.05 * 16 / ny)
        assert np.abs(u - u[:, :1]).max() < 1e-15 * ua.max() + 1e-18  # uniform in x
        errs.append(A.rel_error_scalar(u[:, 1], ua))
    assert abs(A.slope(ns, errs) - gold) < 0.05


def test_poiseuille_profile_within_paper_bound():
    """Sec. IV.A: at Re = 200 with tau = 0.55 (the figure) and N = 26 nodes
    across the channel, the maximum relative error against the parabola is
    below 0.22 %.  (Re read as u_c H / nu.)"""
    ny, tau = 26, 0.55
    uc = 200 * A.nu_of(tau) / ny
    u, ua, _, _ = _poiseuille_steady(ny, tau, uc, tol=1e-12)
    assert np.abs(u[:, 1] - ua).max() / ua.max() < 0.0022


# ---------------------------------------------------------- conservation

def test_periodic_mass_and_momentum_budget():
    """Periodic box with a uniform force: mass is constant to round-off and
    the total momentum grows by exactly N F per step."""
    n, fx, fy = 32, 2e-6, -1e-6
    p = oracle.Params(n, n, tau=0.7, omega3=1.2, omega8=0.9, fx=fx, fy=fy)
    f = oracle.init_state(p, *W.random_flow(n, n, seed=3, u_amp=0.02))
    d0 = oracle.diagnostics(p, f)
    steps = 2000
    d1 = oracle.diagnostics(p, oracle.step(p, f, steps))
    assert abs(d1[0] / d0[0] - 1) < 1e-13
    assert abs(d1[1] - (d0[1] + steps * n * n * fx)) < 1e-12 * n * n
    assert abs(d1[2] - (d0[2] + steps * n * n * fy)) < 1e-12 * n * n


def test_walls_and_lid_conserve_mass():
    """Halfway bounce-back on all four sides, lid moving: total mass is
    conserved to round-off.  The two lid terms of a lid node cancel; at the
    two top corners one diagonal link crosses two walls and carries no wall
    term (reading E6), leaving -U/6 at the left corner and +U/6 at the right
    one, which cancel in the total."""
    n = 24
    p = oracle.Params(n, n, tau=0.6, bc=(1, 1, 1, 1), wall_u=(0, 0, 0, 0.1))
    f = oracle.init_state(p, *W.at_rest(n, n, density_noise=1e-3, seed=2))
    d0 = oracle.diagnostics(p, f)
    d1 = oracle.diagnostics(p, oracle.step(p, f, 3000))
    assert abs(d1[0] / d0[0] - 1) < 1e-14


def test_lid_momentum_injection_first_step():
    """From rest, one step of the cavity gives total x-momentum (n_x - 1) U/3:
    each lid node receives 6 w (e_x U) on the two diagonal links,
    (1/36)*6*U*2 = U/3, except the two corner nodes, whose outer diagonal link
    crosses two walls and carries no term (reading E6): U/6 each.  Bounce-back
    of a rest equilibrium is neutral."""
    n, U = 16, 0.1
    p = oracle.Params(n, n, tau=0.6, bc=(1, 1, 1, 1), wall_u=(0, 0, 0, U))
    f = oracle.init_state(p, *W.at_rest(n, n))
    f1 = oracle.step(p, f, 1)
    d = oracle.diagnostics(p, f1)
    assert abs(d[1] - (n - 1) * U / 3) < 1e-15
    assert abs(d[2]) < 1e-15
    rho_top = f1[:, -1, :].sum(axis=0)  # mass moved from the left top corner to the right one
    assert abs(rho_top[0] - (1 - U / 6)) < 1e-15 and abs(rho_top[-1] - (1 + U / 6)) < 1e-15
    assert np.all(np.abs(rho_top[1:-1] - 1) < 1e-15)


# ------------------------------------------------------------- symmetries

def _mirror_x(f):
    perm = [0, 3, 2, 1, 4, 6, 5, 8, 7]
    return f[perm][:, :, ::-1].copy()


def test_cavity_mirror_symmetry():
    """The cavity with lid speed U from state f equals, mirrored in x, the
    cavity with lid speed -U from the mirrored state."""
    n = 20
    pa = oracle.Params(n, n, tau=0.56, bc=(1, 1, 1, 1), wall_u=(0, 0, 0, 0.1))
    pb = oracle.Params(n, n, tau=0.56, bc=(1, 1, 1, 1), wall_u=(0, 0, 0, -0.1))
    f = W.random_populations(n, n, seed=5)
    a = oracle.step(pa, f, 300)
    b = oracle.step(pb, _mirror_x(f), 300)
    np.testing.assert_allclose(_mirror_x(a), b, rtol=0, atol=1e-15)


def test_rotation_equivariance_periodic():
    """A 90-degree rotation (x, y) -> (-y, x) of a periodic lattice, with the
    force rotated and omega_6, omega_7 exchanged (x^2 y <-> x y^2), commutes
    with the step."""
    n = 12
    rot = [0, 2, 3, 4, 1, 6, 7, 8, 5]  # direction a -> rot[a]
    fx, fy = 1e-4, -3e-4

    def rotate(f):
        g = np.empty_like(f)
        for a in range(9):
            # g[rot[a]][y'][x'] = f[a][y][x] with x' = (-y) mod n, y' = x
            for y in range(n):
                for x in range(n):
                    g[rot[a], x, (-y) % n] = f[a, y, x]
        return g

    pa = oracle.Params(n, n, tau=0.7, omega6=0.8, omega7=1.3, fx=fx, fy=fy)
    pb = oracle.Params(n, n, tau=0.7, omega6=1.3, omega7=0.8, fx=-fy, fy=fx)
    f = W.random_populations(n, n, seed=9)
    np.testing.assert_allclose(rotate(oracle.step(pa, f, 20)), oracle.step(pb, rotate(f), 20),
                               rtol=0, atol=1e-15)


def test_translation_equivariance_periodic():
    n = 10
    p = oracle.Params(n, 7, tau=0.9, fx=1e-4)
    f = W.random_populations(n, 7, seed=11)
    a = np.roll(oracle.step(p, f, 15), (2, 3), axis=(1, 2))
    b = oracle.step(p, np.roll(f, (2, 3), axis=(1, 2)), 15)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def test_step_at_matches_full_step():
    """The sampled single-step helper agrees with the full step (walls, lid,
    force field)."""
    nx, ny = 9, 7
    frc = W.force_field(nx, ny, 1e-3, seed=1)
    p = oracle.Params(nx, ny, tau=0.6, force=frc, bc=(1, 1, 1, 1), wall_u=(0.02, -0.01, 0.03, 0.1))
    f = W.random_populations(nx, ny, seed=2)
    full = oracle.step(p, f, 1)
    xs, ys = np.meshgrid(np.arange(nx), np.arange(ny))
    got = oracle.step_at(p, f, xs.ravel(), ys.ravel())
    np.testing.assert_array_equal(got, full.reshape(9, -1).T)


# ----------------------------------------------- independent formulation

@pytest.mark.parametrize("bc,wall_u", [
    ((0, 0, 0, 0), (0, 0, 0, 0)),
    ((0, 0, 1, 1), (0, 0, 0, 0.05)),
    ((1, 1, 1, 1), (0.02, -0.03, 0.01, 0.1)),
])
def test_oracle_matches_plain_definition_torch(bc, wall_u):
    """The explicit-kernel oracle and the dense-matrix torch formulation agree
    on a small lattice with a force field, every boundary type and several
    steps (to round-off)."""
    nx, ny = 7, 6
    frc = W.force_field(nx, ny, 1e-3, seed=4)
    p = oracle.Params(nx, ny, tau=0.65, omega3=1.1, omega6=0.9, omega7=1.2, omega8=1.4,
                      force=frc, bc=bc, wall_u=wall_u)
    f = W.random_populations(nx, ny, seed=6)
    want = oracle.step(p, f, 5)
    tab = ref_torch.stream_tables(nx, ny, bc, wall_u)
    F = torch.from_numpy(frc.reshape(2, -1).T.copy())
    g = ref_torch.to_node_major(f)
    for _ in range(5):
        g = ref_torch.step(g, F, p.omegas(), tab)
    np.testing.assert_allclose(ref_torch.to_plane_major(g, nx, ny), want, rtol=0, atol=1e-14)


def test_init_matches_plain_definition_torch():
    nx, ny = 5, 4
    frc = W.force_field(nx, ny, 1e-3, seed=8)
    p = oracle.Params(nx, ny, tau=0.7, force=frc)
    rho, ux, uy = W.random_flow(nx, ny, seed=1)
    want = oracle.init_state(p, rho, ux, uy)
    got = ref_torch.init_state(*(torch.from_numpy(a.ravel().copy()) for a in (rho, ux, uy)),
                               torch.from_numpy(frc.reshape(2, -1).T.copy()))
    np.testing.assert_allclose(ref_torch.to_plane_major(got, nx, ny), want, rtol=0, atol=1e-15)
