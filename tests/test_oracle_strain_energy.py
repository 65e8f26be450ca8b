"""Pins of the oracle's strain-rate outputs (S_xx, S_yy, S_xy) and of the
energy sum of its diagnostics (no GPU).

The strain rate comes from the non-equilibrium second moments (Sec. II,
strain-rate relations, combined for omega_3 != omega_4):
    d_x j_x = -3/4 (omega_3 f3neq + omega_4 f4neq),
    d_y j_y = -3/4 (omega_3 f3neq - omega_4 f4neq),
    d_x j_y + d_y j_x = -3 omega_5 f5neq.
Each flow below fixes one part of that by an analytic solution or an exact
symmetry, at the paper's default rates (omega_3 = 1 != omega_4 = 1/tau):

  * Taylor-Green (Sec. III.B): S_yy = dv/dy = -S_xx analytically and
    S_xy = 0.  A wrong sign on the omega_4 term of d_y j_y gives S_yy = +S_xx.
  * Shear wave u = U0 sin(ky), v = 0 (an exact solution of the incompressible
    equations, decaying as exp(-nu k^2 t)): S_xy = U0 k cos(ky) / 2 times the
    decay.  A dropped or doubled factor 1/2 in S_xy, or a sign error, fails.
  * Poiseuille channel with halfway bounce-back (Sec. III.A): 2 S_xy =
    du/dy = F/(2 rho0 nu) (H - 2 y_hat) at steady state.
  * Longitudinal wave u = U0 sin(kx), v = 0: nothing depends on y, so
    d_y j_y = 0 exactly and S_yy must vanish against S_xx, which equals the
    central difference of j_x over rho up to the method's small higher-order
    terms.  A wrong sign on the omega_3 term of either relation breaks one of
    the two (the omega_3 and omega_4 terms are then equal and opposite).
  * Energy 1/2 sum rho |u|^2 of the Taylor-Green vortex: rho0 U0^2 N^2 / 4
    at t = 0 and decaying as exp(-4 nu k^2 t).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tests import analytic as A
from tests.test_oracle_lattice import _poiseuille_steady


def _grid(n):
    x = np.ones((n, 1)) * np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(n, dtype=np.float64)[:, None] * np.ones((1, n))
    return x, y


@pytest.fixture(scope="module")
def taylor_green_64():
    """Taylor-Green 64^2, tau = 0.8, U0 = 0.01, noise 1e-5, after 1000 steps."""
    n, tau, steps = 64, 0.8, 1000
    p = oracle.Params(n, n, tau=tau)
    f0 = oracle.init_state(p, *W.taylor_green(n, 0.01, noise=1e-5, seed=0))
    return p, f0, oracle.step(p, f0, steps), steps


def test_taylor_green_syy_is_minus_sxx(taylor_green_64):
    p, _, f, steps = taylor_green_64
    m = oracle.macroscopic(p, f)
    _, _, sxxa = A.taylor_green(p.nx, 0.01, steps, p.tau)
    # same second-order error as S_xx itself (3e-4 here)
    assert A.rel_error_scalar(m["syy"], -sxxa) < 1e-3
    assert A.rel_error_scalar(m["sxx"], sxxa) < 1e-3
    # S_xy vanishes analytically; the noise leaves ~1e-4 of |S_xx|
    assert np.abs(m["sxy"]).max() < 1e-3 * np.abs(sxxa).max()


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
def test_shear_wave_sxy(tau):
    n, u0, steps = 64, 0.01, 500
    k = 2 * math.pi / n
    _, y = _grid(n)
    p = oracle.Params(n, n, tau=tau)
    ux = u0 * np.sin(k * y)
    f = oracle.step(p, oracle.init_state(p, np.ones((n, n)), ux, np.zeros((n, n))), steps)
    m = oracle.macroscopic(p, f)
    dec = math.exp(-A.nu_of(tau) * k * k * steps)
    # measured 3e-4 .. 8e-4 (second order in k)
    assert A.rel_error_scalar(m["ux"], ux * dec) < 2e-3
    assert A.rel_error_scalar(m["sxy"], 0.5 * u0 * k * np.cos(k * y) * dec) < 2e-3
    # no normal strain in a pure shear flow (measured: S_yy 1e-7 and S_xx,
    # an O(U0^2) term of the decaying rho u_x^2, 2e-4 .. 5e-4 of |S_xy|)
    assert np.abs(m["sxx"]).max() < 2e-3 * np.abs(m["sxy"]).max()
    assert np.abs(m["syy"]).max() < 1e-5 * np.abs(m["sxy"]).max()


@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_poiseuille_shear_rate(tau):
    ny = 32
    u, ua, f, p = _poiseuille_steady(ny, tau, 0.05, tol=1e-12)
    m = oracle.macroscopic(p, f)
    yh = np.arange(ny, dtype=np.float64) + 0.5
    shear = p.fx / (2 * p.rho0 * A.nu_of(tau)) * (ny - 2 * yh)
    # the shear of the parabola is linear, so the method carries it exactly
    # (measured 4e-7 and 5e-13)
    for col in range(p.nx):
        assert A.rel_error_scalar(2 * m["sxy"][:, col], shear) < 1e-5
    assert np.abs(m["syy"]).max() < 1e-12 * np.abs(shear).max()


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
def test_longitudinal_wave_normal_strain(tau):
    n, u0, steps = 64, 0.01, 60
    k = 2 * math.pi / n
    x, _ = _grid(n)
    p = oracle.Params(n, n, tau=tau)
    f = oracle.step(p, oracle.init_state(p, np.ones((n, n)), u0 * np.sin(k * x), np.zeros((n, n))), steps)
    m = oracle.macroscopic(p, f)
    j = m["rho"] * m["ux"]
    fd = (np.roll(j, -1, axis=1) - np.roll(j, 1, axis=1)) / 2 / m["rho"]
    # measured 0.8 % .. 1.3 % (acoustic wave: higher-order terms at k tau)
    assert A.rel_error_scalar(m["sxx"], fd) < 0.05
    # measured 0.14 % of max |S_xx|; a sign error on omega_3 gives 100 %
    assert np.abs(m["syy"]).max() < 0.01 * np.abs(m["sxx"]).max()
    assert np.abs(m["sxy"]).max() < 1e-12 * np.abs(m["sxx"]).max()


def test_taylor_green_energy_sum(taylor_green_64):
    p, f0, f, steps = taylor_green_64
    n, u0 = p.nx, 0.01
    e0 = p.rho0 * u0 * u0 * n * n / 4
    k = 2 * math.pi / n
    d0 = oracle.diagnostics(p, f0)
    d1 = oracle.diagnostics(p, f)
    # t = 0: the analytic field (the seeded 1e-5 noise moves it by 4e-5)
    assert abs(d0[3] / e0 - 1) < 5e-4
    # t = 1000: the exp(-4 nu k^2 t) decay, within the method's 2.4e-3
    assert abs(d1[3] / (e0 * math.exp(-4 * A.nu_of(p.tau) * k * k * steps)) - 1) < 5e-3
