"""The GPU path's per-node arithmetic (cascade.h, compiled for the host in
FP64) against the oracle, on the CPU.

Checks, per node, with random non-equilibrium states, random rates in (0, 2)
and random forces: the step kernels' collision (with and without a body
force) equals the oracle's explicit cascade; the initial-state map equals the
oracle's f^eq - S/2; the hand-written reverse passes (the adjoint kernels'
transposed collision, the initial-state map's reverse) equal central finite
differences of the forward maps.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


@pytest.fixture(scope="module")
def lib():
    from tests.native import build
    path = build.build()
    h = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    h.host_collide_step.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_double,
                                    ctypes.c_int, dp]
    h.host_collide_adj.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_double, dp, dp, dp]
    h.host_init.argtypes = [ctypes.c_double] * 6 + [dp]
    h.host_init_T.argtypes = [ctypes.c_double] * 6 + [dp, dp]
    return h


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _case(rng, rho0):
    f = W * rho0 * (1 + rng.uniform(-0.3, 0.3, 9))
    f = f + rng.uniform(-0.1, 0.1) * np.array([0, 1, 0, -1, 0, 1, -1, -1, 1]) / 9
    w6 = rng.uniform(0.05, 1.95, 6)  # omega_3, omega_4 (= omega_5 here or not), ...
    Fx, Fy = rng.uniform(-1e-2, 1e-2, 2)
    return f, w6, Fx, Fy


def _oracle_omega(w6):
    om = np.zeros(9)
    om[3:9] = w6
    return om


def _collide(lib, d, Fx, Fy, w6, rho0, force=True):
    out = np.empty(9)
    d = np.ascontiguousarray(d)
    w6 = np.ascontiguousarray(w6)
    lib.host_collide_step(_p(d), Fx, Fy, _p(w6), rho0, int(force), _p(out))
    return out


@pytest.mark.parametrize("force", [True, False])
@pytest.mark.parametrize("rho0", [1.0, 0.7])
def test_collision_matches_oracle(lib, force, rho0):
    rng = np.random.default_rng(3)
    for _ in range(200):
        f, w6, Fx, Fy = _case(rng, rho0)
        if not force:
            Fx = Fy = 0.0
        got = _collide(lib, f - W * rho0, Fx, Fy, w6, rho0, force) + W * rho0
        want = oracle.collide(_oracle_omega(w6), Fx, Fy, f)
        np.testing.assert_allclose(got, want, rtol=0, atol=2e-15)


def test_init_matches_oracle(lib):
    rng = np.random.default_rng(4)
    for _ in range(100):
        rho, ux, uy = rng.uniform(0.8, 1.2), *rng.uniform(-0.2, 0.2, 2)
        Fx, Fy = rng.uniform(-1e-2, 1e-2, 2)
        out = np.empty(9)
        lib.host_init(rho, ux, uy, Fx, Fy, 1.0, _p(out))
        want = oracle.equilibrium(rho, ux, uy) - 0.5 * oracle.source(Fx, Fy, ux, uy)
        np.testing.assert_allclose(out + W, want, rtol=0, atol=2e-15)


@pytest.mark.parametrize("rho0", [1.0, 0.7])
def test_collision_reverse_equals_finite_differences(lib, rho0):
    """collide_adj (the adjoint kernels' transposed Jacobian) against central
    finite differences of the step kernels' collision, with respect to the
    populations and the force."""
    rng = np.random.default_rng(5)
    eps = 1e-6
    for _ in range(50):
        f, w6, Fx, Fy = _case(rng, rho0)
        d = f - W * rho0
        aout = rng.normal(size=9)
        ad, aF = np.empty(9), np.empty(2)
        lib.host_collide_adj(_p(d), Fx, Fy, _p(np.ascontiguousarray(w6)), rho0, _p(aout), _p(ad), _p(aF))
        jac = np.empty((9, 9))
        for k in range(9):
            e = np.zeros(9)
            e[k] = eps
            jac[:, k] = (_collide(lib, d + e, Fx, Fy, w6, rho0) - _collide(lib, d - e, Fx, Fy, w6, rho0)) / (2 * eps)
        np.testing.assert_allclose(ad, jac.T @ aout, rtol=1e-7, atol=1e-9)
        jF = np.stack([(_collide(lib, d, Fx + eps, Fy, w6, rho0) - _collide(lib, d, Fx - eps, Fy, w6, rho0)) / (2 * eps),
                       (_collide(lib, d, Fx, Fy + eps, w6, rho0) - _collide(lib, d, Fx, Fy - eps, w6, rho0)) / (2 * eps)],
                      axis=1)
        np.testing.assert_allclose(aF, jF.T @ aout, rtol=1e-7, atol=1e-9)


def test_collision_reverse_without_force(lib):
    """Without a body force the force cotangent is still dL/dF at F = 0 (the
    adjoint of a rollout with a zero force field)."""
    rng = np.random.default_rng(8)
    eps = 1e-6
    for _ in range(20):
        f, w6, _, _ = _case(rng, 1.0)
        d = f - W
        aout = rng.normal(size=9)
        ad, aF = np.empty(9), np.empty(2)
        lib.host_collide_adj(_p(d), 0.0, 0.0, _p(np.ascontiguousarray(w6)), 1.0, _p(aout), _p(ad), _p(aF))
        jF = np.stack([(_collide(lib, d, eps, 0.0, w6, 1.0) - _collide(lib, d, -eps, 0.0, w6, 1.0)) / (2 * eps),
                       (_collide(lib, d, 0.0, eps, w6, 1.0) - _collide(lib, d, 0.0, -eps, w6, 1.0)) / (2 * eps)], axis=1)
        np.testing.assert_allclose(aF, jF.T @ aout, rtol=1e-7, atol=1e-9)


def test_init_reverse_equals_finite_differences(lib):
    rng = np.random.default_rng(6)
    eps = 1e-6
    for _ in range(50):
        x0 = np.array([rng.uniform(0.8, 1.2), *rng.uniform(-0.2, 0.2, 2), *rng.uniform(-1e-2, 1e-2, 2)])
        aout = rng.normal(size=9)
        g = np.empty(5)
        lib.host_init_T(*x0, 1.0, _p(aout), _p(g))

        def F(x):
            o = np.empty(9)
            lib.host_init(*x, 1.0, _p(o))
            return o
        for k in range(5):
            e = np.zeros(5)
            e[k] = eps
            fd = (F(x0 + e) - F(x0 - e)) / (2 * eps) @ aout
            assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd))
