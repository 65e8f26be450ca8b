"""Seeded synthetic inputs for the D2Q9 lattice problems (shared by the tests,
the benchmark, the oracle checks and the GPU runs).

This module holds problem set-up only -- initial fields, force fields, the
relaxation time that gives a Reynolds number -- and none of the lattice
Boltzmann method's own arithmetic.  All random draws use numpy's PCG64
``default_rng(seed)``; every array is float64 and C-contiguous.

Problems (paper Section III):
  * decaying Taylor-Green vortex, periodic square (initial u, v, p);
  * body-force driven Poiseuille channel (start at rest);
  * lid-driven square cavity (at rest, density noise).
Node coordinates are x_i = i, y_j = j; walls sit half a spacing outside the
first and last fluid node.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

CS2 = 1.0 / 3.0  # lattice speed of sound squared (Sec. II)


def viscosity(tau: float) -> float:
    """nu = c_s^2 (tau - 1/2) (Sec. II, nu = c_s^2 (1/omega - 1/2))."""
    return CS2 * (tau - 0.5)


def tau_for(nu: float) -> float:
    return nu / CS2 + 0.5


def taylor_green(n: int, u0: float, mode: int = 1, noise: float = 0.0,
                 seed: int = 0, rho0: float = 1.0, ny: int | None = None):
    """Initial fields of the decaying Taylor-Green vortex (Sec. III):
    u = -u0 cos(kx) sin(ky), v = u0 sin(kx) cos(ky),
    p = p0 [1 - u0^2/(4 c_s^2) (cos 2kx + cos 2ky)], rho = p / c_s^2,
    k = 2 pi mode / n.  Optional i.i.d. uniform(-noise, noise) added to each
    velocity component (seeded)."""
    ny = n if ny is None else ny
    k = 2.0 * math.pi * mode / n
    ky = 2.0 * math.pi * mode / ny
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    ux = -u0 * np.cos(k * x) * np.sin(ky * y)
    uy = u0 * np.sin(k * x) * np.cos(ky * y)
    rho = rho0 * (1.0 - u0 * u0 / (4.0 * CS2) * (np.cos(2 * k * x) + np.cos(2 * ky * y)))
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        ux = ux + rng.uniform(-noise, noise, size=ux.shape)
        uy = uy + rng.uniform(-noise, noise, size=uy.shape)
    return (np.ascontiguousarray(rho), np.ascontiguousarray(ux),
            np.ascontiguousarray(uy))


def at_rest(nx: int, ny: int, rho0: float = 1.0, density_noise: float = 0.0,
            seed: int = 0):
    """Fluid at rest; optional i.i.d. uniform(-a, a) density noise (seeded)."""
    rho = np.full((ny, nx), rho0, dtype=np.float64)
    if density_noise > 0.0:
        rng = np.random.default_rng(seed)
        rho = rho + rng.uniform(-density_noise, density_noise, size=rho.shape)
    z = np.zeros((ny, nx), dtype=np.float64)
    return rho, z, z.copy()


def random_flow(nx: int, ny: int, seed: int, u_amp: float = 0.05,
                rho_amp: float = 0.02, rho0: float = 1.0):
    """Smooth-free random fields for parity tests: rho0 + U(-a, a),
    u, v ~ U(-u_amp, u_amp) independently at every node."""
    rng = np.random.default_rng(seed)
    rho = rho0 + rng.uniform(-rho_amp, rho_amp, size=(ny, nx))
    ux = rng.uniform(-u_amp, u_amp, size=(ny, nx))
    uy = rng.uniform(-u_amp, u_amp, size=(ny, nx))
    return rho, ux, uy


def random_populations(nx: int, ny: int, seed: int, amp: float = 0.2):
    """Positive population vectors scattered around the D2Q9 rest weights
    (4/9, 1/9 x4, 1/36 x4), each entry times (1 + U(-amp, amp)); layout
    [9, ny, nx].  For parity of arbitrary (non-equilibrium) states."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)
    rng = np.random.default_rng(seed)
    f = w[:, None, None] * (1.0 + rng.uniform(-amp, amp, size=(9, ny, nx)))
    return np.ascontiguousarray(f)


def force_field(nx: int, ny: int, std: float, seed: int):
    """Per-node body force [2, ny, nx], i.i.d. N(0, std^2) (seeded)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.normal(0.0, std, size=(2, ny, nx)))


def poiseuille_force(tau: float, u_centre: float, height: int, rho0: float = 1.0) -> float:
    """Body force giving centre-line speed u_c between walls a distance H
    apart: u(y) = F/(2 rho0 nu) y(H - y), so F = 8 rho0 nu u_c / H^2."""
    return 8.0 * rho0 * viscosity(tau) * u_centre / height ** 2


def cavity_tau(n: int, u_lid: float, re: float) -> float:
    """Relaxation time for Re = U N / nu in an N x N cavity."""
    return tau_for(u_lid * n / re)


@dataclass(frozen=True)
class Workload:
    """A named benchmark / parity configuration."""
    name: str
    nx: int
    ny: int
    tau: float
    storage: str
    steps: int


# Configurations the benchmark and the full-size parity tests use.
TAYLOR_GREEN_64 = Workload("taylor_green_64x64_fp64", 64, 64, 0.8, "fp64", 1000)
POISEUILLE_256x64 = Workload("poiseuille_256x64", 256, 64, 0.8, "fp64", 0)
CAVITY_4096 = Workload("cavity_4096x4096_re1000_fp32", 4096, 4096,
                       cavity_tau(4096, 0.1, 1000.0), "fp32", 0)
TG_8192_FP16 = Workload("taylor_green_8192x8192_fp16dev", 8192, 8192, 0.8, "fp16", 0)
TG_512 = Workload("taylor_green_512x512", 512, 512, 0.8, "fp32", 20000)
