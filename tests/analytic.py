"""Analytic solutions and the paper's error norm (Sec. III)."""
import math

import numpy as np

CS2 = 1.0 / 3.0


def nu_of(tau):
    return CS2 * (tau - 0.5)


def taylor_green(n, u0, t, tau, mode=1):
    """u, v, S_xx of the decaying Taylor-Green vortex at time t
    (Sec. III: u = -u0 cos kx sin ky e^{-2 nu k^2 t}, ...,
    S_xx = k u0 sin kx sin ky e^{-2 nu k^2 t}), k = 2 pi mode / n."""
    k = 2 * math.pi * mode / n
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(n, dtype=np.float64)[:, None]
    dec = math.exp(-2 * nu_of(tau) * k * k * t)
    ux = -u0 * np.cos(k * x) * np.sin(k * y) * dec
    uy = u0 * np.sin(k * x) * np.cos(k * y) * dec
    sxx = k * u0 * np.sin(k * x) * np.sin(k * y) * dec
    return ux, uy, sxx


def poiseuille(ny, fx, tau, rho0=1.0):
    """Body-force Poiseuille profile between halfway walls at y = -1/2 and
    y = ny - 1/2: u(yh) = F/(2 rho0 nu) yh (H - yh), yh = j + 1/2, H = ny."""
    yh = np.arange(ny, dtype=np.float64) + 0.5
    return fx / (2 * rho0 * nu_of(tau)) * yh * (ny - yh)


def rel_error_vec(ux_c, uy_c, ux_a, uy_a):
    """Relative global error sum_i ||u_c - u_a|| / sum_i ||u_a|| with the
    Euclidean norm of the node velocity (Sec. III)."""
    num = np.sqrt((ux_c - ux_a) ** 2 + (uy_c - uy_a) ** 2).sum()
    den = np.sqrt(ux_a ** 2 + uy_a ** 2).sum()
    return num / den


def rel_error_scalar(c, a):
    return np.abs(c - a).sum() / np.abs(a).sum()


def slope(ns, errs):
    """Least-squares slope of -log(err) vs log(n)."""
    return -np.polyfit(np.log(np.asarray(ns, float)), np.log(np.asarray(errs)), 1)[0]
