"""Post-processing of lid-driven cavity fields (Sec. IV.C quantities).

Coordinates are normalised by the cavity side L = N: node (i, j) sits at
((i + 1/2)/N, (j + 1/2)/N); the walls are at 0 and 1, the lid at y = 1.
"""
import numpy as np


def stream_function(ux):
    """psi(x, y) = integral of u dy from the bottom wall (psi = 0 there),
    trapezoidal in y with u = 0 on the wall; returns psi at the nodes in units
    of (lattice speed) x (node spacing)."""
    ny = ux.shape[0]
    psi = np.empty_like(ux)
    psi[0] = 0.25 * ux[0]  # half a spacing from the wall, u(wall) = 0
    for j in range(1, ny):
        psi[j] = psi[j - 1] + 0.5 * (ux[j - 1] + ux[j])
    return psi


def vortex_centre(ux, sign=-1.0, window=None):
    """Location of the extremum of the stream function (minimum for the
    primary, clockwise vortex: sign = -1), refined by a least-squares
    quadratic over the 3 x 3 neighbourhood.  window = (x0, x1, y0, y1) in
    normalised coordinates restricts the search.  Returns (x, y)."""
    n_y, n_x = ux.shape
    psi = sign * stream_function(ux)  # extremum -> maximum
    xs = (np.arange(n_x) + 0.5) / n_x
    ys = (np.arange(n_y) + 0.5) / n_y
    mask = np.ones_like(psi, dtype=bool)
    if window is not None:
        x0, x1, y0, y1 = window
        mask &= (xs[None, :] >= x0) & (xs[None, :] <= x1) & (ys[:, None] >= y0) & (ys[:, None] <= y1)
    mask[[0, -1], :] = False
    mask[:, [0, -1]] = False
    j, i = np.unravel_index(np.argmax(np.where(mask, psi, -np.inf)), psi.shape)
    dx, dy = np.meshgrid([-1, 0, 1], [-1, 0, 1])
    A = np.stack([np.ones(9), dx.ravel(), dy.ravel(), dx.ravel() ** 2, dx.ravel() * dy.ravel(),
                  dy.ravel() ** 2], axis=1)
    c = np.linalg.lstsq(A, psi[j - 1:j + 2, i - 1:i + 2].ravel(), rcond=None)[0]
    H = np.array([[2 * c[3], c[4]], [c[4], 2 * c[5]]])
    off = np.linalg.solve(H, -c[1:3])
    return (xs[i] + off[0] / n_x, ys[j] + off[1] / n_y)


def bilinear(field, x, y):
    """Field value at normalised (x, y) by bilinear interpolation of nodes."""
    n_y, n_x = field.shape
    fx, fy = x * n_x - 0.5, y * n_y - 0.5
    i, j = int(np.floor(fx)), int(np.floor(fy))
    tx, ty = fx - i, fy - j
    return ((1 - tx) * (1 - ty) * field[j, i] + tx * (1 - ty) * field[j, i + 1] +
            (1 - tx) * ty * field[j + 1, i] + tx * ty * field[j + 1, i + 1])


def central_difference_strain(ux, uy):
    """Second-order central differences (interior nodes) of the velocity:
    (du/dx, dv/dy, du/dy + dv/dx) in lattice units."""
    dudx = np.full_like(ux, np.nan)
    dvdy = np.full_like(ux, np.nan)
    shear = np.full_like(ux, np.nan)
    dudx[:, 1:-1] = 0.5 * (ux[:, 2:] - ux[:, :-2])
    dvdy[1:-1, :] = 0.5 * (uy[2:, :] - uy[:-2, :])
    dudy = np.full_like(ux, np.nan)
    dvdx = np.full_like(ux, np.nan)
    dudy[1:-1, :] = 0.5 * (ux[2:, :] - ux[:-2, :])
    dvdx[:, 1:-1] = 0.5 * (uy[:, 2:] - uy[:, :-2])
    shear = dudy + dvdx
    return dudx, dvdy, shear


def run_to_steady(lat, check_every=2000, tol=1e-10, max_steps=10_000_000):
    """Step until the relative change of the velocity field between checks,
    sum |u^n - u^(n-check)| / sum |u^n| (the Sec. III norm), falls below tol.
    Returns the last residual."""
    import torch
    prev, r = None, float("inf")
    while lat.time < max_steps:
        lat.step(check_every)
        m = lat.macroscopic(strain=False)
        u = torch.stack([m["ux"], m["uy"]])
        if prev is not None:
            r = ((u - prev).norm(dim=0).sum() / u.norm(dim=0).sum()).item()
            if r < tol:
                break
        prev = u
    return r
