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


def cavity(n, u_lid, tau, storage="fp64"):
    """A lattice for the n x n lid-driven cavity (lid y = 1 moving in +x),
    started from rest."""
    import workloads as W
    from paper_1202_6351_amd import Lattice, Params
    lat = Lattice(Params(n, n, tau=tau, bc=("wall",) * 4, wall_u=(0, 0, 0, u_lid), storage=storage),
                  device="cuda:0")
    return lat.init_equilibrium(*W.at_rest(n, n))


# ---------------------------------------------------- grid convergence (Sec. III.C)

CONV_TAU, CONV_RE = 0.55, 100.0
CONV_GRIDS = (13, 19, 25, 31, 37, 49, 61, 85, 97, 121)


def steady_centrelines(n, tau=CONV_TAU, re=CONV_RE, tol=1e-10):
    """Diffusive scaling: tau fixed, lid speed U = Re nu / n.  Runs the n x n
    cavity (n odd) to a steady state and returns (positions, {(quantity,
    line): values}) on the vertical (x = 1/2) and horizontal (y = 1/2)
    centre lines, velocities in units of U, strain rates in units of U/L."""
    u_lid = re * (tau - 0.5) / 3.0 / n
    lat = cavity(n, u_lid, tau)
    r = run_to_steady(lat, check_every=max(100, 2 * int(round(0.025 * n / u_lid))), tol=tol)
    assert r < tol, (n, r)
    m = {k: v.cpu().numpy() for k, v in lat.macroscopic().items()}
    c = (n - 1) // 2
    q = {"u": m["ux"] / u_lid, "v": m["uy"] / u_lid,
         "dv/dy": m["syy"] * n / u_lid, "du/dy+dv/dx": 2 * m["sxy"] * n / u_lid}
    pos = (np.arange(n) + 0.5) / n
    return pos, {(k, line): (v[:, c] if line == "vertical" else v[c, :])
                 for k, v in q.items() for line in ("vertical", "horizontal")}


def convergence_slopes(grids=CONV_GRIDS, ref=401):
    """Relative error sum |q - q_ref| / sum |q_ref| of every centre-line
    quantity on each grid against the ref x ref solution (cubic-spline
    interpolated onto the coarse nodes), and the least-squares slope of
    -log(error) against log(n).  Returns ({key: slope}, {key: [errors]})."""
    from scipy.interpolate import CubicSpline
    rpos, rq = steady_centrelines(ref)
    sols = [steady_centrelines(n) for n in grids]
    slopes, errors = {}, {}
    for key in rq:
        errs = []
        for pos, q in sols:
            a = CubicSpline(rpos, rq[key])(pos)
            errs.append(np.abs(q[key] - a).sum() / np.abs(a).sum())
        errors[key] = errs
        slopes[key] = -np.polyfit(np.log(np.asarray(grids, float)), np.log(errs), 1)[0]
    return slopes, errors


# ------------------------------------------------------------ stability (Sec. V)

def stays_bounded(lat, n, u_lid, n_adv, local=True):
    """Advance n_adv lid transit times L/U, checking after each that the
    field stays finite and, with `local`, that the largest speed stays below
    5 U (a local excursion, at a lid corner, exceeds it first)."""
    import torch
    chunk = 2 * int(n / u_lid / 2)
    for _ in range(int(n_adv)):
        lat.step(chunk)
        m = lat.macroscopic(strain=False)
        umax = torch.sqrt(m["ux"] ** 2 + m["uy"] ** 2).max().item()
        if not np.isfinite(umax) or (local and umax > 5 * u_lid):
            return False
    return True


def stable_at(n, u_lid, cell_re, n_adv=100, local=True):
    """Impulsively started cavity at cell Reynolds number U/nu: bounded for
    n_adv transit times (stays_bounded's criterion)?"""
    return stays_bounded(cavity(n, u_lid, 3.0 * u_lid / cell_re + 0.5), n, u_lid, n_adv, local)


def max_stable_cell_re(n, u_lid=0.1, lo=10.0, hi=2000.0, rel=0.01, n_adv=100):
    """Largest cell Reynolds number at which the impulsively started cavity
    stays bounded (geometric bisection to a relative width rel)."""
    while hi / lo > 1 + rel:
        mid = (lo * hi) ** 0.5
        lo, hi = (mid, hi) if stable_at(n, u_lid, mid, n_adv) else (lo, mid)
    return lo


def max_stable_cell_re_continuation(n, u_lid=0.1, start=40.0, factor=1.02, n_adv=20):
    """Lid speed fixed, tau lowered stage by stage: each stage restarts from
    the previous stage's state with the cell Reynolds number raised by
    `factor` and runs n_adv transit times.  Returns the last bounded stage."""
    from paper_1202_6351_amd import Lattice, Params
    lat = cavity(n, u_lid, 3.0 * u_lid / start + 0.5)
    assert stays_bounded(lat, n, u_lid, 50)
    rec = start
    while rec < 5000:
        nxt = Lattice(Params(n, n, tau=3.0 * u_lid / (rec * factor) + 0.5, bc=("wall",) * 4,
                             wall_u=(0, 0, 0, u_lid), storage="fp64"), device="cuda:0")
        nxt.restore(lat.snapshot(), lat.time)
        if not stays_bounded(nxt, n, u_lid, n_adv):
            break
        lat, rec = nxt, rec * factor
    return rec


def bounded_for_steps(n, u_lid, tau, steps):
    """Alternate stability test (Sec. V): does the impulsively started n x n
    cavity with lid speed u_lid and relaxation time tau stay bounded (speed
    below 5 U, finite) for `steps` steps?"""
    lat = cavity(n, u_lid, tau)
    chunk = 1002
    while lat.time < steps:
        lat.step(min(chunk, steps - lat.time))
        m = lat.macroscopic(strain=False)
        umax = float((m["ux"] ** 2 + m["uy"] ** 2).sqrt().max())
        if not np.isfinite(umax) or umax > 5 * u_lid:
            return False
    return True


def max_stable_lid_speed(n=26, tau=0.55, steps=50_000, lo=1e-3, hi=1.0, rel=0.01):
    """The largest lid speed for which bounded_for_steps holds; geometric
    bisection to a relative width rel."""
    while hi / lo > 1 + rel:
        mid = (lo * hi) ** 0.5
        lo, hi = (mid, hi) if bounded_for_steps(n, mid, tau, steps) else (lo, mid)
    return lo
