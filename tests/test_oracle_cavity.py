"""Oracle pin of the cavity walls: the lid-driven cavity at Re = 100 converges
at second order (Sec. III.C), which fixes how the lid meets the side walls.

Diffusive scaling (tau = 0.55 on every grid, lid speed U = Re nu / N), grids
13^2, 25^2 and 49^2, each run to a steady state.  The observed order p of each
centre-line quantity comes from the three grids alone,
    (h0^p - h1^p) / (h1^p - h2^p) = |q0 - q1| / |q1 - q2|,  h = 1/N,
with the finer solutions interpolated onto the 13 coarse nodes.  Reading E6
(a link crossing two walls passes through their corner point, at rest) gives
p >= 2.1 for all eight quantities.  With the full lid term on those two corner
links the cavity converges at first order (lowest p about 1.0); with half of
it the lowest p is about 1.2.  Either alternative fails this test.
"""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline
from scipy.optimize import brentq

import oracle
import workloads as W

TAU, RE, GRIDS = 0.55, 100.0, (13, 25, 49)


def _steady_centrelines(n):
    nu = W.viscosity(TAU)
    u_lid = RE * nu / n
    p = oracle.Params(n, n, tau=TAU, bc=(1, 1, 1, 1), wall_u=(0, 0, 0, u_lid))
    f = oracle.init_state(p, *W.at_rest(n, n))
    chunk = max(100, int(0.05 * n / u_lid))
    prev = None
    for _ in range(10000):
        f = oracle.step(p, f, chunk)
        m = oracle.macroscopic(p, f)
        u = np.stack([m["ux"], m["uy"]])
        if prev is not None:
            r = np.sqrt(((u - prev) ** 2).sum(0)).sum() / np.sqrt((u ** 2).sum(0)).sum()
            if r < 1e-9:
                break
        prev = u
    else:
        raise AssertionError(f"{n}^2 cavity not steady")
    c = (n - 1) // 2  # odd n: the centre lines run through nodes
    # velocity in units of U, strain rates in units of U / L (L = n)
    q = {"u": m["ux"] / u_lid, "v": m["uy"] / u_lid,
         "dv/dy": m["syy"] * n / u_lid, "du/dy+dv/dx": 2 * m["sxy"] * n / u_lid}
    pos = (np.arange(n) + 0.5) / n
    return pos, {(k, line): (v[:, c] if line == "vertical" else v[c, :])
                 for k, v in q.items() for line in ("vertical", "horizontal")}


@pytest.fixture(scope="module")
def solutions():
    return [_steady_centrelines(n) for n in GRIDS]


def test_cavity_second_order_three_grids(solutions):
    h = 1.0 / np.array(GRIDS, float)
    at = solutions[0][0]
    orders = {}
    for key in solutions[0][1]:
        vals = [CubicSpline(pos, q[key])(at) for pos, q in solutions]
        ratio = np.abs(vals[0] - vals[1]).sum() / np.abs(vals[1] - vals[2]).sum()
        orders[key] = brentq(lambda p: (h[0] ** p - h[1] ** p) / (h[1] ** p - h[2] ** p) - ratio, 0.1, 6.0)
    print({f"{k[0]} {k[1]}": round(v, 2) for k, v in orders.items()})
    assert all(p > 1.8 for p in orders.values()), orders
