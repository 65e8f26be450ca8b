"""Numerical stability of the cascaded model in the lid-driven cavity
(Sec. V, Table cellReynoldsnumber).

The paper finds the cascaded model stable at higher cell Reynolds numbers
Re_c = U dx / nu than the standard raw-moment MRT model, which in turn is
more stable than SRT.  Here (lid speed 0.1, FP64, omega_4 = omega_5 = 1/tau,
the other rates 1, started impulsively from rest) the cascaded cavity must
stay bounded for 100 lid transit times at the standard-MRT column's cell
Reynolds number on 101^2, 201^2 and 401^2.

The envelope this build measures is pinned as a regression, under two
criteria.  Local: the impulsively started cavity (lid 0.1) counts as stable
while its largest speed stays below 5 U and finite for 100 lid transit times;
it is stable at 95 % and unstable at 105 % of the measured limit 81.3 / 80.9
/ 80.9 (101^2 / 201^2 / 401^2), the same for runs of 5 to 100 transits.
Global (the paper judges instability by the relative global error): stable
while the field stays finite for 100 transits.  Scanned from Re_c 100 to 260
(steps of 2 to 5), every run has a corner excursion above 5 U within its
first eight transits; a run that blows up does so within its first four
transits, and one that survives them stays finite for all 100 with a mean
speed of 0.15 - 0.22 U.  The outcome is not monotone in Re_c: all three grids
stay finite up to Re_c 152, all three blow up from 186 to 204, and isolated
runs blow up in between and above (first at 154 on 201^2 and 401^2, at 178
on 101^2).  The test pins the two robust ends, 150 and 190 / 196.  The
alternate test of Sec. V (26^2 grid, viscosity fixed, largest lid speed that
stays bounded for 50 000 steps) is pinned the same way at tau = 0.52 and 0.6
(measured 0.41 and 0.80).
"""
import os

import pytest

from tests import cavity_tools as C

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table():
    out = {}
    for line in open(os.path.join(GOLDEN, "cell_reynolds.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, srt, mrt, casc = line.split()
        out[int(n)] = (float(srt), float(mrt), float(casc))
    return out


@pytest.mark.parametrize("n", [101, 201, 401])
def test_stable_beyond_standard_mrt_limit(n):
    srt, mrt, _ = _table()[n]
    assert C.stable_at(n, 0.1, mrt, n_adv=100), f"{n}^2 unstable at Re_c {mrt}"


# measured largest stable cell Reynolds number, impulsive start, lid 0.1
IMPULSIVE_LIMIT = {101: 81.3, 201: 80.9, 401: 80.9}


@pytest.mark.parametrize("n", [101, 201, 401])
def test_impulsive_start_envelope(n):
    lim = IMPULSIVE_LIMIT[n]
    assert C.stable_at(n, 0.1, 0.95 * lim, n_adv=100), f"{n}^2 unstable at Re_c {0.95 * lim:.1f}"
    assert not C.stable_at(n, 0.1, 1.05 * lim, n_adv=100), f"{n}^2 stable at Re_c {1.05 * lim:.1f}"


# measured largest lid speed bounded for 50 000 steps on 26^2, by tau
LID_SPEED_LIMIT = {0.52: 0.41, 0.6: 0.80}


@pytest.mark.parametrize("tau", sorted(LID_SPEED_LIMIT))
def test_alternate_lid_speed_limit(tau):
    u = LID_SPEED_LIMIT[tau]
    assert C.bounded_for_steps(26, 0.95 * u, tau, 50_000)
    assert not C.bounded_for_steps(26, 1.05 * u, tau, 50_000)


# Re_c at which all three grids stay finite for 100 transits, and two inside
# the band in which all three blow up during the first transits
GLOBAL_FINITE, GLOBAL_BLOWUP = 150.0, (190.0, 196.0)


@pytest.mark.parametrize("n", [101, 201, 401])
def test_global_criterion_envelope(n):
    assert C.stable_at(n, 0.1, GLOBAL_FINITE, n_adv=100, local=False), f"{n}^2 blew up at Re_c {GLOBAL_FINITE}"
    for re_c in GLOBAL_BLOWUP:
        assert not C.stable_at(n, 0.1, re_c, n_adv=100, local=False), f"{n}^2 finite at Re_c {re_c}"
