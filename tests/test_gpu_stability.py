"""Numerical stability of the cascaded model in the lid-driven cavity
(Sec. V, Table cellReynoldsnumber).

The paper finds the cascaded model stable at higher cell Reynolds numbers
Re_c = U dx / nu than the standard raw-moment MRT model, which in turn is
more stable than SRT.  Here (lid speed 0.1, FP64, omega_4 = omega_5 = 1/tau,
the other rates 1, started impulsively from rest) the cascaded cavity must
stay bounded for 100 lid transit times at the standard-MRT column's cell
Reynolds number on 101^2, 201^2 and 401^2.
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
