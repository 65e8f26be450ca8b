"""Ring schedule of the strip kernel (k_strip), checked on the CPU.

A workgroup of NW wavefronts walks a strip down rows ys..ye-1, NW rows per
iteration.  In iteration `it`, wavefront w computes step 0 of window row
r0 = ys - (NS-1) + NW*it + w into ring 0, then (after a barrier) step s of
row r0 - s from ring s-1 into ring s, and the last step from ring NS-2 to
HBM.  There is a barrier after every step but the last, so the last step of
one iteration and step 0 of the next share a phase.  Ring slots are
row mod RING.

The model replays those phases and checks that every ring read finds the row
it expects, written in an earlier phase, and that no phase both writes and
reads one slot (a race between wavefronts).  It runs the interior walk's
variant too, where step 0 writes every row and the iteration count is padded
to a multiple of three.  The ring sizes of the kernel are read from
lbm_launch.h; one row fewer must fail.
"""
import os
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LAUNCH_H = os.path.join(HERE, "..", "paper_1202_6351_amd", "csrc", "lbm_launch.h")


def _constants():
    text = open(LAUNCH_H).read()
    nw = int(re.search(r"kStripWaves\s*=\s*(\d+)", text).group(1))
    ring = int(re.search(r"kStripRing\s*=\s*(\d+)", text).group(1))
    return nw, ring


def replay(ns, nw, ring, ys, ye, pad3=False, step0_all_rows=False):
    """Replay the phases of one workgroup; raise AssertionError on a hazard."""
    slot = lambda r: (r + 8 * ring) % ring
    content = {}  # (ring, slot) -> (row, phase written)
    nit = (ye - ys + 2 * (ns - 1) + nw - 1) // nw
    if pad3:
        nit = (nit + 2) // 3 * 3
    phase = 0
    ops = {}
    for it in range(nit):
        for s in range(ns):
            if s == 0 and it > 0:
                pass  # shares the phase of the previous iteration's last step
            else:
                phase += 1
            writes, reads = [], []
            for w in range(nw):
                r0 = ys - (ns - 1) + it * nw + w
                if s == 0:
                    if step0_all_rows or r0 < ye + ns - 1:
                        writes.append((0, slot(r0), r0))
                    continue
                r = r0 - s
                if ys - (ns - 1 - s) <= r < ye + (ns - 1 - s):
                    reads += [(s - 1, slot(q), q) for q in (r - 1, r, r + 1)]
                    if s < ns - 1:
                        writes.append((s, slot(r), r))
            for rg, sl, row in reads:
                got = content.get((rg, sl))
                assert got is not None and got[0] == row and got[1] < phase, \
                    f"ring {rg} slot {sl}: want row {row} from an earlier phase, found {got}"
            for rg, sl, row in writes:
                content[(rg, sl)] = (row, phase)
            ops.setdefault(phase, ([], []))
            ops[phase][0].extend((rg, sl) for rg, sl, _ in writes)
            ops[phase][1].extend((rg, sl) for rg, sl, _ in reads)
    for ph, (ws, rs) in ops.items():
        both = set(ws) & set(rs)
        assert not both, f"phase {ph} writes and reads {sorted(both)}"


@pytest.mark.parametrize("variant", ["edge", "interior"])
def test_kernel_rings_are_hazard_free(variant):
    nw, ring = _constants()
    kw = dict(pad3=True, step0_all_rows=True) if variant == "interior" else {}
    for ys in (0, 3, 100):
        for length in range(1, 64):
            replay(3, nw, ring, ys, ys + length, **kw)


def test_one_row_short_races():
    nw, ring = _constants()
    with pytest.raises(AssertionError):
        replay(3, nw, ring - 1, 0, 40)


@pytest.mark.parametrize("nw", [1, 2, 4, 8])
def test_ring_rule(nw):
    """Three fused steps need NW + 2 ring rows; two steps (no barrier between
    the last step and the next step 0) need 2 NW + 2."""
    replay(3, nw, nw + 2, 0, 50)
    replay(2, nw, 2 * nw + 2, 0, 50)
    with pytest.raises(AssertionError):
        replay(3, nw, nw + 1, 0, 50)
    with pytest.raises(AssertionError):
        replay(2, nw, 2 * nw + 1, 0, 50)
