"""Pins of the oracle's square sharing footprints (Sec. 4.3, "Square
Footprints"): hand-enumerated member sets (tests/golden/footprint_windows.txt,
derived in its header) and the design criteria the section states -- every
pixel in its own footprint, one size for all lanes, the closest lanes,
windows shifted inward at the tile's edges so edge lanes share their
neighbours' texels, and more variety between neighbouring 2x2 windows than
the quad intrinsic's fixed placement allows."""
import os

import numpy as np
import pytest

import oracle as o

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "footprint_windows.txt")
SIZES = {"quad2x2": 2, "wave2x2": 2, "square3x3": 3, "square4x4": 4}


def golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        head, ids = line.split(":")
        kind, lx, ly = head.split()
        rows.append((kind, int(lx), int(ly), sorted(int(v) for v in ids.split())))
    return rows


def test_golden_member_sets():
    rows = golden_rows()
    assert len(rows) >= 20 and {r[0] for r in rows} == set(SIZES)
    for kind, lx, ly, ids in rows:
        got = sorted(int(v) for v in o.footprint_members(kind)[ly * 8 + lx])
        assert got == ids, (kind, lx, ly, got, ids)


@pytest.mark.parametrize("kind", list(SIZES))
def test_windows_are_full_squares_containing_the_pixel(kind):
    n = SIZES[kind]
    m = o.footprint_members(kind)
    assert m.shape == (64, n * n)                     # criterion 2: one size for every lane
    for q in range(64):
        row = m[q]
        assert len(set(row.tolist())) == n * n and row.min() >= 0 and row.max() < 64
        assert q in row                               # each lane is in its own footprint (Sec. 4.5)
        xs, ys = row % 8, row // 8
        # an n x n block of the tile: contiguous, inside the tile
        assert xs.max() - xs.min() == n - 1 and ys.max() - ys.min() == n - 1
        # criterion 1: the closest lanes (within n - 1 on each axis)
        assert np.all(np.abs(xs - q % 8) <= n - 1) and np.all(np.abs(ys - q // 8) <= n - 1)


@pytest.mark.parametrize("kind,lo,hi", [("square3x3", 1, 6), ("square4x4", 1, 4)])
def test_square_windows_centred_where_they_fit_and_shifted_inward_at_edges(kind, lo, hi):
    n = SIZES[kind]
    m = o.footprint_members(kind)
    for q in range(64):
        lx, ly = q % 8, q // 8
        for l, ax in ((lx, m[q] % 8), (ly, m[q] // 8)):
            if lo <= l <= hi:                          # fits: the window starts one lane before the pixel
                assert ax.min() == l - 1
            elif l < lo:                               # left/top edge: shifted right/down to the edge
                assert ax.min() == 0
            else:                                      # right/bottom edge: shifted to end at lane 7
                assert ax.max() == 7
    # the edge passage of Sec. 4.3: lanes at the edges filter their neighbours' texels
    same = lambda a, b: set(m[a].tolist()) == set(m[b].tolist())
    for y in range(8):
        assert same(y * 8 + 0, y * 8 + 1) and same(y * 8 + 7, y * 8 + 6)
        assert same(y, 8 + y) and same(7 * 8 + y, 6 * 8 + y)


def test_wave2x2_varies_where_quads_repeat():
    # criterion 3 / Fig. 2: under the quad intrinsic all four lanes of a quad
    # hold the same texels; the 2x2 wave footprints vary between neighbours,
    # so no 2x2 block of lanes shares one member set
    def blocks_with_one_set(kind):
        s = [frozenset(r.tolist()) for r in o.footprint_members(kind)]
        n = 0
        for y in range(7):
            for x in range(7):
                ids = [(y + b) * 8 + x + a for b in range(2) for a in range(2)]
                n += len({s[i] for i in ids}) == 1
        return n, len(set(s))
    quad_blocks, quad_sets = blocks_with_one_set("quad2x2")
    wave_blocks, wave_sets = blocks_with_one_set("wave2x2")
    assert quad_blocks == 16 and quad_sets == 16
    assert wave_blocks == 0 and wave_sets > 2 * quad_sets
    # and each 2x2 wave window is placed by the pixel's own parity pattern:
    # the origin is the pixel itself or one lane before it on each axis
    m = o.footprint_members("wave2x2")
    for q in range(64):
        lx, ly = q % 8, q // 8
        ox, oy = (m[q] % 8).min(), (m[q] // 8).min()
        assert ox in (lx - 1, lx, 6) and oy in (ly - 1, ly, 6)
