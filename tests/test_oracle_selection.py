"""Pins of one-tap STF texel selection and the hash (no GPU).

The selection law is checked as a black box: for each fraction, binary
search over h in [0, 2^32) finds where the selected offset steps up, and the
lengths of the resulting intervals are the selection probabilities.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as o


def boundaries(F: int, filt: str):
    """Smallest h with select(h) >= m for m = 1..n-1 (2^32 if none)."""
    wint = o.axis_weights_int(np.array([F]), filt)[0]
    n = len(wint)
    out = []
    for m in range(1, n):
        lo, hi = 0, 1 << 32                      # invariant: select(hi) >= m or hi = 2^32
        while lo < hi:
            mid = (lo + hi) // 2
            if o.select_axis(np.array([mid], dtype=np.int64), wint[None, :], filt)[0] >= m:
                hi = mid
            else:
                lo = mid + 1
        out.append(lo)
    return wint, out


FRACTIONS = [0, 1, 2, 255, 4096, 21845, 32768, 43690, 65534, 65535]


@pytest.mark.parametrize("F", FRACTIONS)
def test_bilinear_selection_probability_exact(F):
    wint, b = boundaries(F, o.BILINEAR)
    p1 = Fraction((1 << 32) - b[0], 1 << 32)
    assert p1 == Fraction(int(wint[1]), 1 << 16)   # P(k=1) = phi exactly


@pytest.mark.parametrize("F", FRACTIONS)
def test_bicubic_selection_probability_within_2_pow_minus_32(F):
    wint, b = boundaries(F, o.BICUBIC)
    edges = [0] + b + [1 << 32]
    den = 6 << 48
    for k in range(4):
        prob = Fraction(edges[k + 1] - edges[k], 1 << 32)
        assert abs(prob - Fraction(int(wint[k]), den)) <= Fraction(1, 1 << 32)
        if wint[k] == 0:
            assert prob == 0                      # a zero-weight texel is never chosen


def test_selection_monotone_in_h():
    rng = np.random.default_rng(3)
    F = rng.integers(0, 65536, 4000)
    for filt in (o.BILINEAR, o.BICUBIC):
        w = o.axis_weights_int(F, filt)
        h1 = rng.integers(0, 1 << 32, 4000)
        h2 = rng.integers(0, 1 << 32, 4000)
        lo, hi = np.minimum(h1, h2), np.maximum(h1, h2)
        assert np.all(o.select_axis(lo, w, filt) <= o.select_axis(hi, w, filt))
        k = o.select_axis(h1, w, filt)
        # the chosen texel always has a nonzero weight
        assert np.all(np.take_along_axis(w, k[:, None], 1)[:, 0] > 0)


def test_hash_uniformity_and_independence():
    # "parity unpinned" against the pcg4d publication (no test vectors offline):
    # pinned by statistical properties of its outputs over a pixel grid.
    py, px = np.mgrid[0:512, 0:512]
    hx, hy = o.slot_hash(px, py, 0, seed=0, frame=0)
    zx, zy = o.slot_hash(px, py, 1, seed=0, frame=0)
    n = px.size
    for h in (hx, hy, zx, zy):
        counts = np.bincount((h >> np.uint32(24)).astype(np.int64).ravel(), minlength=256)
        chi2 = ((counts - n / 256) ** 2 / (n / 256)).sum()
        assert chi2 < 255 + 6 * np.sqrt(2 * 255)           # ~6 sigma
        bits = ((h.ravel()[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(0)
        assert np.all(np.abs(bits - 0.5) < 6 * 0.5 / np.sqrt(n))
    # joint uniformity of the two coordinates a pixel uses
    cell = ((hx >> np.uint32(28)).astype(np.int64) * 16 + (hy >> np.uint32(28)).astype(np.int64)).ravel()
    counts = np.bincount(cell, minlength=256)
    chi2 = ((counts - n / 256) ** 2 / (n / 256)).sum()
    assert chi2 < 255 + 6 * np.sqrt(2 * 255)
    # neighbouring pixels and slots are uncorrelated
    a = (hx >> np.uint32(8)).astype(np.float64)
    for b in (np.roll(a, 1, 1), np.roll(a, 1, 0), (zx >> np.uint32(8)).astype(np.float64)):
        r = np.corrcoef(a.ravel(), b.ravel())[0, 1]
        assert abs(r) < 6 / np.sqrt(n)


def test_hash_streams_differ():
    py, px = np.mgrid[0:64, 0:64]
    base = o.slot_hash(px, py, 0, 0, 0)[0]
    for args in [(0, 1, 0), (0, 0, 1), (2, 0, 0)]:
        slot, seed, frame = args
        other = o.slot_hash(px, py, slot, seed, frame)[0]
        assert np.mean(other == base) < 0.01


def test_shared_selection_follows_the_first_slot_of_each_size():
    # Sec. 4.5: textures with the same UV and resolution may share one
    # selection; the leader of each size keeps its own random stream
    rng = np.random.default_rng(0)
    a = rng.random((32, 32, 4)); b = rng.random((32, 32, 2)); c = rng.random((16, 16, 1)); d = rng.random((16, 16, 1))
    uv = (rng.random((16, 24, 2)) * 0.8 + 0.1).astype(np.float32)
    assert o.selection_slots([a, b, c, d], True) == [0, 0, 2, 2]
    assert o.selection_slots([a, b, c, d], False) == [0, 1, 2, 3]
    shared = o.stf_filter([a, b, c, d], uv, o.BICUBIC, 3, 1, share_selection=True)
    plain = o.stf_filter([a, b, c, d], uv, o.BICUBIC, 3, 1)
    assert np.array_equal(shared[1][1], shared[0][1]) and np.array_equal(shared[3][1], shared[2][1])
    assert np.array_equal(shared[0][1], plain[0][1]) and np.array_equal(shared[2][1], plain[2][1])
    assert not np.array_equal(plain[1][1], plain[0][1])
    # the follower of slot 0 equals slot 0's stream applied to its texture
    (tb, sb), = o.stf_filter([b], uv, o.BICUBIC, 3, 1)
    assert np.array_equal(shared[1][1], sb) and np.array_equal(shared[1][0], tb)
