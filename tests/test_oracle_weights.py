"""Pins of the oracle's coordinates and filter weights against closed forms,
an independent B-spline definition and exact invariants (no GPU)."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL_F = np.arange(65536, dtype=np.int64)


def cox_de_boor(t: Fraction, p: int = 3) -> Fraction:
    """Centred uniform B-spline of degree p at t, by the Cox-de Boor
    recursion on integer knots (independent of the closed-form pieces)."""
    def N(i, k, x):
        if k == 0:
            return Fraction(1) if i <= x < i + 1 else Fraction(0)
        return (x - i) / k * N(i, k - 1, x) + (i + k + 1 - x) / k * N(i + 1, k - 1, x)
    return N(0, p, t + Fraction(p + 1, 2))


def test_bilinear_weights_sum_exactly():
    w = o.axis_weights_int(ALL_F, o.BILINEAR)
    assert np.all(w.sum(-1) == 1 << 16)
    assert np.all(w >= 0)


def test_bicubic_weights_sum_exactly_for_every_fraction():
    w = o.axis_weights_int(ALL_F, o.BICUBIC)
    assert np.all(w.sum(-1) == 6 * (1 << 48))
    assert np.all(w >= 0)


def test_bicubic_symmetry():
    # reflecting phi -> 1 - phi reverses the order of the four texels
    F = ALL_F[1:]
    a = o.axis_weights_int(F, o.BICUBIC)
    b = o.axis_weights_int((1 << 16) - F, o.BICUBIC)
    assert np.array_equal(a, b[:, ::-1])


def test_bicubic_golden_quarter_points():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "bspline_quarter_points.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        num, den, w0, w1, w2, w3, d = map(int, r)
        F = (num << 16) // den
        wint = o.axis_weights_int(np.array([F]), o.BICUBIC)[0]
        for got, want in zip(wint, (w0, w1, w2, w3)):
            assert Fraction(int(got), 6 << 48) == Fraction(want, d)


@pytest.mark.parametrize("F", [0, 1, 7, 12345, 32768, 40000, 65535])
def test_bicubic_matches_cox_de_boor(F):
    phi = Fraction(F, 1 << 16)
    wint = o.axis_weights_int(np.array([F]), o.BICUBIC)[0]
    dists = [1 + phi, phi, 1 - phi, 2 - phi]          # |x - texel| for i0-1 .. i0+2
    for got, t in zip(wint, dists):
        assert Fraction(int(got), 6 << 48) == cox_de_boor(t)


@pytest.mark.parametrize("filt,delta", [(o.BILINEAR, 0), (o.BICUBIC, 1)])
def test_linear_precision(filt, delta):
    # both filters reproduce linear functions: sum_k w_k (k - delta) = phi
    w = o.axis_weights_int(ALL_F, filt)
    k = np.arange(w.shape[-1]) - delta
    den = o.weight_denominator(filt)
    lhs = (w * k).sum(-1)
    # lhs / den == F / 2^16  <=>  lhs * 2^16 == F * den  (integers; den/2^16 exact)
    assert np.all(lhs == ALL_F * (den >> 16))


def test_bicubic_second_moment():
    # the cubic B-spline has variance 4/12: sum_k w_k (k - 1 - phi)^2 = 1/3
    for F in [0, 3, 999, 32768, 65535]:
        phi = Fraction(F, 1 << 16)
        w = o.axis_weights_int(np.array([F]), o.BICUBIC)[0]
        m2 = sum(Fraction(int(wk), 6 << 48) * (k - 1 - phi) ** 2 for k, wk in enumerate(w))
        assert m2 == Fraction(1, 3)


def test_bilinear_equals_getfilterpmf_listing():
    # Sec. S6: pmf = clamp(1 - |texelFloatCoords - texelIntCoords|, 0, 1) per axis
    rng = np.random.default_rng(0)
    x = (rng.random(2000) * 64 - 8).astype(np.float32)
    i0, F = o.split_coord(x)
    xq = i0 + F / 65536.0                         # the quantised coordinate
    w = o.axis_weights(F, o.BILINEAR)
    for off in range(-1, 3):
        listing = np.clip(1.0 - np.abs(xq - (i0 + off)), 0.0, 1.0)
        mine = w[:, off] if off in (0, 1) else np.zeros_like(listing)
        assert np.array_equal(mine, listing)


def test_texel_float_coord_is_fp32_listing():
    rng = np.random.default_rng(1)
    u = np.concatenate([rng.random(5000), rng.random(100) * 3 - 1, [0.0, 1.0, -0.0, 1e-30, 0.5]])
    u = u.astype(np.float32)
    for size in (256, 2048, 1000, 3):
        want = np.float32(u) * np.float32(size) - np.float32(0.5)   # IEEE FP32 ops
        got = o.texel_float_coord(u, size)
        assert np.array_equal(got.view(np.uint32), want.astype(np.float32).view(np.uint32))


def test_split_coord_definition():
    rng = np.random.default_rng(2)
    xs = np.concatenate([rng.random(3000) * 4096 - 2048,
                         [-1e-10, -0.3, -1.0, 0.0, 1e-9, 0.99999994, 2047.9999, -2048.0]]).astype(np.float32)
    i0, F = o.split_coord(xs)
    for x, i, f in zip(xs, i0, F):
        xf = Fraction(float(x))
        assert 0 <= f < 65536
        assert Fraction(int(i)) + Fraction(int(f), 65536) <= xf < Fraction(int(i)) + Fraction(int(f) + 1, 65536)
