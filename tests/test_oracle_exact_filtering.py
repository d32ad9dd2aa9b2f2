"""Pins of the oracle's exact filtering (Sec. 4.2, "Exact Filtering"): when
the samples shared within a pixel's footprint include every texel of
positive weight under its filter, the pixel returns the deterministic value
of Eq. (3); otherwise the estimator of Eq. (14)."""
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import oracle as o
import workloads as w
from test_oracle_estimator import screen, img, wis_fraction


def covered_from_scratch(c, sels, uvx, uvy, size, filt, members):
    """Whether the selections of c's members include every positive-weight
    texel of c's support (texel identity modulo the size)."""
    x = o.texel_float_coord(uvx[c], size); y = o.texel_float_coord(uvy[c], size)
    i0x, Fx = map(int, o.split_coord(x)); i0y, Fy = map(int, o.split_coord(y))
    d = 1 if filt == o.BICUBIC else 0
    wxi = o.axis_weights_int(np.array([Fx]), filt)[0]
    wyi = o.axis_weights_int(np.array([Fy]), filt)[0]
    need = {((i0x - d + a) % size, (i0y - d + b) % size)
            for a in range(len(wxi)) for b in range(len(wyi)) if wxi[a] > 0 and wyi[b] > 0}
    have = {sels[i] for i in members[c]}
    return need <= have


def exact_value(c, uvx, uvy, T, filt):
    size = T.shape[0]
    x = o.texel_float_coord(uvx[c], size); y = o.texel_float_coord(uvy[c], size)
    i0x, Fx = map(int, o.split_coord(x)); i0y, Fy = map(int, o.split_coord(y))
    d = 1 if filt == o.BICUBIC else 0
    wxi = o.axis_weights_int(np.array([Fx]), filt)[0]
    wyi = o.axis_weights_int(np.array([Fy]), filt)[0]
    den = o.weight_denominator(filt)
    acc = Fraction(0)
    for a, b in product(range(len(wxi)), range(len(wyi))):
        acc += Fraction(int(wxi[a]), den) * Fraction(int(wyi[b]), den) * \
            Fraction(float(T[(i0y - d + b) % size, (i0x - d + a) % size]))
    return acc


@pytest.mark.parametrize("fp", ["quad2x2", "tile8x8"])
def test_exact_filtering_brute_force_bilinear(fp):
    """2x2 pixel screen, bilinear: (a) per seed the oracle returns Eq. (3)
    exactly when the four selections cover the pixel's positive-weight
    texels and Eq. (14) otherwise; (b) the mean over seeds matches the exact
    expectation over every joint selection."""
    tex = np.random.default_rng(21).random((8, 8, 1)).astype(np.float32)
    uv = screen(2, 2, 8, 8.0, off=(3.0, 4.0), angle=0.1)
    uvx, uvy = uv[..., 0].reshape(-1), uv[..., 1].reshape(-1)
    den = o.weight_denominator(o.BILINEAR)
    members = {c: list(range(4)) for c in range(4)}
    cands = []
    for c in range(4):
        x = o.texel_float_coord(uvx[c], 8); y = o.texel_float_coord(uvy[c], 8)
        i0x, Fx = map(int, o.split_coord(x)); i0y, Fy = map(int, o.split_coord(y))
        wxi = o.axis_weights_int(np.array([Fx]), o.BILINEAR)[0]
        wyi = o.axis_weights_int(np.array([Fy]), o.BILINEAR)[0]
        cands.append([((i0x + a) % 8, (i0y + b) % 8, Fraction(int(wxi[a]), den) * Fraction(int(wyi[b]), den))
                      for a, b in product(range(2), range(2)) if wxi[a] > 0 and wyi[b] > 0])

    def value(c, sels, probs):
        if covered_from_scratch(c, sels, uvx, uvy, 8, o.BILINEAR, members):
            return exact_value(c, uvx, uvy, tex[..., 0], o.BILINEAR)
        return wis_fraction(c, sels, probs, uvx, uvy, tex[..., 0], o.BILINEAR, members)

    E = np.zeros(4); E2 = np.zeros(4); p_cov = np.zeros(4)
    for combo in product(*cands):
        pj = 1.0
        for cnd in combo:
            pj *= float(cnd[2])
        sels = {i: combo[i][:2] for i in range(4)}
        probs = {i: combo[i][2] for i in range(4)}
        for c in range(4):
            v = float(value(c, sels, probs))
            E[c] += pj * v; E2[c] += pj * v * v
            p_cov[c] += pj * covered_from_scratch(c, sels, uvx, uvy, 8, o.BILINEAR, members)
    assert np.all(p_cov > 0.05)                 # the case is exercised
    tid = [0, 1, 8, 9]
    N = 300
    acc = np.zeros(4)
    n_exact = 0
    for seed in range(N):
        (v, sel), = o.stf_filter_reuse([tex], uv, o.BILINEAR, seed, 0, fp, exact_filtering=True)
        sels = {i: tuple(int(t) for t in sel[0, tid[i]]) for i in range(4)}
        probs = {i: next(p for cx, cy, p in cands[i] if (cx, cy) == sels[i]) for i in range(4)}
        for c in range(4):
            want = float(value(c, sels, probs))
            assert abs(v[0, tid[c], 0] - want) < 1e-12
            acc[c] += v[0, tid[c], 0]
            n_exact += covered_from_scratch(c, sels, uvx, uvy, 8, o.BILINEAR, members)
    assert n_exact > 0
    sd = np.sqrt(np.maximum(E2 - E ** 2, 1e-18))
    assert np.all(np.abs(acc / N - E) < 5.5 * sd / np.sqrt(N) + 1e-12)


@pytest.mark.parametrize("filt", [o.BILINEAR, o.BICUBIC])
def test_exact_filtering_is_reference_or_estimator(filt):
    tex = np.random.default_rng(3).random((16, 16, 3))
    uv = screen(24, 16, 16, 6.0, off=(2.3, 5.1), angle=0.2)
    wis = img(o.stf_filter_reuse([tex], uv, filt, 5, 1, "tile8x8")[0][0], uv)
    ef = img(o.stf_filter_reuse([tex], uv, filt, 5, 1, "tile8x8", exact_filtering=True)[0][0], uv)
    ref = img(o.reference_filter([tex], uv, filt)[0], uv)
    is_ref = np.all(np.isclose(ef, ref, rtol=0, atol=1e-13), -1)
    is_wis = np.all(ef == wis, -1)
    assert np.all(is_ref | is_wis)
    if filt == o.BILINEAR:
        assert is_ref.mean() > 0.3               # at 6x bilinear the tile covers most supports


def test_exact_filtering_constant_and_self():
    tex = np.full((8, 8, 2), 0.625)
    uv = screen(16, 16, 8, 3.0)
    v = o.stf_filter_reuse([tex], uv, o.BILINEAR, 1, 0, "square3x3", exact_filtering=True)[0][0]
    assert np.allclose(v, 0.625, rtol=0, atol=1e-15)
    # one sample covers the support only where a single texel has positive
    # weight; there the texel is also the Eq. (3) value
    tex = np.random.default_rng(0).random((8, 8, 1))
    a = o.stf_filter_reuse([tex], uv, o.BILINEAR, 2, 0, "self", exact_filtering=True)[0][0]
    b = o.stf_filter_reuse([tex], uv, o.BILINEAR, 2, 0, "self")[0][0]
    assert np.allclose(a, b, rtol=0, atol=1e-15)


def test_exact_filtering_lowers_error_on_magnified_texture():
    # the paper reports lower error with exact filtering for bilinear; on the
    # small magnified workload the mean squared error over 24 frames drops
    tex = w.small_texture(0, 64)
    uv = w.small_screen(64, 64, 64, 4.0, offset_seed=1)
    ref = img(o.reference_filter([tex], uv, o.BILINEAR)[0], uv)
    for fp in ("quad2x2", "square3x3"):
        e_wis = e_ef = 0.0
        for frame in range(24):
            e_wis += np.mean((img(o.stf_filter_reuse([tex], uv, o.BILINEAR, 0, frame, fp)[0][0], uv) - ref) ** 2)
            e_ef += np.mean((img(o.stf_filter_reuse([tex], uv, o.BILINEAR, 0, frame, fp,
                                                    exact_filtering=True)[0][0], uv) - ref) ** 2)
        assert e_ef < e_wis, fp
