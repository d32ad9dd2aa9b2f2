"""Pins of the oracle's comparison estimators (Sec. 4.1): IS, MIS balance
heuristic, pairwise MIS, the regression estimator and their clamped
variants, against what the mathematics fixes: unbiasedness of the MIS
forms (their mean over seeds converges to Eq. (3)), the closed-form
expectation of IS, exactness of the control variate on constant textures,
reduction to one-tap STF, and the clamp bounds."""
import numpy as np
import pytest

import oracle as o
from oracle import estimators_oracle as eo
from test_oracle_estimator import screen, img


def run(est, tex, uv, filt, seed, fp, clamp=False, lut=None, frame=0):
    return img(eo.stf_filter_estimator([tex], uv, filt, seed, frame, fp, est, clamp=clamp, lut=lut)[0][0], uv)


@pytest.mark.parametrize("est", ["mis", "pmis"])
@pytest.mark.parametrize("fp", ["quad2x2", "square3x3"])
def test_mis_forms_are_unbiased(est, fp):
    tex = np.random.default_rng(4).random((8, 8, 1))
    uv = screen(6, 6, 8, 1.7, off=(2.2, 3.1), angle=0.4)
    ref = img(o.reference_filter([tex], uv, o.BILINEAR)[0], uv)
    N = 1500
    vals = np.stack([run(est, tex, uv, o.BILINEAR, s, fp) for s in range(N)])
    mean, sd = vals.mean(0), vals.std(0)
    assert np.all(np.abs(mean - ref) <= 6.0 * sd / np.sqrt(N) + 1e-12)
    # and IS and WIS are biased here: their means miss Eq. (3) somewhere
    wis = np.stack([run("wis", tex, uv, o.BILINEAR, s, fp) for s in range(300)]).mean(0)
    assert np.max(np.abs(wis - ref)) > 1e-3


def test_is_expectation_closed_form():
    # E[IS] = (1/n) sum_i sum_{x in supp p_i} f_c(x) T(x): each shared sample
    # only sees the part of c's filter inside its own PMF's support
    tex = np.random.default_rng(6).random((8, 8, 1))
    uv = screen(4, 4, 8, 1.3, off=(2.6, 1.7), angle=0.2)
    uvx, uvy = uv[..., 0].reshape(-1), uv[..., 1].reshape(-1)
    den = o.weight_denominator(o.BILINEAR)

    def support(c):
        x = o.texel_float_coord(uvx[c], 8); y = o.texel_float_coord(uvy[c], 8)
        i0x, Fx = map(int, o.split_coord(x)); i0y, Fy = map(int, o.split_coord(y))
        wxi = o.axis_weights_int(np.array([Fx]), o.BILINEAR)[0]
        wyi = o.axis_weights_int(np.array([Fy]), o.BILINEAR)[0]
        return {((i0x + a) % 8, (i0y + b) % 8): wxi[a] * wyi[b] / den ** 2
                for a in range(2) for b in range(2) if wxi[a] * wyi[b] > 0}

    sup = [support(c) for c in range(16)]
    members = o.footprint_members("quad2x2")
    tid = [ly * 8 + lx for ly in range(4) for lx in range(4)]
    expect = np.zeros(16)
    for c in range(16):
        mem = [tid.index(m) for m in members[tid[c]]]
        acc = 0.0
        for i in mem:
            acc += sum(sup[c].get(x, 0.0) * tex[x[1], x[0], 0] for x in sup[i])
        expect[c] = acc / len(mem)
    N = 3000
    vals = np.stack([run("is", tex, uv, o.BILINEAR, s, "quad2x2").reshape(-1) for s in range(N)])
    assert np.all(np.abs(vals.mean(0) - expect) <= 6.0 * vals.std(0) / np.sqrt(N) + 1e-12)


@pytest.mark.parametrize("est", ["is", "mis", "pmis", "regression", "wis"])
def test_identical_pmfs_give_the_sample_mean(est):
    # every pixel at the same uv: all PMFs equal, w_i = 1, and every
    # estimator returns the mean of the shared texels
    tex = np.random.default_rng(1).random((8, 8, 2))
    uv = np.full((8, 8, 2), 0.37, np.float32)
    got = eo.stf_filter_estimator([tex], uv, o.BICUBIC, 3, 0, "square3x3", est)[0]
    (_, sel), = o.stf_filter([tex], uv, o.BICUBIC, 3, 0)
    members = o.footprint_members("square3x3")
    T = tex[sel[0, :, 1], sel[0, :, 0]]
    want = T[members].mean(1)
    assert np.allclose(got[0][0], want, rtol=0, atol=1e-13)


def test_self_footprint_is_stf_for_every_estimator():
    tex = np.random.default_rng(2).random((16, 16, 3))
    uv = screen(16, 8, 16, 2.5)
    stf = img(o.stf_filter([tex], uv, o.BILINEAR, 4, 1)[0][0], uv)
    for est in ("is", "mis", "pmis", "regression"):
        assert np.allclose(run(est, tex, uv, o.BILINEAR, 4, "self", frame=1), stf, rtol=0, atol=1e-14), est


def test_regression_is_exact_on_constant_textures():
    tex = np.full((16, 16, 1), 0.3)
    uv = screen(16, 16, 16, 2.0, angle=0.3)
    got = run("regression", tex, uv, o.BICUBIC, 5, "square4x4")
    assert np.allclose(got, 0.3, rtol=0, atol=1e-12)
    # IS is not (its weights do not sum to n)
    assert np.max(np.abs(run("is", tex, uv, o.BICUBIC, 5, "square4x4") - 0.3)) > 1e-3


@pytest.mark.parametrize("est", ["is", "mis", "pmis", "regression", "wis"])
def test_clamp_bounds_and_wis_needs_none(est):
    tex = np.random.default_rng(9).random((16, 16, 2))
    uv = screen(24, 16, 16, 3.0, angle=0.2)
    v = eo.stf_filter_estimator([tex], uv, o.BICUBIC, 6, 0, "square3x3", est, clamp=True)[0][0]
    u = eo.stf_filter_estimator([tex], uv, o.BICUBIC, 6, 0, "square3x3", est)[0][0]
    assert np.all((v == u) | (v == v.clip(0, 1)))          # clamping only moves values inward
    assert np.all((v >= 0) & (v <= 1))                      # texels are in [0, 1]
    if est == "wis":                                        # Eq. (5): already inside the hull
        assert np.allclose(u, v, rtol=0, atol=1e-14)
