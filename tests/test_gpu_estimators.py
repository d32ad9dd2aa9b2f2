"""The comparison estimators of Sec. 4.1 (IS, MIS balance heuristic,
pairwise MIS, regression; each also clamped) on the GPU against the FP64
oracle, through the C ABI. Selection is bit-exact. These estimators are not
convex combinations, so the FP32 tolerance is 1e-5 relative to the sum of
the absolute terms each estimate adds up (the oracle's "magnitude").

Every pixel is compared, the regression estimate too, whose coefficient
beta = sum d_i w_i T_i / D (d_i = w_i - wbar, D = sum d_i^2) amplifies
rounding: each d_i carries an absolute error of a few units of rounding u
times |w_i| + |wbar| (FP32 w_i and wbar), so by Cauchy-Schwarz the relative
errors of D and of the numerator are at most c u sum (|w_i| + |wbar|) |d_i| / D
<= 2 c u sqrt(sum w_i^2 / D) = 2 c u / sqrt(spread), spread = D / sum w_i^2.
beta enters the estimate as beta cv / n, a term of the magnitude, so the
tolerance of the regression estimate is the magnitude's divided by
sqrt(spread) (1e-5 is far above 2 c u for the handful of roundings here);
where spread is so small that this exceeds the magnitude itself, FP32 may
legitimately find D = 0 and beta = 0, and the bound still covers it."""
import numpy as np
import pytest

import oracle as o
from oracle import estimators_oracle as eo
import workloads as w

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu
REL = 1e-5
FILTERS = {"bilinear": o.BILINEAR, "bicubic": o.BICUBIC}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def image(vals, uv):
    return o.tiles_to_image(vals, o.all_tiles(uv.shape[1], uv.shape[0]), uv.shape[1], uv.shape[0])


def rotated_screen(width, height, tex_size, mag, angle, off):
    py, px = np.mgrid[0:height, 0:width].astype(np.float64)
    x, y = (px + 0.5) / mag, (py + 0.5) / mag
    c, s = np.cos(angle), np.sin(angle)
    return (np.stack([c * x - s * y + off[0], s * x + c * y + off[1]], -1) / tex_size).astype(np.float32)


# the plain Eq. (14) estimator without clamping is the optimised path, covered by the parity tests
ESTIMATOR_CASES = [(e, c) for e in ["is", "mis", "pmis", "regression", "wis"] for c in (False, True)
                   if (e, c) != ("wis", False)]


@pytest.mark.parametrize("est,clamp", ESTIMATOR_CASES)
@pytest.mark.parametrize("filt,fp", [("bilinear", "quad2x2"), ("bilinear", "square3x3"), ("bicubic", "square3x3"),
                                     ("bicubic", "wave2x2"), ("bilinear", "lut"), ("bicubic", "tile8x8")])
def test_estimator_parity(est, clamp, filt, fp):
    rng = np.random.default_rng(5)
    tex = (rng.random((64, 64, 4)) * 2 - 0.5).astype(np.float16)
    uv = rotated_screen(72, 40, 64, 3.0, 0.35, (4.1, 7.3))
    lut = rng.integers(0, 64, (64, 10)).astype(np.uint8) if fp == "lut" else None
    out, sel = stf.filter_reuse([dev(tex)], dev(uv), fp, filt, 8, 3, lut=dev(lut) if lut is not None else None,
                                sel=True, estimator=est, clamp=clamp)
    diag = []
    (rv, rs), = eo.stf_filter_estimator([tex], uv, FILTERS[filt], 8, 3, fp, est, clamp=clamp, lut=lut,
                                        diagnostics=diag)
    torch.cuda.synchronize()
    assert np.array_equal(sel.cpu().numpy()[0], image(rs, uv))
    got = out[0].cpu().numpy().astype(np.float64)
    want = image(rv, uv)
    mag = image(diag[0]["magnitude"], uv)
    cond = np.ones(want.shape)
    if est == "regression":
        spread = image(diag[0]["spread"][..., None], uv)
        cond = np.broadcast_to(1.0 / np.sqrt(np.clip(spread, 1e-300, 1.0)), want.shape)
    tol = REL * np.maximum(mag, np.abs(want)) * cond + 1e-30
    err = np.abs(got - want)
    bad = err > tol
    assert not bad.any(), f"{bad.sum()} beyond tolerance, worst {np.max(err / tol):.3g}x"


def test_estimators_rank_like_the_paper_on_the_magnified_plane():
    # Sec. 5.1: Eq. (14) has lower error than IS, MIS and regression at
    # magnification; clamping lowers the error of the unbounded estimators
    tex = w.plane_albedo(0, 256)
    uv, _, _, _ = w.perspective_plane(480, 272, 256, 4.0, 16.0)
    dt, duv = [dev(tex)], dev(uv)
    ref = stf.filter_reference(dt, duv, "bilinear")[0]

    def mse(est, clamp=False):
        e = 0.0
        for frame in range(4):
            outp = stf.filter_reuse(dt, duv, "square3x3", "bilinear", 0, frame, estimator=est, clamp=clamp)[0]
            e += float(torch.mean((outp[..., :3] - ref[..., :3]) ** 2))
        return e

    e = {k: mse(k) for k in ("wis", "is", "mis", "pmis", "regression")}
    ec = {k: mse(k, True) for k in ("is", "mis", "regression")}
    assert e["wis"] < min(e["is"], e["mis"], e["regression"])
    for k in ec:
        assert ec[k] <= e[k]
