"""Exact filtering (Sec. 4.2) on the GPU against the FP64 oracle, through the
C ABI: selection bit-exact, colours within 1e-5 relative (as the other
parity tests); where the whole-tile picks cover a pixel's support the GPU
value is the GPU's own Eq. (3) value bit for bit."""
import numpy as np
import pytest

import oracle as o
import workloads as w

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu
REL = 1e-5
FILTERS = {"bilinear": o.BILINEAR, "bicubic": o.BICUBIC}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def image(vals, uv):
    return o.tiles_to_image(vals, o.all_tiles(uv.shape[1], uv.shape[0]), uv.shape[1], uv.shape[0])


def support_scale(tex, uv, filt):
    T = np.abs(o.texture_values(tex))
    th, tw = T.shape[:2]
    n, d = (4, 1) if filt == o.BICUBIC else (2, 0)
    i0x, _ = o.split_coord(o.texel_float_coord(uv[..., 0], tw))
    i0y, _ = o.split_coord(o.texel_float_coord(uv[..., 1], th))
    m = np.zeros(uv.shape[:2] + (T.shape[2],))
    for b in range(n):
        for a in range(n):
            m = np.maximum(m, T[(i0y - d + b) % th, (i0x - d + a) % tw])
    return m


def rotated_screen(width, height, tex_size, mag, angle, off):
    py, px = np.mgrid[0:height, 0:width].astype(np.float64)
    x, y = (px + 0.5) / mag, (py + 0.5) / mag
    c, s = np.cos(angle), np.sin(angle)
    return (np.stack([c * x - s * y + off[0], s * x + c * y + off[1]], -1) / tex_size).astype(np.float32)


@pytest.mark.parametrize("filt", ["bilinear", "bicubic"])
@pytest.mark.parametrize("fp", ["quad2x2", "wave2x2", "square3x3", "square4x4", "tile8x8", "lut"])
@pytest.mark.parametrize("texkind", ["rgba8", "rgba16f", "rg16f"])
def test_exact_filtering_parity(filt, fp, texkind):
    rng = np.random.default_rng(7)
    if texkind == "rgba8":
        tex = w.small_texture(3, 64)
    elif texkind == "rgba16f":
        tex = rng.random((64, 64, 4)).astype(np.float16)
    else:
        tex = (rng.random((64, 64, 2)) * 2 - 1).astype(np.float16)
    uv = rotated_screen(100, 60, 64, 7.0, 0.3, (5.2, 9.7))
    lut = rng.integers(0, 64, (64, 12)).astype(np.uint8) if fp == "lut" else None
    outs, sel = stf.filter_reuse([dev(tex)], dev(uv), fp, filt, 4, 2, lut=dev(lut) if lut is not None else None,
                                 sel=True, exact_filtering=True)
    (rv, rs), = o.stf_filter_reuse([tex], uv, FILTERS[filt], 4, 2, fp, lut=lut, exact_filtering=True)
    assert np.array_equal(host(sel)[0], image(rs, uv))
    got = host(outs[0]).astype(np.float64)
    want = image(rv, uv)
    tol = REL * np.maximum(np.abs(want), support_scale(tex, uv, FILTERS[filt])) + 1e-30
    bad = np.abs(got - want) > tol
    assert not bad.any(), f"{bad.sum()} values beyond tolerance"


@pytest.mark.parametrize("fp", ["quad2x2", "square3x3", "tile8x8"])
@pytest.mark.parametrize("nt", [2, 3, 4])
def test_exact_filtering_several_textures(fp, nt):
    """Exact filtering with two to four textures of different formats and
    sizes in one call (with three or more the slots run one after another)."""
    rng = np.random.default_rng(9)
    texs = [w.small_texture(3, 64), rng.random((64, 64, 4)).astype(np.float16),
            (rng.random((32, 32, 2)) * 2 - 1).astype(np.float16),
            rng.integers(0, 256, (16, 16, 1), dtype=np.uint8)][:nt]
    uv = rotated_screen(90, 50, 64, 6.0, 0.4, (3.1, 7.3))
    outs, sel = stf.filter_reuse([dev(t) for t in texs], dev(uv), fp, "bicubic", 6, 1, sel=True,
                                 exact_filtering=True)
    ref = o.stf_filter_reuse(texs, uv, o.BICUBIC, 6, 1, fp, exact_filtering=True)
    sel = host(sel)
    for i, (tex, (rv, rs)) in enumerate(zip(texs, ref)):
        assert np.array_equal(sel[i], image(rs, uv)), f"slot {i} selection"
        got = host(outs[i]).astype(np.float64)
        want = image(rv, uv)
        tol = REL * np.maximum(np.abs(want), support_scale(tex, uv, o.BICUBIC)) + 1e-30
        bad = np.abs(got - want) > tol
        assert not bad.any(), f"slot {i}: {bad.sum()} values beyond tolerance"


@pytest.mark.parametrize("texkind", ["rgba16f", "rgba32f", "r8"])
def test_covered_pixels_equal_gpu_reference_bitwise(texkind):
    rng = np.random.default_rng(2)
    tex = {"rgba16f": rng.random((32, 32, 4)).astype(np.float16),
           "rgba32f": rng.random((32, 32, 4)).astype(np.float32),
           "r8": rng.integers(0, 256, (32, 32, 1), dtype=np.uint8)}[texkind]
    uv = w.small_screen(128, 96, 32, 9.0, offset_seed=3)
    t, duv = [dev(tex)], dev(uv)
    ef = host(stf.filter_reuse(t, duv, "tile8x8", "bilinear", 1, 0, exact_filtering=True)[0])
    wis = host(stf.filter_reuse(t, duv, "tile8x8", "bilinear", 1, 0)[0])
    ref = host(stf.filter_reference(t, duv, "bilinear")[0])
    (rv, _), = o.stf_filter_reuse([tex], uv, o.BILINEAR, 1, 0, "tile8x8", exact_filtering=True)
    oref = image(o.reference_filter([tex], uv, o.BILINEAR)[0], uv)
    covered = np.all(image(rv, uv) == oref, -1)
    assert covered.mean() > 0.5
    assert np.array_equal(ef[covered], ref[covered])
    assert np.array_equal(ef[~covered], wis[~covered])


def test_exact_filtering_lowers_error_over_frames():
    tex = w.small_texture(0, 256)
    uv = w.small_screen(512, 512, 256, 8.0)
    t, duv = [dev(tex)], dev(uv)
    ref = stf.filter_reference(t, duv, "bilinear")[0]
    e = {False: 0.0, True: 0.0}
    for frame in range(8):
        for ef in (False, True):
            out = stf.filter_reuse(t, duv, "quad2x2", "bilinear", 0, frame, exact_filtering=ef)[0]
            e[ef] += float(torch.mean((out - ref) ** 2))
    assert e[True] < e[False]
