"""Four-texture 4K material workload: 3840x2160 perspective plane, albedo
RGBA8 2048^2 + normal RG16F 2048^2 + roughness R8 1024^2 + mask R8 512^2,
frames with Halton sub-pixel jitter and frame-indexed seeds, bilinear and
bicubic, one-tap / reuse / deterministic. Parity on sampled tiles (selection
bit-exact, colours to 1e-5 relative) plus multi-frame properties."""
import numpy as np
import pytest

import oracle as o
import workloads as w

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu
W4K, H4K = 3840, 2160


@pytest.fixture(scope="module")
def scene():
    texs = w.material_set(0)
    return texs, [torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in texs]


def frame_uv(frame):
    uv, _, _, _ = w.perspective_plane(W4K, H4K, 2048, 2.0, 32.0, jitter=w.frame_jitter(frame))
    return uv


def support_scale(tex, uv, filt):
    T = np.abs(o.decode_texels(tex))
    th, tw = tex.shape[:2]
    n, d = (4, 1) if filt == o.BICUBIC else (2, 0)
    i0x, _ = o.split_coord(o.texel_float_coord(uv[..., 0], tw))
    i0y, _ = o.split_coord(o.texel_float_coord(uv[..., 1], th))
    m = np.zeros(uv.shape[:-1] + (tex.shape[2],))
    for b in range(n):
        for a in range(n):
            m = np.maximum(m, T[(i0y - d + b) % th, (i0x - d + a) % tw])
    return m


@pytest.mark.parametrize("filt,fp,frame", [("bicubic", "tile8x8", 3), ("bilinear", "quad2x2", 7),
                                           ("bicubic", None, 11)])
def test_four_texture_4k_sampled_parity(scene, filt, fp, frame):
    texs, dt = scene
    uv = frame_uv(frame)
    duv = torch.from_numpy(uv).cuda()
    seed = 1000 + frame                      # frame-indexed seed
    ftag = o.BICUBIC if filt == "bicubic" else o.BILINEAR
    if fp is None:
        outs, sel = stf.filter(dt, duv, filt, seed, frame, sel=True)
    else:
        outs, sel = stf.filter_reuse(dt, duv, fp, filt, seed, frame, sel=True)
    torch.cuda.synchronize()
    tiles_all = o.all_tiles(W4K, H4K)
    tiles = tiles_all[np.random.default_rng(frame).choice(len(tiles_all), 300, replace=False)]
    if fp is None:
        ref = o.stf_filter(texs, uv, ftag, seed, frame, tiles=tiles)
    else:
        ref = o.stf_filter_reuse(texs, uv, ftag, seed, frame, fp, tiles=tiles)
    px = tiles[:, 0:1] * 8 + (np.arange(64) % 8)[None]
    py = tiles[:, 1:2] * 8 + (np.arange(64) // 8)[None]
    sel_h = sel.cpu().numpy()
    for slot, tex in enumerate(texs):
        assert np.array_equal(sel_h[slot][py, px], ref[slot][1]), f"slot {slot} selection"
        g = outs[slot].cpu().numpy()[py, px].astype(np.float64)
        want = ref[slot][0]
        sc = support_scale(tex, uv[py, px], ftag)
        tol = 1e-5 * np.maximum(np.abs(want), sc) + 1e-30
        assert np.all(np.abs(g - want) <= tol), f"slot {slot} colours"


def test_sixteen_frames_converge_and_reuse_beats_stf(scene):
    """Averaging 16 jittered frames with frame-indexed seeds: reuse is
    closer to the deterministic filter than one-tap STF for every texture
    (per-frame and averaged), at 1/4 resolution to keep the test short."""
    texs, dt = scene
    errs_r, errs_s = np.zeros(4), np.zeros(4)
    for frame in range(16):
        uv, _, _, _ = w.perspective_plane(960, 540, 2048, 2.0, 32.0, jitter=w.frame_jitter(frame))
        duv = torch.from_numpy(uv).cuda()
        ref = stf.filter_reference(dt, duv, "bicubic")
        r = stf.filter_reuse(dt, duv, "tile8x8", "bicubic", 1000 + frame, frame)
        s = stf.filter(dt, duv, "bicubic", 1000 + frame, frame)
        for t in range(4):
            errs_r[t] += float(((r[t] - ref[t]) ** 2).mean())
            errs_s[t] += float(((s[t] - ref[t]) ** 2).mean())
    assert np.all(errs_r < errs_s), (errs_r, errs_s)
