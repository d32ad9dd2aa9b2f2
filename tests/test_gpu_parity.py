"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar: texel selection bit-exact; colours within 1e-5 relative to the larger
of |oracle| and the largest texel magnitude under the pixel's own filter
(the FP32 convex combination has no cancellation, so its error scales with
the texels it mixes). Inputs are seeded and synthetic.
"""
import numpy as np
import pytest

import oracle as o
import workloads as w

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu
REL = 1e-5
FILTERS = {"bilinear": o.BILINEAR, "bicubic": o.BICUBIC}
ALL_FP = ["self", "quad2x2", "wave2x2", "square3x3", "square4x4", "tile8x8"]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def support_scale(tex, uv, filt):
    """Per pixel and channel: max |T| over the pixel's own filter support."""
    T = np.abs(o.decode_texels(tex))
    th, tw = tex.shape[:2]
    n, d = (4, 1) if filt == o.BICUBIC else (2, 0)
    i0x, _ = o.split_coord(o.texel_float_coord(uv[..., 0], tw))
    i0y, _ = o.split_coord(o.texel_float_coord(uv[..., 1], th))
    m = np.zeros(uv.shape[:2] + (tex.shape[2],))
    for b in range(n):
        for a in range(n):
            m = np.maximum(m, T[(i0y - d + b) % th, (i0x - d + a) % tw])
    return m


def assert_close(gpu, ref, scale, what=""):
    tol = REL * np.maximum(np.abs(ref), scale) + 1e-30
    err = np.abs(gpu.astype(np.float64) - ref)
    bad = err > tol
    assert not bad.any(), f"{what}: {bad.sum()} values beyond tolerance, worst {np.max(err / tol):.3g}x"


def oracle_image(vals, uv, tiles=None):
    if tiles is None:
        tiles = o.all_tiles(uv.shape[1], uv.shape[0])
    return o.tiles_to_image(vals, tiles, uv.shape[1], uv.shape[0])


def run_case(texs, uv, filt, fp, seed=0, frame=0, lut=None):
    """Full-image parity of stf_filter_reuse (or stf_filter for fp=None)."""
    ftag = FILTERS[filt]
    dt = [dev(t) for t in texs]
    duv = dev(uv)
    if fp is None:
        outs, sel = stf.filter(dt, duv, filt, seed, frame, sel=True)
        ref = o.stf_filter(texs, uv, ftag, seed, frame)
    else:
        lut_t = dev(lut.astype(np.uint8)) if lut is not None else None
        outs, sel = stf.filter_reuse(dt, duv, fp, filt, seed, frame, lut=lut_t, sel=True)
        ref = o.stf_filter_reuse(texs, uv, ftag, seed, frame, fp, lut=lut)
    sel = host(sel)
    for slot, (tex, (rv, rs)) in enumerate(zip(texs, ref)):
        want_sel = oracle_image(rs, uv)
        assert np.array_equal(sel[slot], want_sel), f"slot {slot}: selection differs"
        gv = host(outs[slot])
        assert_close(gv, oracle_image(rv, uv), support_scale(tex, uv, ftag), f"slot {slot} {fp}")
    return outs, sel


def small_textures(seed=0):
    return [w.small_texture(seed)]


# --------------------------------------------------------------- small workload

@pytest.mark.parametrize("fp", [None, "self", "quad2x2"])
def test_small_workload_full(fp):
    """256^2 RGBA8, 512x512 fronto-parallel quad at 8x, bilinear, seed 0."""
    run_case(small_textures(), w.small_screen(), "bilinear", fp)


@pytest.mark.parametrize("filt", ["bilinear", "bicubic"])
@pytest.mark.parametrize("fp", ALL_FP + [None])            # None: one-tap STF (row-linear waves)
def test_all_footprints_ragged_screen(filt, fp):
    # 61x37: partial tiles on both axes; rotated quad at 3.3x
    tex = w.tile_texture_rgba8(3, 64)
    uv = w.small_screen(61, 37, 64, 3.3, offset_seed=4)
    run_case([tex], uv, filt, fp, seed=7, frame=3)


@pytest.mark.parametrize("fp", ["square3x3", "tile8x8"])
def test_multi_texture_formats(fp):
    texs = [w.plane_albedo(1, 64), w.plane_normal(1, 64), w.r8_texture(2, 32),
            np.random.default_rng(0).random((16, 16, 4)).astype(np.float32)]
    uv = w.small_screen(40, 24, 64, 5.0, offset_seed=1)
    run_case(texs, uv, "bicubic", fp, seed=11)


@pytest.mark.parametrize("k", [9, 16, 17, 40])
def test_lut_footprint(k):
    """Tables of up to 16 entries are read from LDS, longer ones from global memory."""
    rng = np.random.default_rng(5)
    lut = rng.integers(0, 64, (64, k))
    lut[::3, 0] = np.arange(64)[::3]          # some rows name the pixel itself
    uv = w.small_screen(48, 32, 64, 4.0, offset_seed=2)
    run_case([w.tile_texture_rgba8(1, 64)], uv, "bicubic", "lut", seed=2, lut=lut)


def test_tile_bins_fallback_under_minification():
    # texels 1.5 apart per pixel: the tile's texels exceed the bin window and
    # the kernel takes the per-record path; results must not change
    uv = w.small_screen(64, 64, 256, 1 / 1.5, offset_seed=3)
    run_case([w.small_texture(1)], uv, "bicubic", "tile8x8", seed=1)


@pytest.mark.parametrize("filt,mag,seam", [("bicubic", 1.05, False), ("bilinear", 0.85, False),
                                           ("bicubic", 1.05, True)])
def test_tile_bins_window_from_wave_minimum(filt, mag, seam):
    """Near 1x the tile's support starts spread over more texels than the
    window centred on lane 0 allows but at most 12 - N: the kernel places the
    window at the wave's smallest start instead (61x45 screen: partial tiles;
    seam: the screen starts 20 texels before the wrap-around in u and v, so
    windows straddle it)."""
    uv = w.small_screen(61, 45, 256, mag, offset_seed=2)
    if seam:
        uv = ((uv + np.float32(236.0 / 256.0)) % np.float32(1.0)).astype(np.float32)
    n, margin = (4, 4) if filt == "bicubic" else (2, 5)
    i0x, _ = o.split_coord(o.texel_float_coord(uv[:40, :56, 0], 256))
    starts = i0x.reshape(5, 8, 7, 8).swapaxes(1, 2).reshape(5, 7, 64)
    d = (starts - starts[..., :1] + 128) % 256 - 128                  # offsets across the wrap
    spread = d.max(-1) - d.min(-1)
    assert np.all(spread > margin) and np.all(spread <= 12 - n)      # full tiles: second placement
    run_case([w.small_texture(1)], uv, filt, "tile8x8", seed=6, frame=1)


def test_tiny_inputs():
    run_case([w.tile_texture_rgba8(1, 4)], w.small_screen(1, 1, 4, 2.0), "bicubic", "tile8x8")
    run_case([w.tile_texture_rgba8(1, 4)], w.small_screen(3, 9, 4, 2.0), "bilinear", "quad2x2")
    # one-tap STF runs row-linear: one lane of one wave, and a row shorter than a wave
    run_case([w.tile_texture_rgba8(1, 4)], w.small_screen(1, 1, 4, 2.0), "bicubic", None)
    run_case([w.tile_texture_rgba8(1, 4), w.r8_texture(2, 16)], w.small_screen(3, 9, 4, 2.0), "bilinear", None)


# --------------------------------------------------------------- plane workload

@pytest.fixture(scope="module")
def plane():
    uv, _, _, info = w.perspective_plane()
    return [w.plane_albedo(), w.plane_normal()], uv


def test_plane_selection_full_and_sampled_colours(plane):
    """1920x1080 perspective plane, 2048^2 RGBA16F + RG16F, bicubic, whole-tile
    reuse (the benchmarked launch): selection bit-exact and colours within
    the tolerance on every pixel of both textures."""
    texs, uv = plane
    dt = [dev(t) for t in texs]
    duv = dev(uv)
    outs, sel = stf.filter_reuse(dt, duv, "tile8x8", "bicubic", 0, 0, sel=True)
    sel = host(sel)
    tiles_all = o.all_tiles(1920, 1080)
    for slot, tex in enumerate(texs):
        s = o.stf_samples(tex, uv, tiles_all, slot, o.BICUBIC, 0, 0)
        want = o.tiles_to_image(np.stack([s["sx"], s["sy"]], -1), tiles_all, 1920, 1080)
        assert np.array_equal(sel[slot], want), f"slot {slot} selection"
    ref = o.stf_filter_reuse(texs, uv, o.BICUBIC, 0, 0, "tile8x8", tiles=tiles_all)
    for slot, tex in enumerate(texs):
        want = o.tiles_to_image(ref[slot][0], tiles_all, 1920, 1080)
        assert_close(host(outs[slot]), want, support_scale(tex, uv, o.BICUBIC), f"plane slot {slot}")


def test_plane_reference_and_stf(plane):
    texs, uv = plane
    dt = [dev(t) for t in texs]
    duv = dev(uv)
    ref_g = [host(x) for x in stf.filter_reference(dt, duv, "bicubic")]
    stf_g = [host(x) for x in stf.filter(dt, duv, "bicubic", 0, 0)]
    rng = np.random.default_rng(1)
    tiles_all = o.all_tiles(1920, 1080)
    tiles = tiles_all[rng.choice(len(tiles_all), 300, replace=False)]
    px = tiles[:, 0:1] * 8 + (np.arange(64) % 8)[None]
    py = tiles[:, 1:2] * 8 + (np.arange(64) // 8)[None]
    mu = o.reference_filter(texs, uv, o.BICUBIC, tiles=tiles)
    st = o.stf_filter(texs, uv, o.BICUBIC, 0, 0, tiles=tiles)
    for slot, tex in enumerate(texs):
        sc = support_scale(tex, uv, o.BICUBIC)[py, px]
        assert_close(ref_g[slot][py, px], mu[slot], sc, "reference")
        assert np.array_equal(stf_g[slot][py, px], st[slot][0].astype(np.float32)), "stf texels exact"


# --------------------------------------------------------------- properties

def test_constant_texture_exact_on_gpu():
    tex = np.full((64, 64, 4), 0.375, np.float16)
    uv = w.small_screen(64, 64, 64, 3.0, offset_seed=0)
    for fp in ALL_FP:
        out = host(stf.filter_reuse([dev(tex)], dev(uv), fp, "bicubic", 3)[0])
        assert np.all(out == np.float32(0.375)), fp


@pytest.mark.parametrize("filt", ["bilinear", "bicubic"])
def test_float_bin_sums_path(filt):
    """STF_FLOAT_BIN_SUMS: the whole-tile kernel's FP32-atomic sums of 1/p
    (the path a wave takes only when it holds a pick of probability below
    2^-34) on two textures of a ragged screen: selection bit-exact, colours
    to the oracle's tolerance, and within that of the exact integer sums."""
    texs = [w.tile_texture_rgba8(3, 64), w.small_texture(5)[:64, :64].copy()]
    uv = w.small_screen(61, 37, 64, 3.3, offset_seed=4)
    ftag = FILTERS[filt]
    dt, duv = [dev(t) for t in texs], dev(uv)
    outs, sel = stf.filter_reuse(dt, duv, "tile8x8", filt, 7, 3, sel=True, float_bin_sums=True)
    exact = stf.filter_reuse(dt, duv, "tile8x8", filt, 7, 3)
    ref = o.stf_filter_reuse(texs, uv, ftag, 7, 3, "tile8x8")
    sel = host(sel)
    for slot, (tex, (rv, rs)) in enumerate(zip(texs, ref)):
        assert np.array_equal(sel[slot], oracle_image(rs, uv)), f"slot {slot}: selection differs"
        scale = support_scale(tex, uv, ftag)
        assert_close(host(outs[slot]), oracle_image(rv, uv), scale, f"slot {slot} float sums")
        assert_close(host(outs[slot]), host(exact[slot]).astype(np.float64), scale, f"slot {slot} vs integer sums")


def test_flat_waves_exact_and_mixed_waves_close():
    """RGBA16F 64^2 whose columns < 32 hold one constant texel value and the
    rest seeded noise, 128x64 screen at 2x, whole-tile reuse: every tile
    whose 64 supports lie in the constant columns returns that value bit for
    bit (the wave shares one texel), the image matches the oracle."""
    rng = np.random.Generator(np.random.PCG64(11))
    tex = rng.random((64, 64, 4)).astype(np.float16)
    tex[:, :32] = np.float16(0.3)
    uv = w.small_screen(128, 64, 64, 2.0, offset_seed=3)
    outs, _ = run_case([tex], uv, "bicubic", "tile8x8", seed=5)
    out = host(outs[0])
    i0x, _ = o.split_coord(o.texel_float_coord(uv[..., 0], 64))
    cols = (i0x[..., None] - 1 + np.arange(4)) % 64              # bicubic support columns
    inside = np.all(cols < 32, axis=-1).reshape(8, 8, 16, 8)      # [tile row, y, tile col, x]
    flat_tiles = inside.all(axis=(1, 3))
    assert flat_tiles.any() and not flat_tiles.all()
    want = np.float32(np.float16(0.3))
    blocks = out.reshape(8, 8, 16, 8, 4)
    for ty, tx in zip(*np.nonzero(flat_tiles)):
        assert np.all(blocks[ty, :, tx] == want), (ty, tx)


def lone_pixels(sel, uv, tex_size):
    """Pixels of full 8x8 tiles whose bilinear support (its texels of positive
    weight) holds no pick of another pixel of the same tile."""
    H, W = uv.shape[:2]
    i0x, Fx = o.split_coord(o.texel_float_coord(uv[..., 0], tex_size))
    i0y, Fy = o.split_coord(o.texel_float_coord(uv[..., 1], tex_size))
    tiles = lambda a: a.reshape(H // 8, 8, W // 8, 8, *a.shape[2:]).swapaxes(1, 2).reshape(H // 8, W // 8, 64, *a.shape[2:])
    sx, sy = tiles(sel[..., 0]), tiles(sel[..., 1])
    bx, by, fx, fy = tiles(i0x), tiles(i0y), tiles(Fx), tiles(Fy)
    dx = (sx[..., None, :] - bx[..., :, None]) % tex_size          # [ty, tx, c, i]
    dy = (sy[..., None, :] - by[..., :, None]) % tex_size
    inside = ((dx == 0) | ((dx == 1) & (fx[..., :, None] > 0))) & ((dy == 0) | ((dy == 1) & (fy[..., :, None] > 0)))
    inside &= ~np.eye(64, dtype=bool)
    lone = ~inside.any(-1)                                           # [ty, tx, c]
    return lone.reshape(H // 8, W // 8, 8, 8).swapaxes(1, 2).reshape(H, W)


def test_whole_tile_lone_picks_equal_stf_bit_exact():
    """Whole-tile bins at 1.6x, bilinear (low enough for lone picks, high
    enough that every tile's supports fit the 12x12 bin window): a pixel
    whose support holds no other pick of its tile returns its one-tap value
    bit for bit, the exact fallback of Eq. (14)."""
    tex = w.tile_texture_rgba8(7, 256)
    uv = w.small_screen(1024, 512, 256, 1.6, offset_seed=9)
    i0x, _ = o.split_coord(o.texel_float_coord(uv[..., 0], 256))
    starts = i0x.reshape(64, 8, 128, 8).swapaxes(1, 2).reshape(64, 128, 64)
    assert np.all(starts.max(-1) - starts.min(-1) <= 5)               # the window fits every tile
    reuse, sel = stf.filter_reuse([dev(tex)], dev(uv), "tile8x8", "bilinear", 2, 0, sel=True)
    one = stf.filter([dev(tex)], dev(uv), "bilinear", 2, 0)
    lone = lone_pixels(host(sel)[0], uv, 256)
    assert lone.sum() > 100
    assert np.array_equal(host(reuse[0])[lone], host(one[0])[lone])


def test_self_and_disjoint_equal_stf_bit_exact():
    tex = w.tile_texture_rgba8(2, 256)
    uv_far = w.small_screen(64, 64, 256, 1 / 8)        # supports never overlap
    uv_mag = w.small_screen(64, 64, 256, 6.0, offset_seed=5)
    a = host(stf.filter([dev(tex)], dev(uv_mag), "bicubic", 4)[0])
    b = host(stf.filter_reuse([dev(tex)], dev(uv_mag), "self", "bicubic", 4)[0])
    assert np.array_equal(a, b)
    a = host(stf.filter([dev(tex)], dev(uv_far), "bicubic", 4)[0])
    for fp in ALL_FP:
        b = host(stf.filter_reuse([dev(tex)], dev(uv_far), fp, "bicubic", 4)[0])
        assert np.array_equal(a, b), fp


def test_convex_hull_on_gpu():
    tex = w.tile_texture_rgba8(6, 64)
    uv = w.small_screen(128, 64, 64, 4.0, offset_seed=6)
    T = o.decode_texels(tex)
    i0x, _ = o.split_coord(o.texel_float_coord(uv[..., 0], 64))
    i0y, _ = o.split_coord(o.texel_float_coord(uv[..., 1], 64))
    vals = np.stack([T[(i0y - 1 + b) % 64, (i0x - 1 + a) % 64] for a in range(4) for b in range(4)], 0)
    lo, hi = vals.min(0), vals.max(0)
    for fp in ALL_FP:
        out = host(stf.filter_reuse([dev(tex)], dev(uv), fp, "bicubic", 8)[0]).astype(np.float64)
        slack = 4 * np.finfo(np.float32).eps
        assert np.all(out >= lo - slack) and np.all(out <= hi + slack), fp


def test_side_stream_launches_match_current_stream():
    """The entry points enqueue on the stream they are given (the current
    torch stream by default): results computed on a side stream of default
    priority equal those of the current stream, bit for bit."""
    tex = dev(w.tile_texture_rgba8(2, 64))
    uv = dev(w.small_screen(64, 48, 64, 3.0, offset_seed=1))
    calls = {
        "reuse": lambda **k: stf.filter_reuse([tex], uv, "tile8x8", "bicubic", 3, **k)[0],
        "quad": lambda **k: stf.filter_reuse([tex], uv, "quad2x2", "bilinear", 3, **k)[0],
        "stf": lambda **k: stf.filter([tex], uv, "bicubic", 3, **k)[0],
        "reference": lambda **k: stf.filter_reference([tex], uv, "bicubic", **k)[0],
    }
    want = {name: host(fn()) for name, fn in calls.items()}
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):                   # current stream = side
        got = {name: fn() for name, fn in calls.items()}
    side.synchronize()
    explicit = {name: fn(stream=side) for name, fn in calls.items()}
    side.synchronize()
    for name in calls:
        assert np.array_equal(host(got[name]), want[name]), name
        assert np.array_equal(host(explicit[name]), want[name]), name


def test_graph_capture_replays_match_eager():
    """A whole-tile reuse launch and a one-tap launch of two textures captured
    in one HIP graph (torch.cuda.CUDAGraph): each replay, after new UVs are
    written in place and eager launches run in between, equals the eager
    result bit for bit (the launches allocate nothing and clear nothing)."""
    texs = [dev(w.tile_texture_rgba8(2, 64)), dev(w.small_texture(5)[:64, :64].copy())]
    uv = dev(w.small_screen(64, 48, 64, 3.0, offset_seed=1))
    outs = [torch.empty((48, 64, 4), device="cuda") for _ in texs]
    one = [torch.empty((48, 64, 4), device="cuda") for _ in texs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                   # warm-up outside the capture
        stf.filter_reuse(texs, uv, "tile8x8", "bicubic", 7, out=outs)
        stf.filter(texs, uv, "bicubic", 7, out=one)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        stf.filter_reuse(texs, uv, "tile8x8", "bicubic", 7, out=outs)
        stf.filter(texs, uv, "bicubic", 7, out=one)
    for k in range(3):
        uv.copy_(dev(w.small_screen(64, 48, 64, 3.0 + k, offset_seed=10 + k)))
        want_r = [host(x) for x in stf.filter_reuse(texs, uv, "tile8x8", "bicubic", 7)]
        want_s = [host(x) for x in stf.filter(texs, uv, "bicubic", 7)]
        graph.replay()
        torch.cuda.synchronize()
        for got, want in zip(outs + one, want_r + want_s):
            assert np.array_equal(host(got), want), k


def test_deterministic_bits(plane):
    texs, uv = plane
    dt = [dev(t) for t in texs]
    duv = dev(uv)
    a = [host(x) for x in stf.filter_reuse(dt, duv, "tile8x8", "bicubic", 9)]
    b = [host(x) for x in stf.filter_reuse(dt, duv, "tile8x8", "bicubic", 9)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_reuse_psnr_gain_on_plane(plane):
    """Whole-tile reuse improves PSNR over one-tap STF by >= 10 dB on the
    1080p bicubic plane (the quality half of the headline metric)."""
    texs, uv = plane
    dt = [dev(texs[0])]
    duv = dev(uv)
    ref = host(stf.filter_reference(dt, duv, "bicubic")[0])
    s = host(stf.filter(dt, duv, "bicubic", 0)[0])
    r = host(stf.filter_reuse(dt, duv, "tile8x8", "bicubic", 0)[0])
    gain = o.psnr(r[..., :3], ref[..., :3]) - o.psnr(s[..., :3], ref[..., :3])
    assert gain >= 10.0, gain


# --------------------------------------------------------------- maximum sizes

def test_maximum_texture_extents_and_seams():
    """Textures at the largest extent per axis (32768 texels), sampled across
    the wrap seam, whole-tile reuse and quads."""
    rng = np.random.default_rng(21)
    wide = rng.integers(0, 256, (4, 32768, 4), dtype=np.uint8)
    tall = rng.integers(0, 256, (32768, 16, 1), dtype=np.uint8)     # rows of 16 bytes (pitch rule)
    py, px = np.mgrid[0:24, 0:72].astype(np.float64)
    uv = np.empty((24, 72, 2), np.float32)
    uv[..., 0] = 1.0 + (px - 36) * 0.3 / 32768        # u crosses 1.0: texel 32767 next to texel 0
    uv[..., 1] = (py + 0.5) / 24 * 0.9 + 0.05
    run_case([wide], uv, "bicubic", "tile8x8", seed=2)
    run_case([wide], uv, "bilinear", "quad2x2", seed=3)
    uvt = uv[..., ::-1].copy()
    run_case([tall], uvt, "bicubic", "tile8x8", seed=4)


@pytest.mark.parametrize("shape", [(8, 32768), (32768, 8)])
def test_maximum_screen_extents(shape):
    """Screens at the largest extent per axis (32768 pixels)."""
    H, W = shape
    tex = w.small_texture(5, 64)
    py, px = np.mgrid[0:H, 0:W].astype(np.float64)
    uv = np.empty((H, W, 2), np.float32)
    uv[..., 0] = ((px + 0.5) / 6.0 / 64) % 1.0
    uv[..., 1] = ((py + 0.5) / 6.0 / 64) % 1.0
    run_case([tex], uv, "bilinear", "tile8x8", seed=9)
    run_case([tex], uv, "bicubic", None, seed=10)          # one-tap: 256 row runs of 128 pixels
