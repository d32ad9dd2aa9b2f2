"""Latent textures decoded by the MLP on the matrix cores, against the FP64
oracle (decode every texel in FP64, then filter), through the C ABI.

Selection is bit-exact (it does not depend on the decode). Colours: the
GPU rounds the latents (when a scale or the FP16 format makes them inexact)
and the hidden activations to BF16 and accumulates in FP32; the tests bound
the resulting decode error of every texel by propagating those roundings
through |W| in FP64 (bound_decode), and a filtered colour, a convex
combination of decoded texels, may differ by at most the largest bound
under its filter support plus the usual 1e-5 relative FP32 term."""
import numpy as np
import pytest

import oracle as o
import workloads as w

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu
REL = 1e-5
U_BF16 = 2.0 ** -8          # unit roundoff of BF16 (8 significant bits)
U_F32 = 2.0 ** -24


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gamma(n):
    return n * U_F32 / (1 - n * U_F32)


def bound_decode(x, layers, u_in):
    """Per texel and output channel: bound on |GPU decode - FP64 decode| for
    FP64 inputs x [..., 8], with inputs rounded with relative error u_in,
    activations rounded to BF16 and FP32 sums of K terms (error gamma(K))."""
    a = np.asarray(x, dtype=np.float64)
    e = u_in * np.abs(a)                                   # input rounding
    for li, (wt, b) in enumerate(layers):
        W = np.asarray(wt, dtype=np.float64)
        bb = np.asarray(b, dtype=np.float64)
        z = a @ W.T + bb
        aw = np.abs(W)
        mag = (np.abs(a) + e) @ aw.T + np.abs(bb)
        ez = e @ aw.T + gamma(W.shape[1] + 1) * mag        # propagated + accumulation
        if li < len(layers) - 1:
            h = np.maximum(z, 0.0)
            e = ez + U_BF16 * (h + ez)                     # ReLU is 1-Lipschitz; BF16 rounding
            a = h
        else:
            return ez


def support_max(values, uv, filt):
    V = np.abs(values)
    th, tw = values.shape[:2]
    n, d = (4, 1) if filt == o.BICUBIC else (2, 0)
    i0x, _ = o.split_coord(o.texel_float_coord(uv[..., 0], tw))
    i0y, _ = o.split_coord(o.texel_float_coord(uv[..., 1], th))
    m = np.zeros(uv.shape[:2] + (values.shape[2],))
    for b in range(n):
        for a in range(n):
            m = np.maximum(m, V[(i0y - d + b) % th, (i0x - d + a) % tw])
    return m


def image(vals, uv):
    return o.tiles_to_image(vals, o.all_tiles(uv.shape[1], uv.shape[0]), uv.shape[1], uv.shape[0])


def device_latents(stored, kind):
    t = torch.from_numpy(np.ascontiguousarray(stored)).cuda()
    if kind == "bf16":
        return t.view(torch.int16).view(torch.bfloat16)
    if kind == "fp8":
        return t.view(torch.float8_e4m3fn)
    return t                                               # float16


def latent_case(kind, seed, size):
    lat = w.latent_grid(seed, size).astype(np.float64)
    scale = w.amax_scale(lat, kind) if kind == "fp8" else None
    stored = w.quantize(lat, kind, scale)
    oracle_kind = {"f16": "f16", "bf16": "bf16", "fp8": "fp8"}[kind]
    x = o.dequantize(stored, oracle_kind, scale)           # FP64 latents the oracle decodes
    exact_in = kind == "bf16" and scale is None
    u_in = 0.0 if exact_in else U_BF16 + U_F32
    return stored, scale, x, u_in


def decoder_on_gpu(layers):
    return stf.pack_decoder([(torch.from_numpy(np.ascontiguousarray(wt)).cuda(),
                              torch.from_numpy(np.ascontiguousarray(b)).cuda()) for wt, b in layers])


def check(gpu, ref, uv, filt, decoded, ebound, what):
    tol = support_max(ebound, uv, filt) * (1 + 1e-6) + REL * np.maximum(np.abs(ref), support_max(decoded, uv, filt))
    err = np.abs(gpu.astype(np.float64) - ref)
    bad = err > tol
    assert not bad.any(), f"{what}: {bad.sum()} beyond bound, worst {np.max(err / tol):.3g}x"
    return float(err.max()), float(np.max(err / tol))


@pytest.mark.parametrize("kind", ["bf16", "f16", "fp8"])
@pytest.mark.parametrize("filt", ["bilinear", "bicubic"])
@pytest.mark.parametrize("fp", [None, "self", "quad2x2", "square3x3", "tile8x8"])
def test_decoded_parity(kind, filt, fp):
    layers = w.decoder_weights(1)
    stored, scale, x, u_in = latent_case(kind, 2, 64)
    decoded = o.mlp_decode(x, layers)
    ebound = bound_decode(x, layers, u_in)
    uv = w.small_screen(136, 72, 64, 4.0, offset_seed=5)          # ragged: 17 x 9 tiles
    ftag = {"bilinear": o.BILINEAR, "bicubic": o.BICUBIC}[filt]
    dec = decoder_on_gpu(layers)
    dt = [device_latents(stored, kind)]
    duv = torch.from_numpy(uv).cuda()
    sc = [None if scale is None else list(scale)]
    if fp is None:
        outs, sel = stf.filter(dt, duv, filt, 3, 1, sel=True, scales=sc, decoder=dec)
        ref = o.stf_filter([decoded], uv, ftag, 3, 1)
    else:
        outs, sel = stf.filter_reuse(dt, duv, fp, filt, 3, 1, sel=True, scales=sc, decoder=dec)
        ref = o.stf_filter_reuse([decoded], uv, ftag, 3, 1, fp)
    rv, rs = ref[0]
    assert np.array_equal(host(sel)[0], image(rs, uv)), "selection differs"
    got = host(outs[0])
    assert got.shape == (72, 136, 4)
    check(got, image(rv, uv), uv, ftag, decoded, ebound, f"{kind} {filt} {fp}")


@pytest.mark.parametrize("fp", [None, "quad2x2", "square3x3", "tile8x8"])
@pytest.mark.parametrize("nt", [2, 3, 4])
def test_decoded_parity_several_latent_textures(fp, nt):
    """Several latent textures in one call (one decoder): the exchanging
    kernels run their slots one after another. Textures of different sizes
    and storage kinds; every slot against the oracle."""
    layers = w.decoder_weights(2)
    cases = [("bf16", 4, 64), ("fp8", 5, 32), ("f16", 6, 64), ("fp8", 7, 16)][:nt]
    stored, scales, decoded, bounds = [], [], [], []
    for kind, seed, size in cases:
        st, sc, x, u_in = latent_case(kind, seed, size)
        stored.append(device_latents(st, kind))
        scales.append(None if sc is None else list(sc))
        decoded.append(o.mlp_decode(x, layers))
        bounds.append(bound_decode(x, layers, u_in))
    uv = w.small_screen(72, 40, 64, 3.0, offset_seed=9)            # ragged: 9 x 5 tiles
    dec = decoder_on_gpu(layers)
    duv = torch.from_numpy(uv).cuda()
    if fp is None:
        outs, sel = stf.filter(stored, duv, "bicubic", 5, 2, sel=True, scales=scales, decoder=dec)
        ref = o.stf_filter(decoded, uv, o.BICUBIC, 5, 2)
    else:
        outs, sel = stf.filter_reuse(stored, duv, fp, "bicubic", 5, 2, sel=True, scales=scales, decoder=dec)
        ref = o.stf_filter_reuse(decoded, uv, o.BICUBIC, 5, 2, fp)
    sel = host(sel)
    for i in range(nt):
        rv, rs = ref[i]
        assert np.array_equal(sel[i], image(rs, uv)), f"slot {i} selection differs"
        check(host(outs[i]), image(rv, uv), uv, o.BICUBIC, decoded[i], bounds[i], f"slot {i} of {nt}, {fp}")


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_decoded_reference_parity(kind):
    # Eq. (3) over decoded texels: every tap of every pixel is decoded
    layers = w.decoder_weights(4)
    stored, scale, x, u_in = latent_case(kind, 6, 64)
    decoded = o.mlp_decode(x, layers)
    uv = w.small_screen(72, 40, 64, 3.0, offset_seed=2)
    out = stf.filter_reference([device_latents(stored, kind)], torch.from_numpy(uv).cuda(), "bicubic",
                               scales=[None if scale is None else list(scale)], decoder=decoder_on_gpu(layers))[0]
    ref = o.reference_filter([decoded], uv, o.BICUBIC)[0]
    check(host(out), image(ref, uv), uv, o.BICUBIC, decoded, bound_decode(x, layers, u_in), kind)


def test_decoder_texel_centres_are_plain_decodes():
    # at texel centres the bilinear one-tap pick is the texel itself, so the
    # output is the decode of that texel alone; BF16 latents are exact
    # inputs, so only the activation roundings remain
    layers = w.decoder_weights(7)
    stored, scale, x, u_in = latent_case("bf16", 8, 32)
    c = ((np.arange(32) + 0.5) / 32).astype(np.float32)
    uv = np.stack(np.broadcast_arrays(c[None, :], c[:, None]), -1).astype(np.float32)
    out = host(stf.filter([device_latents(stored, "bf16")], torch.from_numpy(uv).cuda(), "bilinear",
                          decoder=decoder_on_gpu(layers))[0])
    want = o.mlp_decode(x, layers)
    bound = bound_decode(x, layers, u_in)
    err = np.abs(out - want)
    assert np.all(err <= bound * (1 + 1e-6) + 1e-30)
    # the worst-case bound is loose; the typical error is a few BF16 ulps of
    # the activations (a misplaced weight or lane would be of order |y|)
    assert err.max() < 0.02 * np.abs(want).max()
    assert err.mean() < 1e-2 * np.abs(want).mean()


def test_decoder_zero_weights_give_bias():
    # W = 0: every texel decodes to b3 exactly (b3 is kept in FP32)
    layers = [(np.zeros((64, 8), np.float32), np.zeros(64, np.float32)),
              (np.zeros((64, 64), np.float32), np.zeros(64, np.float32)),
              (np.zeros((4, 64), np.float32), np.array([0.1, -2.5, 3.0e-3, 7.0], np.float32))]
    stored, _, _, _ = latent_case("fp8", 9, 32)
    uv = w.small_screen(40, 24, 32, 2.0)
    out = host(stf.filter_reuse([device_latents(stored, "fp8")], torch.from_numpy(uv).cuda(), "tile8x8",
                                "bicubic", decoder=decoder_on_gpu(layers))[0])
    assert np.array_equal(out, np.broadcast_to(layers[2][1], out.shape))


def test_decoded_full_size_sampled():
    """1024^2 x 8 FP8 latents with per-channel scales, 1920x1080 perspective
    plane at 4x-16x, bicubic whole-tile reuse: full selection bit-exact and
    colours of 600 sampled tiles within the bound."""
    layers = w.decoder_weights(0)
    stored, scale, x, u_in = latent_case("fp8", 0, 1024)
    uv, _, _, _ = w.perspective_plane(1920, 1080, 1024, 4.0, 16.0)
    dec = decoder_on_gpu(layers)
    outs, sel = stf.filter_reuse([device_latents(stored, "fp8")], torch.from_numpy(uv).cuda(), "tile8x8",
                                 "bicubic", 11, 0, sel=True, scales=[list(scale)], decoder=dec)
    tiles_all = o.all_tiles(1920, 1080)
    pick = np.random.default_rng(0).choice(len(tiles_all), 600, replace=False)
    tiles = tiles_all[pick]
    decoded = o.mlp_decode(x, layers)
    rv, rs = o.stf_filter_reuse([decoded], uv, o.BICUBIC, 11, 0, "tile8x8", tiles=tiles)[0]
    px = tiles[:, 0:1] * 8 + (np.arange(64) % 8)[None]
    py = tiles[:, 1:2] * 8 + (np.arange(64) // 8)[None]
    ok = (px < 1920) & (py < 1080)
    s = host(sel)[0]
    got = host(outs[0])
    assert np.array_equal(s[py[ok], px[ok]], rs[ok])
    ebound = bound_decode(x, layers, u_in)
    uvs = uv[py[ok], px[ok]][:, None, :]
    tol = support_max(ebound, uvs, o.BICUBIC)[:, 0] * (1 + 1e-6) + \
        REL * np.maximum(np.abs(rv[ok]), support_max(decoded, uvs, o.BICUBIC)[:, 0])
    err = np.abs(got[py[ok], px[ok]].astype(np.float64) - rv[ok])
    assert np.all(err <= tol), f"worst {np.max(err / tol):.3g}x of the bound"


# ----------------------------------------------------------------- FP8 decoder

U_FP8 = 2.0 ** -4           # unit roundoff of FP8 E4M3 (4 significant bits)
SUB_FP8 = 2.0 ** -10        # half the subnormal spacing of FP8 E4M3


def bound_decode_fp8(x, layers, exact_inputs):
    """Bound on |GPU FP8 decode - FP64 decode|: inputs and activations
    rounded to FP8 E4M3 (relative 2^-4, absolute 2^-10 below the normal
    range), weights stored as FP8 of W / s with s = max|W| / 448, FP32
    accumulation."""
    a = np.asarray(x, dtype=np.float64)
    e = np.zeros_like(a) if exact_inputs else np.maximum(U_FP8 * np.abs(a), SUB_FP8)
    for li, (wt, b) in enumerate(layers):
        W = np.asarray(wt, dtype=np.float64)
        bb = np.asarray(b, dtype=np.float64)
        s = np.abs(W).max() / 448.0
        dW = np.maximum(U_FP8 * np.abs(W), s * SUB_FP8)
        z = a @ W.T + bb
        aw = np.abs(W)
        ez = e @ aw.T + (np.abs(a) + e) @ dW.T
        ez = ez + gamma(W.shape[1] + 1) * ((np.abs(a) + e) @ (aw + dW).T + np.abs(bb)) + U_F32 * (np.abs(z) + ez)
        if li < len(layers) - 1:
            h = np.maximum(z, 0.0)
            e = ez + np.maximum(U_FP8 * (h + ez), SUB_FP8)
            a = h
        else:
            return ez


@pytest.mark.parametrize("kind", ["fp8", "bf16"])
@pytest.mark.parametrize("fp", [None, "quad2x2", "tile8x8"])
def test_fp8_decoder_parity(kind, fp):
    layers = w.decoder_weights(2)
    stored, scale, x, _ = latent_case(kind, 3, 64)
    decoded = o.mlp_decode(x, layers)
    ebound = bound_decode_fp8(x, layers, exact_inputs=(kind == "fp8" and scale is None))
    uv = w.small_screen(104, 56, 64, 4.0, offset_seed=6)
    dec = stf.pack_decoder([(torch.from_numpy(np.ascontiguousarray(a)).cuda(),
                             torch.from_numpy(np.ascontiguousarray(b)).cuda()) for a, b in layers], precision="fp8")
    dt, duv = [device_latents(stored, kind)], torch.from_numpy(uv).cuda()
    sc = [None if scale is None else list(scale)]
    if fp is None:
        outs, sel = stf.filter(dt, duv, "bicubic", 1, 0, sel=True, scales=sc, decoder=dec)
        (rv, rs), = o.stf_filter([decoded], uv, o.BICUBIC, 1, 0)
    else:
        outs, sel = stf.filter_reuse(dt, duv, fp, "bicubic", 1, 0, sel=True, scales=sc, decoder=dec)
        (rv, rs), = o.stf_filter_reuse([decoded], uv, o.BICUBIC, 1, 0, fp)
    assert np.array_equal(host(sel)[0], image(rs, uv))
    got = host(outs[0])
    check(got, image(rv, uv), uv, o.BICUBIC, decoded, ebound, f"fp8 decoder {kind} {fp}")
    # FP8 arithmetic is coarse but not vacuous: the typical error is a few
    # percent of the output range
    err = np.abs(got - image(rv, uv))
    assert err.mean() < 0.05 * np.abs(decoded).max()


def test_fp8_decoder_at_texel_centres_matches_a_simulated_fp8_decode():
    # at texel centres one-tap STF returns the decode of the texel itself;
    # compare with an FP64 simulation of the FP8 arithmetic (weights,
    # latents and activations rounded to OCP E4M3 by torch's CPU cast)
    layers = w.decoder_weights(5)
    lat = w.latent_grid(9, 32).astype(np.float64)
    codes = w.quantize(lat, "fp8")
    c = ((np.arange(32) + 0.5) / 32).astype(np.float32)
    uv = np.stack(np.broadcast_arrays(c[None, :], c[:, None]), -1).astype(np.float32)
    dec = stf.pack_decoder([(torch.from_numpy(np.ascontiguousarray(a)).cuda(),
                             torch.from_numpy(np.ascontiguousarray(b)).cuda()) for a, b in layers], precision="fp8")
    got = host(stf.filter([device_latents(codes, "fp8")], torch.from_numpy(uv).cuda(), "bilinear", decoder=dec)[0])

    def q8(v):
        return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(torch.float8_e4m3fn).to(
            torch.float64).numpy()

    a = o.fp8e4m3_value(codes)
    for li, (wt, b) in enumerate(layers):
        W = wt.astype(np.float64)
        s = np.float32(np.abs(wt).max()) / np.float32(448.0)
        Wq = q8(W / s)
        z = s * (a @ Wq.T + b.astype(np.float64) / s)
        a = q8(np.maximum(z, 0.0)) if li < 2 else z
    # only the FP32 accumulation order and scale products differ, which can
    # move an activation across an FP8 rounding boundary now and then: nearly
    # every output agrees to 1e-3 of the range
    err = np.abs(got - a)
    assert np.mean(err <= 1e-3 * np.abs(a).max()) >= 0.99
