"""Adjoint through the latent decoder (stf_backward_decoder) against the FP64
oracle (oracle.stf_adjoint_decoder), through the C ABI, and autograd fitting
of a latent grid plus decoder.

Tolerance, derived from the arithmetic. The texel adjoint g_x reaches the
decoder with the error bound the texel-adjoint tests use, 1e-5 of
G_x = sum_c sum_i a_ci |dL/dout_c| (the adjoint of |dL/dout|; the a_ci are
non-negative). Then every product runs in FP32 with exact products and
sequential FP32 sums of K terms (error gamma(K) of the sum of absolute
terms): K = 4, 64, 64 for d2, d1 and dL/dl, and 16 texels per block, the
blocks of a wave and the waves for the weight gradients. So each output is
compared with REL_CHAIN (plus gamma of the summation depth for the weight
gradients) times its magnitude: the same backward pass run on |W|, G_x and
|activations| with the same ReLU pattern. The ReLU pattern itself is a
decision taken in floating point: at a texel whose pre-activation lies
within its FP32 error bound of zero the GPU may take the other branch, and
either branch gives a valid derivative. Such a texel's latent gradient is not
compared (what is unique is), and its whole contribution, taken with every
unit that may be active, is added to the weight-gradient tolerance."""
import numpy as np
import pytest

import oracle as o
import workloads as w

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu
U = 2.0 ** -24
ETA_G = 1e-5                      # texel adjoint bound (as in the texel-adjoint tests)


def gamma(n):
    return n * U / (1 - n * U)


REL_CHAIN = ETA_G + gamma(4) + 2 * gamma(64) + 4 * U


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def tile_grads(g, W, H):
    tiles = o.all_tiles(W, H)
    px = tiles[:, 0:1] * 8 + (np.arange(64) % 8)[None]
    py = tiles[:, 1:2] * 8 + (np.arange(64) // 8)[None]
    valid = (px < W) & (py < H)
    return np.where(valid[..., None], g[np.minimum(py, H - 1), np.minimum(px, W - 1)], 0.0)


def magnitudes(lat, layers, G):
    """Per texel (rows of lat [n, 8], G [n, 4]): the backward pass on
    absolute values (|W|, G, |activations|) with the texel's ReLU pattern,
    and which texels are ambiguous: a pre-activation within twice its FP32
    error bound of zero, so the GPU may take the other branch there. For
    those the pattern is replaced by every unit that may be active (the
    magnitudes then bound the whole contribution either way)."""
    (W1, b1), (W2, b2), (W3, b3) = [(np.asarray(a, np.float64), np.asarray(b, np.float64)) for a, b in layers]
    z1 = lat @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    e1 = 2 * (gamma(9) * (np.abs(lat) @ np.abs(W1).T + np.abs(b1)) + U * np.abs(lat) @ np.abs(W1).T)
    z2 = h1 @ W2.T + b2
    e2 = 2 * gamma(65) * ((h1 + e1) @ np.abs(W2).T + np.abs(b2)) + e1 @ np.abs(W2).T
    amb = np.any(np.abs(z1) <= e1, axis=1) | np.any(np.abs(z2) <= e2, axis=1)
    on1 = np.where(amb[:, None], z1 > -e1, z1 > 0)
    on2 = np.where(amb[:, None], z2 > -e2, z2 > 0)
    a1 = np.where(on1, np.abs(z1) + e1, 0.0)
    a2 = np.where(on2, np.abs(z2) + e2, 0.0)
    m2 = (G @ np.abs(W3)) * on2
    m1 = (m2 @ np.abs(W2)) * on1
    ml = m1 @ np.abs(W1)
    per_texel = [(m1[:, :, None] * np.abs(lat)[:, None, :], m1), (m2[:, :, None] * a1[:, None, :], m2),
                 (G[:, :, None] * a2[:, None, :], G)]
    return ml, per_texel, amb


CASES = [("bicubic", "tile8x8", "f16", 32), ("bicubic", "quad2x2", "fp8", 32), ("bilinear", "square3x3", "bf16", 32),
         ("bicubic", "self", "f16", 32), ("bilinear", "tile8x8", "fp8", 32),
         ("bicubic", "tile8x8", "f16", 4),        # 16 texels: one block of the decoder adjoint
         ("bicubic", "tile8x8", "bf16", 256)]     # 2048 blocks, a few dozen reached: a sparse block list


@pytest.mark.parametrize("filt,fp,kind,size", CASES)
def test_decoder_adjoint_matches_oracle(filt, fp, kind, size):
    _check_case(filt, fp, kind, size, (72, 40, 3.0))


def test_decoder_adjoint_whole_grid_two_blocks_per_wave():
    # a 256x256 view at 1x covers the 256^2 grid: 4096 blocks of 16 texels for
    # 2048 waves, so every wave runs two blocks and every workgroup sums four
    _check_case("bicubic", "tile8x8", "fp8", 256, (256, 256, 1.0))


def _check_case(filt, fp, kind, size, screen):
    rng = np.random.default_rng(11)
    lat = w.latent_grid(2, max(size, 8))[:size, :size].astype(np.float64)
    scale = w.amax_scale(lat, kind) if kind == "fp8" else rng.uniform(0.5, 2.0, 8).astype(np.float32).astype(np.float64)
    stored = w.quantize(lat, kind, scale)
    layers32 = w.mlp_weights(4)
    layers = [(a.astype(np.float64), b.astype(np.float64)) for a, b in layers32]
    uv = w.small_screen(screen[0], screen[1], size, screen[2], offset_seed=5)
    H, W = uv.shape[:2]
    g = rng.standard_normal((H, W, 4)).astype(np.float32)
    dlayers_t = [(dev(a), dev(b)) for a, b in layers32]
    tex_t = {"f16": lambda s: dev(s), "bf16": lambda s: dev(s.view(np.int16)).view(torch.bfloat16),
             "fp8": lambda s: dev(s).view(torch.float8_e4m3fn)}[kind](stored)
    dec = stf.pack_decoder(dlayers_t)
    ftag = o.BICUBIC if filt == "bicubic" else o.BILINEAR
    # the forward selection does not depend on the decode: check it once
    _, sel = stf.filter_reuse([tex_t], dev(uv), fp, filt, 6, 1, sel=True, scales=[list(scale)], decoder=dec)
    (dlat,), dl = stf.backward_decoder([tex_t], dev(uv), [dev(g)], dlayers_t, dec, fp, filt, 6, 1,
                                       scales=[list(scale)])
    torch.cuda.synchronize()
    tex = (stored, kind, scale, layers)
    G = tile_grads(g, W, H)
    (want_lat,), want = o.stf_adjoint_decoder([tex], uv, ftag, 6, 1, fp, [G])
    s = o.stf_samples(tex, uv, o.all_tiles(W, H), 0, ftag, 6, 1)
    assert np.array_equal(sel[0].cpu().numpy(), o.tiles_to_image(np.stack([s["sx"], s["sy"]], -1),
                                                                 o.all_tiles(W, H), W, H))
    # magnitudes: the texel adjoint of |dL/dout|, then |W| with the same ReLU pattern
    gmag = o.stf_adjoint([tex], uv, ftag, 6, 1, fp, [np.abs(G)])[0]
    latv = o.dequantize(stored, kind, scale)
    hit = np.any(gmag != 0, axis=-1)
    ml, per_texel, amb = magnitudes(latv[hit], layers, gmag[hit])
    assert amb.mean() < 0.05, amb.mean()
    got_lat = dlat.cpu().numpy().astype(np.float64)
    tol_lat = np.zeros(got_lat.shape)
    sc = np.asarray(scale, np.float64)
    tol_lat[hit] = np.where(amb[:, None], np.inf, REL_CHAIN * ml * sc) + 1e-30
    err = np.abs(got_lat - want_lat)
    assert np.all(err <= tol_lat), f"dlatent: worst {np.max(err / np.maximum(tol_lat, 1e-30)):.3g}x the bound"
    # weight gradients: rounding of every term, plus the whole contribution
    # of the ambiguous texels (where either branch is a valid derivative)
    n_terms = int(hit.sum())
    rel_w = REL_CHAIN + gamma(64) + gamma(n_terms) + gamma(stf_waves(size))
    for li in range(3):
        for which in (0, 1):
            terms = per_texel[li][which]
            tol = rel_w * terms.sum(0) + terms[amb].sum(0) + 1e-30
            gg = dl[li][which].cpu().numpy().astype(np.float64)
            e = np.abs(gg - want[li][which])
            assert np.all(e <= tol), f"layer {li} {'bW'[which]}: worst {np.max(e / tol):.3g}x the bound"


def test_zero_gradient_visits_no_block():
    # no block is listed: the latent and weight gradients stay as they were
    layers32 = w.mlp_weights(3)
    dlayers_t = [(dev(a), dev(b)) for a, b in layers32]
    dec = stf.pack_decoder(dlayers_t)
    tex = dev(w.latent_grid(1, 64).astype(np.float16))
    uv = dev(w.small_screen(40, 24, 64, 2.0, offset_seed=2))
    dl = torch.full((64, 64, 8), 0.25, device="cuda")
    dly = [(torch.full_like(a, 0.5), torch.full_like(b, -0.5)) for a, b in dlayers_t]
    stf.backward_decoder([tex], uv, [torch.zeros((24, 40, 4), device="cuda")], dlayers_t, dec, "tile8x8", "bicubic",
                         1, 0, dlatent=[dl], dlayers=dly)
    torch.cuda.synchronize()
    assert bool((dl == 0.25).all())
    assert all(bool((a == 0.5).all()) and bool((b == -0.5).all()) for a, b in dly)


def stf_waves(size):
    return min((size * size + 15) // 16, 2048)         # one block of 16 texels per step


def test_accumulates_and_two_slots():
    # two latent textures of different sizes in one call share the decoder:
    # the weight gradients add up over both; outputs accumulate (+=)
    rng = np.random.default_rng(2)
    layers32 = w.mlp_weights(1)
    dlayers_t = [(dev(a), dev(b)) for a, b in layers32]
    dec = stf.pack_decoder(dlayers_t)
    lats = [w.latent_grid(3, 32).astype(np.float16), w.latent_grid(4, 16).astype(np.float16)]
    uv = dev(w.small_screen(40, 24, 32, 2.5, offset_seed=1))
    g = [dev(rng.standard_normal((24, 40, 4)).astype(np.float32)) for _ in range(2)]
    texs = [dev(l) for l in lats]
    both = stf.backward_decoder(texs, uv, g, dlayers_t, dec, "tile8x8", "bicubic", 2, 0)
    one = [stf.backward_decoder([texs[i]], uv, [g[i]], dlayers_t, dec, "tile8x8", "bicubic", 2, 0) for i in range(2)]
    # the second texture is slot 1 in the joint call: its random numbers differ, so compare sums of
    # independent calls only for slot 0's latents and accumulate-twice semantics
    twice = stf.backward_decoder([texs[0]], uv, [g[0]], dlayers_t, dec, "tile8x8", "bicubic", 2, 0)
    stf.backward_decoder([texs[0]], uv, [g[0]], dlayers_t, dec, "tile8x8", "bicubic", 2, 0,
                         dlatent=twice[0], dlayers=twice[1])
    torch.cuda.synchronize()
    assert torch.allclose(both[0][0], one[0][0][0], rtol=1e-5, atol=1e-7)
    assert torch.allclose(twice[0][0], 2 * one[0][0][0], rtol=1e-5, atol=1e-7)
    for li in range(3):
        for k in range(2):
            assert torch.allclose(twice[1][li][k], 2 * one[0][1][li][k], rtol=1e-5, atol=1e-6)


def test_latent_and_decoder_fitting():
    """Fit an FP32 latent grid (stored FP16 for the forward pass) and the
    decoder MLP (packed to BF16) to the deterministic filter of a target
    colour texture over four seeded views, through stf_decoder_autograd."""
    rng = np.random.default_rng(0)
    target = dev(w.tile_texture_rgba8(5, 32).astype(np.float32) / 255.0)
    views = [dev(w.small_screen(64, 48, 32, 2.5 + k, offset_seed=k)) for k in range(4)]
    refs = [stf.filter_reference([target], uv, "bicubic")[0] for uv in views]
    lat = torch.tensor(rng.standard_normal((32, 32, 8)).astype(np.float32) * 0.5, device="cuda", requires_grad=True)
    params = [torch.tensor(a, device="cuda", requires_grad=True) for layer in w.mlp_weights(7) for a in layer]
    opt = torch.optim.Adam([lat] + params, lr=0.01)
    losses = []
    for it in range(80):
        opt.zero_grad()
        layers = [(params[0], params[1]), (params[2], params[3]), (params[4], params[5])]
        loss = 0.0
        for k, (uv, ref) in enumerate(zip(views, refs)):
            out = stf.stf_decoder_autograd(lat, layers, uv, "tile8x8", "bicubic", seed=it, frame=k)
            loss = loss + ((out - ref) ** 2).mean()
        loss.backward()
        assert all(p.grad is not None and torch.isfinite(p.grad).all() for p in [lat] + params)
        opt.step()
        losses.append(float(loss.detach()))
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])
