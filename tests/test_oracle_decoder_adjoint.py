"""Pins of the oracle's adjoint through the latent decoder (the neural-texture
setting, Sec. 1 and Sec. 5.6, differentiated through Eq. (14)): central
differences of the whole FP64 forward pass (Eq. (14) over decoded latents)
with respect to latents and every decoder weight and bias; the closed form of
the output bias gradient (the weights of Eq. (14) are normalised); and the
affine regime, where the decoder is one matrix."""
import numpy as np
import pytest

import oracle as o
import workloads as w

FILT = o.BICUBIC


def _screen(width=24, height=16, size=16, mag=3.0, seed=1):
    return w.small_screen(width, height, size, mag, offset_seed=seed)


def _problem(seed=0, size=16):
    rng = np.random.default_rng(seed)
    lat = rng.standard_normal((size, size, 8))
    scale = rng.uniform(0.5, 2.0, 8)
    layers = [(np.asarray(a, np.float64), np.asarray(b, np.float64)) for a, b in w.mlp_weights(seed)]
    uv = _screen(size=size, seed=seed + 1)
    tiles = o.all_tiles(uv.shape[1], uv.shape[0])
    G = rng.standard_normal((len(tiles), 64, 4))
    return lat, scale, layers, uv, G


def _loss(lat, scale, layers, uv, G, footprint):
    out = o.stf_filter_reuse([(lat, "f32", scale, layers)], uv, FILT, 5, 2, footprint)[0][0]
    return float(np.sum(out * G))


def _pattern(lat, scale, layers):
    """Signs of every pre-activation of every texel (the ReLU pattern)."""
    h = o.dequantize(lat, "f32", scale).reshape(-1, 8)
    sig = []
    for li, (wt, b) in enumerate(layers[:-1]):
        z = h @ wt.T + b
        sig.append(z > 0)
        h = np.maximum(z, 0.0)
    return np.concatenate(sig, axis=1)


@pytest.mark.parametrize("footprint", ["tile8x8", "square3x3"])
def test_central_differences(footprint):
    lat, scale, layers, uv, G = _problem(3)
    tex = (lat, "f32", scale, layers)
    (dlat,), lg = o.stf_adjoint_decoder([tex], uv, FILT, 5, 2, footprint, [G])
    rng = np.random.default_rng(7)
    base_pattern = _pattern(lat, scale, layers)
    checked = 0

    def fd(perturb):
        # central difference; the loss is affine in each single parameter
        # while no ReLU input changes sign, so it is exact up to rounding
        h = 1e-6
        (l1, s1, y1), (l2, s2, y2) = perturb(h), perturb(-h)
        if not (np.array_equal(_pattern(l1, s1, y1), base_pattern) and
                np.array_equal(_pattern(l2, s2, y2), base_pattern)):
            return None
        return (_loss(l1, s1, y1, uv, G, footprint) - _loss(l2, s2, y2, uv, G, footprint)) / (2 * h)

    # latents, at texels the screen touches (dlat != 0) and one it does not
    hit = np.argwhere(np.any(dlat != 0, axis=-1))
    assert len(hit) > 10
    for k in list(rng.choice(len(hit), 6, replace=False)):
        y, x = hit[k]
        c = int(rng.integers(8))

        def pert(h, y=y, x=x, c=c):
            l2 = lat.copy()
            l2[y, x, c] += h
            return l2, scale, layers
        v = fd(pert)
        if v is not None:
            assert np.isclose(v, dlat[y, x, c], rtol=1e-6, atol=1e-8), ("latent", y, x, c, v, dlat[y, x, c])
            checked += 1
    # every weight and bias of the decoder
    for li in range(3):
        for which in (0, 1):
            arr = layers[li][which]
            for _ in range(3):
                idx = tuple(int(rng.integers(n)) for n in arr.shape)

                def pert(h, li=li, which=which, idx=idx):
                    ly = [(a.copy(), b.copy()) for a, b in layers]
                    ly[li][which][idx] += h
                    return lat, scale, ly
                v = fd(pert)
                if v is not None:
                    want = lg[li][which][idx]
                    assert np.isclose(v, want, rtol=1e-6, atol=1e-8), (li, which, idx, v, want)
                    checked += 1
    assert checked >= 18


def test_output_bias_gradient_closed_form():
    # Eq. (14) normalises its weights (sum_i a_ci = 1 for every on-screen
    # pixel) and b3 adds to every decoded texel, so dL/db3 = sum_c dL/dout_c
    lat, scale, layers, uv, G = _problem(5)
    tiles = o.all_tiles(uv.shape[1], uv.shape[0])
    px = tiles[:, 0:1] * 8 + (np.arange(64) % 8)[None]
    py = tiles[:, 1:2] * 8 + (np.arange(64) // 8)[None]
    on = (px < uv.shape[1]) & (py < uv.shape[0])
    for fp in ("tile8x8", "quad2x2", "square4x4"):
        _, lg = o.stf_adjoint_decoder([(lat, "f32", scale, layers)], uv, FILT, 1, 0, fp, [G])
        assert np.allclose(lg[2][1], np.sum(G[on], axis=0), rtol=1e-12, atol=1e-12), fp


def test_affine_regime_is_one_matrix():
    # non-negative latents, weights and biases keep every ReLU input
    # positive: the decoder is x -> W3 W2 W1 x + const, so the latent
    # gradient is (W3 W2 W1)^T g_x and dW1 = sum_x (W3 W2)^T g_x x^T
    rng = np.random.default_rng(2)
    lat = rng.uniform(0.0, 1.0, (16, 16, 8))
    layers = [(rng.uniform(0.0, 0.3, (64, 8)), rng.uniform(0.1, 0.2, 64)),
              (rng.uniform(0.0, 0.1, (64, 64)), rng.uniform(0.1, 0.2, 64)),
              (rng.standard_normal((4, 64)) * 0.1, rng.standard_normal(4))]
    uv = _screen(seed=4)
    tiles = o.all_tiles(uv.shape[1], uv.shape[0])
    G = rng.standard_normal((len(tiles), 64, 4))
    tex = (lat, "f32", None, layers)
    (dlat,), lg = o.stf_adjoint_decoder([tex], uv, FILT, 9, 1, "tile8x8", [G])
    g_tex = o.stf_adjoint([tex], uv, FILT, 9, 1, "tile8x8", [G])[0]
    W1, W2, W3 = (a for a, _ in layers)
    M = W3 @ W2 @ W1
    assert np.allclose(dlat, g_tex @ M, rtol=1e-12, atol=1e-13)
    want_dw1 = np.einsum("yxo,yxi->oi", g_tex @ (W3 @ W2), lat)
    assert np.allclose(lg[0][0], want_dw1, rtol=1e-12, atol=1e-12)


def test_scale_and_quantised_storage():
    # the gradient is taken with respect to the stored value: latent = stored
    # * scale, so it carries the scale as a factor; FP16 storage decodes
    # exactly, so it matches FP32 storage of the same values
    lat, scale, layers, uv, G = _problem(8)
    h = lat.astype(np.float16)
    (d16,), g16 = o.stf_adjoint_decoder([(h, "f16", scale, layers)], uv, FILT, 2, 0, "tile8x8", [G])
    (d32,), g32 = o.stf_adjoint_decoder([(h.astype(np.float64), "f32", scale, layers)], uv, FILT, 2, 0,
                                        "tile8x8", [G])
    assert np.array_equal(d16, d32)
    (d1,), _ = o.stf_adjoint_decoder([(h.astype(np.float64) * scale, "f32", None, layers)], uv, FILT, 2, 0,
                                     "tile8x8", [G])
    assert np.allclose(d32, d1 * scale, rtol=1e-12, atol=1e-14)
