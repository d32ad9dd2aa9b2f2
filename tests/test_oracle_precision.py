"""Pins of the oracle's reduced-precision decodes and the latent decoder MLP
(no GPU)."""
import os

import numpy as np

import oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fp8_e4m3_golden_values():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fp8_e4m3_values.txt"))
            if l.strip() and not l.startswith("#")]
    for code, val in rows:
        got = o.fp8e4m3_value(np.array([int(code, 16)]))[0]
        if val == "nan":
            assert np.isnan(got)
        else:
            assert got == float(val) and np.signbit(got) == val.startswith("-")


def test_fp8_e4m3_structure():
    v = o.fp8e4m3_value(np.arange(256))
    pos = v[:128]
    finite = ~np.isnan(pos)
    assert finite.sum() == 127                          # only 0x7F is NaN in the positive half
    assert np.all(np.diff(pos[finite]) > 0)             # strictly increasing codes
    assert np.array_equal(v[128:][finite], -pos[finite])
    # every value is a float16 value (3 mantissa bits, exponents within range)
    assert np.array_equal(pos[finite].astype(np.float16).astype(np.float64), pos[finite])


def test_bf16_values():
    bits = np.array([0x0000, 0x3F80, 0xBF80, 0x4049, 0x7F80, 0x0001])
    got = o.bf16_value(bits)
    assert got[0] == 0.0 and got[1] == 1.0 and got[2] == -1.0 and np.isinf(got[4])
    assert got[3] == np.float32(np.frombuffer(np.uint32(0x40490000).tobytes(), np.float32)[0])
    assert got[5] == 2.0 ** -133                        # smallest bfloat16 subnormal


def test_mlp_decode_closed_form():
    # layer 1 computes (x, -x) for the first 4 inputs (other units 0), layer 2
    # passes the 8 values through, layer 3 outputs ReLU(x) - ReLU(-x) = x:
    # the decoder returns the first four latents exactly
    W1 = np.zeros((64, 8)); W2 = np.zeros((64, 64)); W3 = np.zeros((4, 64))
    for i in range(4):
        W1[i, i] = 1.0
        W1[4 + i, i] = -1.0
    for j in range(8):
        W2[j, j] = 1.0
    for i in range(4):
        W3[i, i] = 1.0
        W3[i, 4 + i] = -1.0
    layers = [(W1, np.zeros(64)), (W2, np.zeros(64)), (W3, np.zeros(4))]
    x = np.random.default_rng(0).standard_normal((100, 8))
    assert np.allclose(o.mlp_decode(x, layers), x[:, :4], atol=0)
    # biases shift the output; ReLU clips negative hidden units
    layers[2] = (W3, np.array([0.5, -1.0, 2.0, 0.0]))
    assert np.allclose(o.mlp_decode(x, layers), x[:, :4] + [0.5, -1.0, 2.0, 0.0])


def test_dequantize_scales_channels():
    codes = np.array([[0x38, 0x40, 0xc0, 0x08]], dtype=np.uint8)
    v = o.dequantize(codes, "fp8", [2.0, 0.5, 1.0, 4.0])
    assert np.array_equal(v, [[2.0, 1.0, -2.0, 0.0625]])


def test_fp8_and_bf16_match_torch_cpu_casts():
    # torch's CPU float8_e4m3fn and bfloat16 types implement the same formats
    import torch
    codes = torch.arange(256, dtype=torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = o.fp8e4m3_value(np.arange(256))
    assert np.array_equal(np.isnan(ref), np.isnan(got))
    ok = ~np.isnan(ref)
    assert np.array_equal(ref[ok], got[ok]) and np.array_equal(np.signbit(ref[ok]), np.signbit(got[ok]))
    bits = torch.randint(0, 1 << 16, (4096,), generator=torch.Generator().manual_seed(3), dtype=torch.int32)
    bits = bits[((bits >> 7) & 0xFF) != 0xFF]           # finite patterns
    ref = bits.to(torch.int16).view(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(o.bf16_value(bits.numpy().astype(np.uint16)), ref)


def test_texture_values_forms():
    rng = np.random.default_rng(5)
    b = rng.integers(0, 256, (8, 8, 4), dtype=np.uint8)
    assert np.array_equal(o.texture_values(b), b / 255.0)
    assert np.array_equal(o.texture_values((b, "unorm8", None)), b / 255.0)
    assert np.array_equal(o.texture_values((b, "unorm8", [1, 2, 4, 8])), b / 255.0 * [1, 2, 4, 8])
    h = rng.standard_normal((8, 8, 2)).astype(np.float16)
    assert np.array_equal(o.texture_values((h.view(np.uint16), "f16", [3, -1])), h.astype(np.float64) * [3, -1])


def _tiny_screen(seed):
    rng = np.random.default_rng(seed)
    return (rng.random((16, 16, 2)) * 0.3 + 0.1).astype(np.float32)


def test_reuse_and_adjoint_scale_linearly():
    # a per-channel scale commutes with every filter: Eq. (3), one-tap STF and
    # Eq. (14) are linear in the texels with weights independent of them
    rng = np.random.default_rng(9)
    h = rng.random((16, 16, 4)).astype(np.float16)
    sc = np.array([0.5, 2.0, -3.0, 1.0])
    uv = _tiny_screen(1)
    for fp in ("self", "quad2x2", "tile8x8"):
        a = o.stf_filter_reuse([h], uv, "bicubic", 7, 2, fp)[0]
        b = o.stf_filter_reuse([(h, "f16", sc)], uv, "bicubic", 7, 2, fp)[0]
        assert np.array_equal(a[1], b[1])
        assert np.allclose(b[0], a[0] * sc, rtol=1e-14, atol=1e-15)
    r0 = o.reference_filter([h], uv, "bilinear")[0]
    r1 = o.reference_filter([(h, "f16", sc)], uv, "bilinear")[0]
    assert np.allclose(r1, r0 * sc, rtol=1e-14, atol=1e-15)
    g = rng.standard_normal((4, 64, 4))
    d0 = o.stf_adjoint([h], uv, "bicubic", 7, 2, "tile8x8", [g])[0]
    d1 = o.stf_adjoint([(h, "f16", sc)], uv, "bicubic", 7, 2, "tile8x8", [g])[0]
    assert np.allclose(d1, d0 * sc, rtol=1e-14, atol=1e-15)


def test_latent_texture_filters_decoded_values():
    # the identity-like decoder returns the first four latents, so filtering
    # the latent grid equals filtering those channels directly
    W1 = np.zeros((64, 8)); W2 = np.zeros((64, 64)); W3 = np.zeros((4, 64))
    for i in range(4):
        W1[i, i], W1[4 + i, i] = 1.0, -1.0
        W3[i, i], W3[i, 4 + i] = 1.0, -1.0
    for j in range(8):
        W2[j, j] = 1.0
    layers = [(W1, np.zeros(64)), (W2, np.zeros(64)), (W3, np.zeros(4))]
    rng = np.random.default_rng(11)
    lat = rng.standard_normal((16, 16, 8)).astype(np.float16)
    uv = _tiny_screen(2)
    a = o.stf_filter_reuse([(lat, "f16", None, layers)], uv, "bicubic", 3, 0, "tile8x8")[0]
    b = o.stf_filter_reuse([lat[..., :4].astype(np.float64)], uv, "bicubic", 3, 0, "tile8x8")[0]
    assert np.array_equal(a[1], b[1]) and np.allclose(a[0], b[0], rtol=1e-14, atol=1e-15)
