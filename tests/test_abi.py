"""The C-ABI library loads and exports every symbol include/stf.h declares;
argument validation rejects bad calls on the host before any launch (no GPU
compute is run here)."""
import ctypes
import os
import re

import pytest

import paper_2504_05562_amd as stf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "stf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stf_[a-z_]+)\s*\(", text)))


def _define(name):
    text = open(os.path.join(ROOT, "include", "stf.h")).read()
    return int(re.search(r"#define\s+" + name + r"\s+(\d+)", text).group(1))


def test_library_exports_every_declared_symbol():
    lib = stf.library()
    names = declared_functions()
    assert {"stf_filter", "stf_filter_reuse", "stf_filter_reference", "stf_backward",
            "stf_last_error", "stf_version"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert stf.version() == 2


def test_texture_descriptor_layout():
    # stf_texture: pointer, 2 x int32, int64, 2 x int32, pointer, pointer
    assert ctypes.sizeof(stf.Texture) == 48
    assert stf.Texture.scale.offset == 32 and stf.Texture.decoder.offset == 40
    assert ctypes.sizeof(stf.Mlp) == 56
    assert ctypes.sizeof(stf.Reuse) == 24 and stf.Reuse.flags.offset == 16


_NAN_SCALE = (ctypes.c_float * 4)(1.0, float("nan"), 1.0, 1.0)


def _call_filter(tex, ntex, scr, prm):
    lib = stf.library()
    out = (ctypes.c_void_p * 4)(16, 32, 48, 64)
    return lib.stf_filter(tex, ntex, scr, prm, out, None, None)


def _good():
    tex = (stf.Texture * 1)()
    tex[0].data = 256
    tex[0].width = 64
    tex[0].height = 64
    tex[0].pitch_bytes = 64 * 4
    tex[0].format = 0
    scr = stf.Screen(4096, 16, 16)
    prm = stf.Params(1, 0, 0, 0)
    return tex, scr, prm


@pytest.mark.parametrize("mutate,code,needle", [
    (lambda t, s, p: setattr(s, "uv", None), -1, "uv"),
    (lambda t, s, p: setattr(s, "width", 0), -1, "screen"),
    (lambda t, s, p: setattr(p, "filter", 7), -1, "filter"),
    (lambda t, s, p: setattr(p, "address", 1), -2, "address"),
    (lambda t, s, p: setattr(t[0], "format", 99), -1, "format"),
    (lambda t, s, p: setattr(t[0], "width", 48), -1, "powers of two"),
    (lambda t, s, p: setattr(t[0], "height", 2), -1, "powers of two"),
    (lambda t, s, p: setattr(t[0], "pitch_bytes", 100), -1, "pitch"),
    (lambda t, s, p: setattr(t[0], "data", None), -1, "data"),
    (lambda t, s, p: setattr(t[0], "reserved", 1), -1, "reserved"),
    (lambda t, s, p: setattr(t[0], "format", 8), -1, "decoder"),
    (lambda t, s, p: setattr(t[0], "decoder", 4096), -1, "not latent"),
    (lambda t, s, p: setattr(t[0], "scale", ctypes.cast(_NAN_SCALE, ctypes.c_void_p)), -1, "scale"),
])
def test_validation_errors(mutate, code, needle):
    tex, scr, prm = _good()
    mutate(tex, scr, prm)
    rc = _call_filter(tex, 1, ctypes.byref(scr), ctypes.byref(prm))
    assert rc == code
    assert needle in stf.library().stf_last_error().decode()


def test_validation_counts_and_nulls():
    lib = stf.library()
    tex, scr, prm = _good()
    assert _call_filter(tex, 0, ctypes.byref(scr), ctypes.byref(prm)) == -1
    assert _call_filter(tex, 5, ctypes.byref(scr), ctypes.byref(prm)) == -1
    assert lib.stf_filter(None, 1, ctypes.byref(scr), ctypes.byref(prm), None, None, None) == -1
    assert lib.stf_filter_reuse(tex, 1, ctypes.byref(scr), ctypes.byref(prm), None, None, None, None) == -1
    bad_fp = stf.Reuse(42, 0, None)
    out = (ctypes.c_void_p * 1)(4096)
    assert lib.stf_filter_reuse(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(bad_fp), out, None, None) == -1
    bad_flags = stf.Reuse(5, 0, None, 4, 0)
    assert lib.stf_filter_reuse(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(bad_flags), out, None, None) == -1
    bad_est = stf.Reuse(5, 0, None, 0, 7)
    assert lib.stf_filter_reuse(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(bad_est), out, None, None) == -1
    ef_is = stf.Reuse(5, 0, None, 1, 1)
    assert lib.stf_filter_reuse(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(ef_is), out, None, None) == -2
    clamp_bwd = stf.Reuse(5, 0, None, 2, 0)
    dq = (ctypes.c_void_p * 1)(4096)
    assert lib.stf_backward(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(clamp_bwd), dq, dq, None) == -2
    ef = stf.Reuse(5, 0, None, 1, 0)
    dp = (ctypes.c_void_p * 1)(4096)
    assert lib.stf_backward(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(ef), dp, dp, None) == -2
    lut_missing = stf.Reuse(6, 4, None)
    assert lib.stf_filter_reuse(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(lut_missing), out, None, None) == -1
    assert b"lut" in lib.stf_last_error()


def test_backward_gradient_alignment():
    # dL/dout is read as one vector of the slot's channels per pixel: RGBA
    # needs 16-byte alignment; the gradient texels need 4
    lib = stf.library()
    tex, scr, prm = _good()
    plain = stf.Reuse(5, 0, None, 0, 0)
    dtex = (ctypes.c_void_p * 1)(8192)
    for bad in (4100, 4104, 4108):
        dout = (ctypes.c_void_p * 1)(bad)
        assert lib.stf_backward(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(plain), dout, dtex,
                                None) == -1
        assert b"16-byte" in lib.stf_last_error()
    dout = (ctypes.c_void_p * 1)(4096)
    odd = (ctypes.c_void_p * 1)(8194)
    assert lib.stf_backward(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(plain), dout, odd, None) == -1
    assert b"aligned" in lib.stf_last_error()


def test_latent_and_decoder_validation():
    lib = stf.library()
    tex, scr, prm = _good()
    tex[0].format = 10                                   # FP8 latents, 8 bytes per texel
    tex[0].pitch_bytes = 64 * 8
    tex[0].decoder = 4100                                # misaligned
    assert _call_filter(tex, 1, ctypes.byref(scr), ctypes.byref(prm)) == -1
    assert b"aligned" in lib.stf_last_error()
    two = (stf.Texture * 2)(tex[0], tex[0])
    two[0].decoder, two[1].decoder = 4096, 8192         # two different decoders in one call
    assert _call_filter(two, 2, ctypes.byref(scr), ctypes.byref(prm)) == -2
    # the adjoint does not go through the decoder
    tex[0].decoder = 4096
    r = stf.Reuse(5, 0, None)
    ptrs = (ctypes.c_void_p * 1)(4096)
    assert lib.stf_backward(tex, 1, ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(r), ptrs, ptrs, None) == -2
    # the packer validates its pointers before launching anything
    m = stf.Mlp(4096, 4096, 4096, None, 4096, 4096, 0, 0)
    assert lib.stf_decoder_pack(ctypes.byref(m), ctypes.c_void_p(4096), None) == -1
    m = stf.Mlp(4096, 4096, 4096, 4096, 4096, 4096, 2, 0)
    assert lib.stf_decoder_pack(ctypes.byref(m), ctypes.c_void_p(4096), None) == -1
    m = stf.Mlp(4096, 4096, 4096, 4096, 4096, 4096, 1, 5)
    assert lib.stf_decoder_pack(ctypes.byref(m), ctypes.c_void_p(4096), None) == -1
    m = stf.Mlp(4096, 4096, 4096, 4096, 4096, 4096, 0, 0)
    assert lib.stf_decoder_pack(ctypes.byref(m), ctypes.c_void_p(4104), None) == -1
    assert lib.stf_decoder_pack(None, ctypes.c_void_p(4096), None) == -1


def test_footprint_generator_validation():
    lib = stf.library()
    good = stf.FootprintParams(9, 32, 1.4, 10000, 30, 0, 0)
    n = lib.stf_footprint_workspace_bytes(ctypes.byref(good))
    assert n >= 30 * 64 * 32 * 8 and n % 256 == 0
    for bad in (stf.FootprintParams(1, 32, 1.4, 10, 3, 0, 0), stf.FootprintParams(9, 0, 1.4, 10, 3, 0, 0),
                stf.FootprintParams(9, 32, 0.0, 10, 3, 0, 0), stf.FootprintParams(9, 32, 1.4, 0, 3, 0, 0),
                stf.FootprintParams(9, 32, 1.4, 10, 0, 0, 0), stf.FootprintParams(9, 32, 1.4, 10, 3, 0, 1)):
        assert lib.stf_footprint_workspace_bytes(ctypes.byref(bad)) == -1
    assert lib.stf_footprint_generate(ctypes.byref(good), None, n, ctypes.c_void_p(4096), None, None) == -1
    assert lib.stf_footprint_generate(ctypes.byref(good), ctypes.c_void_p(4096), n - 1, ctypes.c_void_p(4096),
                                      None, None) == -1
    assert b"workspace" in lib.stf_last_error()
    assert lib.stf_footprint_generate(ctypes.byref(good), ctypes.c_void_p(4096 + 64), n, ctypes.c_void_p(4096),
                                      None, None) == -1


def test_params_layout_and_flags():
    assert ctypes.sizeof(stf.Params) == 24
    tex, scr, prm = _good()
    prm.flags = 4                       # neither STF_SHARE_SELECTION nor STF_FLOAT_BIN_SUMS
    assert _call_filter(tex, 1, ctypes.byref(scr), ctypes.byref(prm)) == -1
    assert (stf.SHARE_SELECTION, stf.FLOAT_BIN_SUMS) == (_define("STF_SHARE_SELECTION"), _define("STF_FLOAT_BIN_SUMS"))
    prm.flags, prm.reserved = 1, 3
    assert _call_filter(tex, 1, ctypes.byref(scr), ctypes.byref(prm)) == -1
