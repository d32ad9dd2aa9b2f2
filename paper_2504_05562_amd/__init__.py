"""Python binding of libstf.so: stochastic texture filtering with sample reuse
on MI355X (gfx950).

Argument marshalling only: every step of the filtering runs in the HIP
kernels behind the C ABI of include/stf.h. PyTorch provides device memory and
the stream; there is no CPU fallback. Importing works without a GPU; calling
anything without the built library raises.

Textures are torch tensors [H, W, C] on the GPU: uint8 with C=4 (RGBA8 UNORM)
or C=1 (R8 UNORM), float16 with C=4 (RGBA16F) or C=2 (RG16F), float32 with
C=4 (RGBA32F) or C=1 (R32F), bfloat16 or float8_e4m3fn with C=4. Each texture
may carry a per-channel dequantization scale (`scales`). UV is float32
[H, W, 2]. Outputs are float32 [H, W, C] per texture.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

__all__ = [
    "BILINEAR", "BICUBIC", "FOOTPRINTS", "FORMATS", "library", "lib_path", "version",
    "filter", "filter_reuse", "filter_reference", "backward", "StfError", "pack_decoder",
    "generate_footprints", "generate_footprints_static", "footprint_set", "stf_reuse_autograd",
    "backward_decoder", "stf_decoder_autograd",
]

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libstf.so")

BILINEAR = 0
BICUBIC = 1
FILTERS = {"bilinear": BILINEAR, "bicubic": BICUBIC}
FOOTPRINTS = {"self": 0, "quad2x2": 1, "wave2x2": 2, "square3x3": 3, "square4x4": 4, "tile8x8": 5, "lut": 6}
# (torch dtype name, channels) -> (stf_format, bytes per texel)
FORMATS = {
    ("uint8", 4): (0, 4), ("float16", 4): (1, 8), ("float16", 2): (2, 4),
    ("uint8", 1): (3, 1), ("float32", 4): (4, 16), ("float32", 1): (5, 4),
    ("bfloat16", 4): (6, 8), ("float8_e4m3fn", 4): (7, 4),
    ("float16", 8): (8, 16), ("bfloat16", 8): (9, 16), ("float8_e4m3fn", 8): (10, 8),
}
# 8-channel textures are latent grids, decoded to RGBA by a packed decoder
LATENT_FORMATS = (8, 9, 10)
LATENT_OUT_CHANNELS = 4
STF_MAX_TEXTURES = 4


class StfError(RuntimeError):
    pass


class Texture(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch_bytes", ctypes.c_int64), ("format", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("scale", ctypes.c_void_p), ("decoder", ctypes.c_void_p)]


class Mlp(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("w1", "b1", "w2", "b2", "w3", "b3")] + \
               [("precision", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class MlpGrad(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("w1", "b1", "w2", "b2", "w3", "b3")]


DECODER_BYTES = 14736
DECODER_PRECISIONS = {"bf16": 0, "fp8": 1}


class FootprintParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n_cand", ctypes.c_int32), ("sigma", ctypes.c_float),
                ("trials", ctypes.c_int32), ("restarts", ctypes.c_int32), ("seed", ctypes.c_uint32),
                ("reserved", ctypes.c_int32)]


class Screen(ctypes.Structure):
    _fields_ = [("uv", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("filter", ctypes.c_int32), ("address", ctypes.c_int32),
                ("seed", ctypes.c_uint32), ("frame", ctypes.c_uint32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


SHARE_SELECTION = 1
FLOAT_BIN_SUMS = 2


class Reuse(ctypes.Structure):
    _fields_ = [("footprint", ctypes.c_int32), ("lut_k", ctypes.c_int32), ("lut", ctypes.c_void_p),
                ("flags", ctypes.c_int32), ("estimator", ctypes.c_int32)]


EXACT_FILTERING = 1
CLAMP = 2
ESTIMATORS = {"wis": 0, "is": 1, "mis": 2, "pmis": 3, "regression": 4}


_lib = None
_SYMBOLS = ("stf_filter", "stf_filter_reuse", "stf_filter_reference", "stf_backward",
            "stf_decoder_pack", "stf_footprint_workspace_bytes", "stf_footprint_generate",
            "stf_footprint_generate_static", "stf_backward_decoder", "stf_backward_decoder_workspace_bytes",
            "stf_last_error", "stf_version")


def library() -> ctypes.CDLL:
    """Load libstf.so (built in-tree by build.py). Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise StfError(f"{lib_path} is missing: build it with paper_2504_05562_amd/build.py")
        lib = ctypes.CDLL(lib_path)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        tex_args = [P(Texture), ctypes.c_int32, P(Screen), P(Params)]
        lib.stf_filter.argtypes = tex_args + [P(vp), vp, vp]
        lib.stf_filter_reuse.argtypes = tex_args + [P(Reuse), P(vp), vp, vp]
        lib.stf_filter_reference.argtypes = tex_args + [P(vp), vp]
        lib.stf_backward.argtypes = tex_args + [P(Reuse), P(vp), P(vp), vp]
        lib.stf_decoder_pack.argtypes = [P(Mlp), vp, vp]
        lib.stf_footprint_workspace_bytes.argtypes = [P(FootprintParams)]
        lib.stf_footprint_workspace_bytes.restype = ctypes.c_int64
        lib.stf_footprint_generate.argtypes = [P(FootprintParams), vp, ctypes.c_int64, vp, vp, vp]
        lib.stf_footprint_generate.restype = ctypes.c_int
        lib.stf_backward_decoder_workspace_bytes.argtypes = [P(Texture), ctypes.c_int32]
        lib.stf_backward_decoder_workspace_bytes.restype = ctypes.c_int64
        lib.stf_backward_decoder.argtypes = tex_args + [P(Reuse), P(vp), P(Mlp), P(vp), P(MlpGrad), vp,
                                                        ctypes.c_int64, vp]
        lib.stf_backward_decoder.restype = ctypes.c_int
        lib.stf_footprint_generate_static.argtypes = [P(FootprintParams), vp, vp, vp]
        lib.stf_footprint_generate_static.restype = ctypes.c_int
        for name in ("stf_filter", "stf_filter_reuse", "stf_filter_reference", "stf_backward",
                     "stf_decoder_pack", "stf_version"):
            getattr(lib, name).restype = ctypes.c_int
        lib.stf_last_error.restype = ctypes.c_char_p
        lib.stf_last_error.argtypes = []
        _lib = lib
    return _lib


def version() -> int:
    return library().stf_version()


def _check(rc: int) -> None:
    if rc != 0:
        msg = library().stf_last_error().decode()
        raise StfError(f"stf status {rc}: {msg}")


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


MLP_SHAPES = [((64, 8), (64,)), ((64, 64), (64,)), ((4, 64), (4,))]


def _mlp_arrays(layers, what="decoder"):
    """The six arrays of [(W1 [64,8], b1), (W2 [64,64], b2), (W3 [4,64], b3)],
    checked to be contiguous float32 GPU tensors of those shapes."""
    import torch
    if len(layers) != 3:
        raise ValueError(f"{what}: three (W, b) layers expected")
    flat = []
    for (wt, bt), (ws, bs) in zip(layers, MLP_SHAPES):
        for t, sh in ((wt, ws), (bt, bs)):
            if (not isinstance(t, torch.Tensor) or tuple(t.shape) != sh or t.dtype != torch.float32
                    or not t.is_cuda or not t.is_contiguous()):
                raise ValueError(f"{what} arrays must be contiguous float32 GPU tensors of shape {sh}")
            flat.append(t)
    return flat


def pack_decoder(layers, stream=None, precision="bf16"):
    """Pack the latent decoder MLP [(W1 [64,8], b1), (W2 [64,64], b2),
    (W3 [4,64], b3)] (float32 GPU tensors) with stf_decoder_pack for BF16 or
    FP8 matrix-core arithmetic. Returns the packed uint8 GPU tensor to pass
    as `decoder=`."""
    import torch
    flat = _mlp_arrays(layers)
    packed = torch.empty(DECODER_BYTES, dtype=torch.uint8, device=flat[0].device)
    m = Mlp(*[t.data_ptr() for t in flat], DECODER_PRECISIONS[precision], 0)
    _check(library().stf_decoder_pack(ctypes.byref(m), ctypes.c_void_p(packed.data_ptr()), _stream_handle(stream)))
    return packed


def generate_footprints(k=9, n_cand=32, sigma=1.4, trials=10000, restarts=30, seed=0, device="cuda",
                        stream=None):
    """Pseudorandom sparse sharing footprints (stf_footprint_generate):
    returns (lut uint8 GPU tensor [64, k-1] for footprint='lut', score int64
    GPU tensor [1])."""
    import torch
    lib = library()
    prm = FootprintParams(int(k), int(n_cand), float(sigma), int(trials), int(restarts), int(seed) & 0xFFFFFFFF, 0)
    nbytes = lib.stf_footprint_workspace_bytes(ctypes.byref(prm))
    if nbytes < 0:
        raise StfError(lib.stf_last_error().decode())
    ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    lut = torch.empty((64, int(k) - 1), dtype=torch.uint8, device=device)
    score = torch.empty(1, dtype=torch.int64, device=device)
    _check(lib.stf_footprint_generate(ctypes.byref(prm), ctypes.c_void_p(ws.data_ptr() + off), ctypes.c_int64(nbytes),
                                      ctypes.c_void_p(lut.data_ptr()), ctypes.c_void_p(score.data_ptr()),
                                      _stream_handle(stream)))
    return lut, score


FOOTPRINT_STATIC_BYTES = 4 << 20


def generate_footprints_static(k=9, n_cand=32, sigma=1.4, trials=10000, restarts=30, seed=0, lut=None,
                               score=None, device="cuda", stream=None):
    """generate_footprints through stf_footprint_generate_static: the library
    uses its static per-GPU workspace and allocates nothing. With `lut`
    (uint8 GPU tensor [64, k-1]) and `score` (int64 GPU tensor [1]) given,
    this function allocates nothing either."""
    import torch
    if lut is None:
        lut = torch.empty((64, int(k) - 1), dtype=torch.uint8, device=device)
    if score is None:
        score = torch.empty(1, dtype=torch.int64, device=device)
    if (lut.dtype != torch.uint8 or tuple(lut.shape) != (64, int(k) - 1) or not lut.is_cuda
            or not lut.is_contiguous()):
        raise ValueError(f"lut must be a contiguous uint8 GPU tensor [64, {int(k) - 1}]")
    if score.dtype != torch.int64 or score.numel() < 1 or not score.is_cuda:
        raise ValueError("score must be an int64 GPU tensor of at least one element")
    prm = FootprintParams(int(k), int(n_cand), float(sigma), int(trials), int(restarts), int(seed) & 0xFFFFFFFF, 0)
    _check(library().stf_footprint_generate_static(ctypes.byref(prm), ctypes.c_void_p(lut.data_ptr()),
                                                   ctypes.c_void_p(score.data_ptr()), _stream_handle(stream)))
    return lut, score


def footprint_set(frames, k=9, n_cand=32, sigma=1.4, trials=10000, restarts=30, seed=0, device="cuda"):
    """`frames` footprint LUTs with seeds seed, seed + 1, ... (uint8 GPU
    tensor [frames, 64, k-1]); frame f filters with set[f % frames], which
    cycles the patterns over frames (Sec. 4.3)."""
    import torch
    return torch.stack([generate_footprints(k, n_cand, sigma, trials, restarts, seed + f, device)[0]
                        for f in range(int(frames))])


def _texture_descs(textures: Sequence, need_data: bool = True, scales=None, decoder=None):
    """Descriptors, filtered channels per texture, and the host scale arrays
    (kept alive by the caller for the duration of the call)."""
    if not 1 <= len(textures) <= STF_MAX_TEXTURES:
        raise ValueError(f"1..{STF_MAX_TEXTURES} textures expected")
    if scales is not None and len(scales) != len(textures):
        raise ValueError("one scale entry (or None) per texture expected")
    arr = (Texture * len(textures))()
    chans = []
    keep = []
    for i, t in enumerate(textures):
        if t.dim() != 3:
            raise ValueError("texture tensors are [H, W, C]")
        key = (str(t.dtype).replace("torch.", ""), int(t.shape[2]))
        if key not in FORMATS:
            raise ValueError(f"unsupported texture dtype/channels {key}")
        fmt, bpp = FORMATS[key]
        if need_data:
            if not t.is_cuda:
                raise ValueError("textures must be GPU tensors")
            C, W = int(t.shape[2]), int(t.shape[1])
            if (C > 1 and t.stride(2) != 1) or (W > 1 and t.stride(1) != C):
                raise ValueError("texels must be packed within a row")
        arr[i].data = t.data_ptr() if need_data else None
        arr[i].width = int(t.shape[1])
        arr[i].height = int(t.shape[0])
        arr[i].pitch_bytes = int(t.stride(0)) * t.element_size()
        arr[i].format = fmt
        arr[i].reserved = 0
        sc = None if scales is None else scales[i]
        if sc is not None:
            vals = [float(v) for v in sc]
            if len(vals) != int(t.shape[2]):
                raise ValueError(f"texture {i}: {int(t.shape[2])} scale values expected")
            buf = (ctypes.c_float * len(vals))(*vals)
            keep.append(buf)
            arr[i].scale = ctypes.cast(buf, ctypes.c_void_p)
        else:
            arr[i].scale = None
        if fmt in LATENT_FORMATS:
            if decoder is None:
                raise ValueError(f"texture {i} holds latents: pass decoder= (from pack_decoder)")
            if (decoder.dtype != __import__("torch").uint8 or decoder.numel() != DECODER_BYTES
                    or not decoder.is_cuda or not decoder.is_contiguous()):
                raise ValueError(f"decoder must be the contiguous uint8 GPU tensor of {DECODER_BYTES} bytes "
                                 "from pack_decoder")
            arr[i].decoder = decoder.data_ptr()
        else:
            arr[i].decoder = None
        chans.append(LATENT_OUT_CHANNELS if fmt in LATENT_FORMATS else int(t.shape[2]))
    return arr, chans, keep


def _screen(uv):
    import torch
    if uv.dtype != torch.float32 or uv.dim() != 3 or uv.shape[2] != 2 or not uv.is_cuda or not uv.is_contiguous():
        raise ValueError("uv must be a contiguous float32 GPU tensor [H, W, 2]")
    return Screen(uv.data_ptr(), int(uv.shape[1]), int(uv.shape[0]))


def _params(filter, seed, frame, share_selection=False, float_bin_sums=False):
    f = FILTERS[filter] if isinstance(filter, str) else int(filter)
    return Params(f, 0, int(seed) & 0xFFFFFFFF, int(frame) & 0xFFFFFFFF,
                  (SHARE_SELECTION if share_selection else 0) | (FLOAT_BIN_SUMS if float_bin_sums else 0), 0)


def _check_buffers(name, bufs, shapes, device):
    """The kernels write (or atomically add) whole [rows, cols, C] FP32 arrays
    through these pointers: one contiguous float32 tensor of exactly that
    shape per texture, on the launch device, or the call is refused here."""
    import torch
    if len(bufs) != len(shapes):
        raise ValueError(f"{name}: {len(shapes)} tensors expected, got {len(bufs)}")
    for i, (b, sh) in enumerate(zip(bufs, shapes)):
        if not isinstance(b, torch.Tensor) or b.dtype != torch.float32 or not b.is_cuda or not b.is_contiguous():
            raise ValueError(f"{name}[{i}] must be a contiguous float32 GPU tensor")
        if tuple(b.shape) != tuple(sh):
            raise ValueError(f"{name}[{i}] has shape {tuple(b.shape)}, {tuple(sh)} expected")
        if b.device != device:
            raise ValueError(f"{name}[{i}] is on {b.device}, the screen on {device}")


def _outputs(uv, chans, out=None):
    import torch
    H, W = int(uv.shape[0]), int(uv.shape[1])
    if out is None:
        out = [torch.empty((H, W, c), dtype=torch.float32, device=uv.device) for c in chans]
    else:
        out = list(out)
        _check_buffers("out", out, [(H, W, c) for c in chans], uv.device)
    ptrs = (ctypes.c_void_p * len(out))(*[o.data_ptr() for o in out])
    return out, ptrs


def _reuse(footprint, lut, exact_filtering=False, estimator="wis", clamp=False):
    fp = FOOTPRINTS[footprint] if isinstance(footprint, str) else int(footprint)
    flags = (EXACT_FILTERING if exact_filtering else 0) | (CLAMP if clamp else 0)
    est = ESTIMATORS[estimator] if isinstance(estimator, str) else int(estimator)
    if lut is None:
        return Reuse(fp, 0, None, flags, est)
    if (lut.dtype != __import__("torch").uint8 or lut.dim() != 2 or lut.shape[0] != 64 or not lut.is_contiguous()
            or not lut.is_cuda):
        raise ValueError("lut must be a contiguous uint8 GPU tensor [64, K]")
    return Reuse(fp, int(lut.shape[1]), lut.data_ptr(), flags, est)


def filter(textures, uv, filter="bicubic", seed=0, frame=0, sel=False, out=None, stream=None, scales=None, decoder=None,
           share_selection=False):
    """One-tap STF (stf_filter). Returns a list of outputs, plus the int32
    selection tensor [ntex, H, W, 2] if sel=True. `scales` holds, per
    texture, None or one dequantization scale per channel."""
    import torch
    lib = library()
    descs, chans, _keep = _texture_descs(textures, scales=scales, decoder=decoder)
    scr = _screen(uv)
    prm = _params(filter, seed, frame, share_selection)
    out, ptrs = _outputs(uv, chans, out)
    s = torch.empty((len(textures),) + tuple(uv.shape[:2]) + (2,), dtype=torch.int32, device=uv.device) if sel else None
    _check(lib.stf_filter(descs, len(textures), ctypes.byref(scr), ctypes.byref(prm), ptrs,
                          ctypes.c_void_p(s.data_ptr() if s is not None else None), _stream_handle(stream)))
    return (out, s) if sel else out


def filter_reuse(textures, uv, footprint="tile8x8", filter="bicubic", seed=0, frame=0, lut=None,
                 sel=False, out=None, stream=None, scales=None, decoder=None, exact_filtering=False,
                 estimator="wis", clamp=False, share_selection=False, float_bin_sums=False):
    """STF with sample reuse (stf_filter_reuse). `lut` is a uint8 GPU tensor
    [64, K] of tile pixel ids for footprint='lut'; exact_filtering selects
    STF_REUSE_EXACT_FILTERING; estimator ('wis' = Eq. (14), 'is', 'mis',
    'pmis', 'regression') and clamp select the comparison estimators;
    float_bin_sums sets STF_FLOAT_BIN_SUMS (a testing aid)."""
    import torch
    lib = library()
    descs, chans, _keep = _texture_descs(textures, scales=scales, decoder=decoder)
    scr = _screen(uv)
    prm = _params(filter, seed, frame, share_selection, float_bin_sums)
    r = _reuse(footprint, lut, exact_filtering, estimator, clamp)
    out, ptrs = _outputs(uv, chans, out)
    s = torch.empty((len(textures),) + tuple(uv.shape[:2]) + (2,), dtype=torch.int32, device=uv.device) if sel else None
    _check(lib.stf_filter_reuse(descs, len(textures), ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(r), ptrs,
                                ctypes.c_void_p(s.data_ptr() if s is not None else None), _stream_handle(stream)))
    return (out, s) if sel else out


def filter_reference(textures, uv, filter="bicubic", out=None, stream=None, scales=None, decoder=None):
    """Deterministic filter of Eq. (3) (stf_filter_reference)."""
    lib = library()
    descs, chans, _keep = _texture_descs(textures, scales=scales, decoder=decoder)
    scr = _screen(uv)
    prm = _params(filter, 0, 0)
    out, ptrs = _outputs(uv, chans, out)
    _check(lib.stf_filter_reference(descs, len(textures), ctypes.byref(scr), ctypes.byref(prm), ptrs,
                                    _stream_handle(stream)))
    return out


def backward(textures, uv, grads, footprint="tile8x8", filter="bicubic", seed=0, frame=0, lut=None,
             dtex=None, stream=None, scales=None, share_selection=False, float_bin_sums=False):
    """Adjoint of filter_reuse (stf_backward): accumulates dL/dT into `dtex`
    (float32 [H_t, W_t, C] per texture; zero-initialised if not given)."""
    import torch
    lib = library()
    descs, chans, _keep = _texture_descs(textures, scales=scales)
    scr = _screen(uv)
    prm = _params(filter, seed, frame, share_selection, float_bin_sums)
    r = _reuse(footprint, lut)
    tex_shapes = [(int(t.shape[0]), int(t.shape[1]), c) for t, c in zip(textures, chans)]
    if dtex is None:
        dtex = [torch.zeros(sh, dtype=torch.float32, device=uv.device) for sh in tex_shapes]
    else:
        dtex = list(dtex)
        _check_buffers("dtex", dtex, tex_shapes, uv.device)
    grads = list(grads)
    H, W = int(uv.shape[0]), int(uv.shape[1])
    _check_buffers("grads", grads, [(H, W, c) for c in chans], uv.device)
    gp = (ctypes.c_void_p * len(grads))(*[g.data_ptr() for g in grads])
    dp = (ctypes.c_void_p * len(dtex))(*[d.data_ptr() for d in dtex])
    _check(lib.stf_backward(descs, len(textures), ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(r), gp, dp,
                            _stream_handle(stream)))
    return dtex


def backward_decoder(textures, uv, grads, layers, decoder, footprint="tile8x8", filter="bicubic", seed=0, frame=0,
                     lut=None, scales=None, dlatent=None, dlayers=None, share_selection=False, precision="bf16",
                     stream=None):
    """Adjoint of filter_reuse over latent textures through the decoder
    (stf_backward_decoder): accumulates dL/d(stored latent) into `dlatent`
    (float32 [H_t, W_t, 8] per texture) and the FP32 decoder's weight and
    bias gradients into `dlayers` (same structure as `layers`, the FP32
    weights `decoder` was packed from); both zero-initialised if not given."""
    import torch
    lib = library()
    descs, chans, _keep = _texture_descs(textures, scales=scales, decoder=decoder)
    if any(d.format not in LATENT_FORMATS for d in descs):
        raise ValueError("backward_decoder takes latent textures (8 channels)")
    scr = _screen(uv)
    prm = _params(filter, seed, frame, share_selection)
    r = _reuse(footprint, lut)
    flat = _mlp_arrays(layers)
    if dlayers is None:
        dlayers = [(torch.zeros_like(wt), torch.zeros_like(bt)) for wt, bt in layers]
    gflat = _mlp_arrays(dlayers, "gradient")
    shapes = [(int(t.shape[0]), int(t.shape[1]), 8) for t in textures]
    if dlatent is None:
        dlatent = [torch.zeros(sh, dtype=torch.float32, device=uv.device) for sh in shapes]
    else:
        dlatent = list(dlatent)
        _check_buffers("dlatent", dlatent, shapes, uv.device)
    grads = list(grads)
    H, W = int(uv.shape[0]), int(uv.shape[1])
    _check_buffers("grads", grads, [(H, W, 4)] * len(textures), uv.device)
    nbytes = lib.stf_backward_decoder_workspace_bytes(descs, len(textures))
    if nbytes < 0:
        raise StfError(lib.stf_last_error().decode())
    ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=uv.device)
    off = (-ws.data_ptr()) % 256
    m = Mlp(*[t.data_ptr() for t in flat], DECODER_PRECISIONS[precision], 0)
    mg = MlpGrad(*[t.data_ptr() for t in gflat])
    gp = (ctypes.c_void_p * len(grads))(*[g.data_ptr() for g in grads])
    dp = (ctypes.c_void_p * len(dlatent))(*[d.data_ptr() for d in dlatent])
    _check(lib.stf_backward_decoder(descs, len(textures), ctypes.byref(scr), ctypes.byref(prm), ctypes.byref(r), gp,
                                    ctypes.byref(m), dp, ctypes.byref(mg), ctypes.c_void_p(ws.data_ptr() + off),
                                    ctypes.c_int64(nbytes), _stream_handle(stream)))
    return dlatent, dlayers


def _autograd_function():
    import torch

    class STFReuse(torch.autograd.Function):
        """Differentiable reuse STF of one texture (float32 [H, W, C], C in
        {1, 4}): forward = stf_filter_reuse, backward = stf_backward. The
        weights depend only on UV and random numbers, so the gradient with
        respect to UV is not defined (returned as None)."""

        @staticmethod
        def forward(ctx, texture, uv, footprint, filter, seed, frame):
            ctx.save_for_backward(texture, uv)
            ctx.cfg = (footprint, filter, seed, frame)
            return filter_reuse([texture.detach()], uv.detach(), footprint, filter, seed, frame)[0]

        @staticmethod
        def backward(ctx, grad_out):
            texture, uv = ctx.saved_tensors
            footprint, filt, seed, frame = ctx.cfg
            g = backward([texture], uv, [grad_out.contiguous().float()], footprint, filt, seed, frame)[0]
            return g.view_as(texture), None, None, None, None, None

    return STFReuse


_STFReuse = None
_STFDecoderReuse = None


def _decoder_autograd_function():
    import torch

    class STFDecoderReuse(torch.autograd.Function):
        """Differentiable reuse STF of a latent grid through the decoder MLP:
        forward = FP16 storage of the latents, stf_decoder_pack (BF16) and
        stf_filter_reuse; backward = stf_backward_decoder (FP32 decoder,
        rounding to FP16 and BF16 passed straight through)."""

        @staticmethod
        def forward(ctx, latents, w1, b1, w2, b2, w3, b3, uv, footprint, filter, seed, frame):
            layers = [(w1.detach(), b1.detach()), (w2.detach(), b2.detach()), (w3.detach(), b3.detach())]
            stored = latents.detach().to(torch.float16).contiguous()
            dec = pack_decoder(layers)
            ctx.save_for_backward(stored, uv, dec, w1, b1, w2, b2, w3, b3)
            ctx.cfg = (footprint, filter, seed, frame)
            return filter_reuse([stored], uv.detach(), footprint, filter, seed, frame, decoder=dec)[0]

        @staticmethod
        def backward(ctx, grad_out):
            stored, uv, dec, w1, b1, w2, b2, w3, b3 = ctx.saved_tensors
            footprint, filt, seed, frame = ctx.cfg
            layers = [(w1.detach(), b1.detach()), (w2.detach(), b2.detach()), (w3.detach(), b3.detach())]
            (dlat,), dl = backward_decoder([stored], uv, [grad_out.contiguous().float()], layers, dec, footprint, filt,
                                           seed, frame)
            return (dlat, dl[0][0], dl[0][1], dl[1][0], dl[1][1], dl[2][0], dl[2][1],
                    None, None, None, None, None)

    return STFDecoderReuse


def stf_decoder_autograd(latents, layers, uv, footprint="tile8x8", filter="bicubic", seed=0, frame=0):
    """torch.autograd entry for neural textures: reuse STF of an FP32 latent
    grid [H_t, W_t, 8] (stored as FP16 for the forward pass) decoded by the
    MLP `layers` [(W1, b1), (W2, b2), (W3, b3)] of FP32 tensors (packed to
    BF16 for the forward pass); differentiable with respect to the latents
    and every weight and bias."""
    global _STFDecoderReuse
    if _STFDecoderReuse is None:
        _STFDecoderReuse = _decoder_autograd_function()
    (w1, b1), (w2, b2), (w3, b3) = layers
    return _STFDecoderReuse.apply(latents, w1, b1, w2, b2, w3, b3, uv, footprint, filter, seed, frame)


def stf_reuse_autograd(texture, uv, footprint="tile8x8", filter="bicubic", seed=0, frame=0):
    """torch.autograd entry: reuse STF of a float32 texture, differentiable
    with respect to the texels."""
    global _STFReuse
    if _STFReuse is None:
        _STFReuse = _autograd_function()
    return _STFReuse.apply(texture, uv, footprint, filter, seed, frame)
