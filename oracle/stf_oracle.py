"""Step-by-step FP64 reference for STF with sample reuse (test infrastructure only).

Every function cites the passage of the paper it follows. Floating point is
FP64 except where the paper fixes FP32 (the texel-space coordinate of the
Sec. 4.5 listing). Integer work (texel selection) is exact.

Readings taken where the paper is silent (all listed in the design notes):
  * 2D one-tap sampling is separable: one uniform per axis inverts that
    axis' CDF (the bilinear and B-spline 2D weights are products of 1D ones).
  * The sub-texel fraction is quantised to 16 bits; the quantised fraction is
    used consistently for selection, PMFs and the deterministic filter.
  * CDF inversion uses exact integer thresholds ("h at or above a threshold
    selects the next texel"), so selection is exact in any precision.
  * Random numbers come from the pcg4d hash (Jarzynski and Olano 2020) of
    (px, py, frame, seed + (slot >> 1) * 0x9E3779B9); even slots use its
    first two outputs, odd slots the last two.
  * Addressing is WRAP on power-of-two textures; texel identity for the
    estimator is the texel index modulo the texture size.
  * RGBA8/R8 UNORM decode to byte/255 (no sRGB); FP16/FP32 decode exactly.
  * Sharing footprints are defined on tile pixel coordinates (lx, ly) of an
    8x8 screen tile; pixels outside the screen take part in no footprint.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "BILINEAR", "BICUBIC", "FOOTPRINTS", "TILE",
    "texel_float_coord", "split_coord", "axis_weights_int", "axis_weights",
    "weight_denominator", "pcg4d", "slot_hash", "select_axis",
    "footprint_members", "decode_texels", "stf_samples",
    "stf_filter", "stf_filter_reuse", "reference_filter", "stf_adjoint",
    "tiles_to_image", "all_tiles", "psnr",
    "fp8e4m3_value", "bf16_value", "dequantize", "mlp_decode", "decode_latent_texture",
    "texture_values", "selection_slots", "mlp_backward", "stf_adjoint_decoder",
]

BILINEAR = "bilinear"
BICUBIC = "bicubic"
TILE = 8
FOOTPRINTS = ("self", "quad2x2", "wave2x2", "square3x3", "square4x4", "tile8x8", "lut")

_TWO16 = 1 << 16
_TWO32 = 1 << 32
_TWO48 = 1 << 48
_GOLDEN = 0x9E3779B9


# --------------------------------------------------------------------------
# a2: texel-space coordinates and per-axis filter weights
# --------------------------------------------------------------------------

def texel_float_coord(u, size: int) -> np.ndarray:
    """Texel-space coordinate of a texture coordinate, Sec. 4.5 listing:
    texelFloatCoords = uv * txDim - 0.5, evaluated in FP32 as the listing
    does (two roundings, no fused multiply-add).

    Each FP32 operation is formed exactly in FP64 and rounded once to FP32;
    FP64 has more than 2*24+2 bits so the double rounding is innocuous."""
    u64 = np.asarray(u, dtype=np.float32).astype(np.float64)
    prod = (u64 * float(size)).astype(np.float32)           # RN32(u * size)
    return (prod.astype(np.float64) - 0.5).astype(np.float32)  # RN32(. - 0.5)


def split_coord(x) -> tuple[np.ndarray, np.ndarray]:
    """Integer texel index i0 = floor(x) and the 16-bit quantised sub-texel
    fraction F = floor(2^16 (x - i0)), so that the fraction is phi = F / 2^16.
    Exact for FP32 x."""
    xd = np.asarray(x, dtype=np.float32).astype(np.float64)
    i0 = np.floor(xd)
    F = np.floor(xd * 65536.0) - i0 * 65536.0
    return i0.astype(np.int64), F.astype(np.int64)


def weight_denominator(filt: str) -> int:
    """Integer weights are expressed over this common denominator."""
    return _TWO16 if filt == BILINEAR else 6 * _TWO48


def axis_weights_int(F, filt: str) -> np.ndarray:
    """Per-axis filter weights at quantised fraction phi = F/2^16 as exact
    integers over weight_denominator(filt); last axis indexes the texels of
    the support in increasing coordinate order.

    Bilinear (tent): texels i0, i0+1 get 1-phi and phi; this is the per-axis
    factor of GetFilterPMF in Sec. S6, clamp(1 - |x - i|, 0, 1).

    Bicubic B-spline (named in Sec. 5.4): the uniform cubic B-spline kernel
    b(t) = (4 - 6t^2 + 3|t|^3)/6 for |t| <= 1 and (2 - |t|)^3/6 for
    1 <= |t| <= 2, evaluated at the distances 1+phi, phi, 1-phi, 2-phi of
    texels i0-1, i0, i0+1, i0+2; multiplied by 6 * 2^48 these are integers."""
    F = np.asarray(F, dtype=np.int64)
    G = _TWO16 - F
    if filt == BILINEAR:
        return np.stack([G, F], axis=-1)
    if filt != BICUBIC:
        raise ValueError(filt)
    F2 = F * F
    F3 = F2 * F
    w0 = G * G * G
    w1 = 3 * F3 - 6 * F2 * _TWO16 + 4 * _TWO48
    w2 = -3 * F3 + 3 * F2 * _TWO16 + 3 * F * _TWO32 + _TWO48
    w3 = F3
    return np.stack([w0, w1, w2, w3], axis=-1)


def axis_weights(F, filt: str) -> np.ndarray:
    """FP64 per-axis filter weights (the per-axis PMF, Sec. 4.2: for a
    normalised nonnegative filter the PMF equals the weight)."""
    return axis_weights_int(F, filt).astype(np.float64) / float(weight_denominator(filt))


# --------------------------------------------------------------------------
# a3: counter-based hash
# --------------------------------------------------------------------------

def pcg4d(x, y, z, w):
    """pcg4d hash of Jarzynski and Olano, "Hash Functions for GPU Rendering"
    (JCGT 9(3), 2020): an LCG step on each component, a round of cross
    multiplications, a xor-shift by 16 and a second round of cross
    multiplications, all modulo 2^32."""
    m = np.uint32(1664525)
    a = np.uint32(1013904223)
    v = [np.asarray(c, dtype=np.uint32) * m + a for c in (x, y, z, w)]
    x, y, z, w = v
    x = x + y * w
    y = y + z * x
    z = z + x * y
    w = w + y * z
    x = x ^ (x >> np.uint32(16))
    y = y ^ (y >> np.uint32(16))
    z = z ^ (z >> np.uint32(16))
    w = w ^ (w >> np.uint32(16))
    x = x + y * w
    y = y + z * x
    z = z + x * y
    w = w + y * z
    return x, y, z, w


def slot_hash(px, py, slot: int, seed: int, frame: int):
    """Two uniform 32-bit integers (h_x, h_y) for pixel (px, py) and texture
    slot `slot`: pcg4d(px, py, frame, seed + (slot >> 1) * 0x9E3779B9), first
    two outputs for even slots, last two for odd slots."""
    key = (int(seed) + (slot >> 1) * _GOLDEN) % _TWO32
    px = np.asarray(px).astype(np.uint32)
    py = np.asarray(py).astype(np.uint32)
    ones = np.ones_like(px)
    with np.errstate(over="ignore"):
        h = pcg4d(px, py, ones * np.uint32(frame % _TWO32), ones * np.uint32(key))
    return (h[0], h[1]) if slot % 2 == 0 else (h[2], h[3])


# --------------------------------------------------------------------------
# a4: one-tap STF selection (Sec. 2.2 and Sec. S1)
# --------------------------------------------------------------------------

def select_axis(h, wint: np.ndarray, filt: str) -> np.ndarray:
    """Invert one axis' CDF with the uniform integer h in [0, 2^32).

    The offset k is the number of cumulative integer weights C_m (m < n-1)
    that h * (denominator / 2^32) reaches or exceeds. Bilinear: k = 1 iff
    h >= (1-phi) * 2^32, which has probability exactly phi. B-spline: the
    comparison h * 6 * 2^16 >= C_m is between integers below 2^51, so every
    offset is chosen with probability within 2^-32 of its weight."""
    h = np.asarray(h).astype(np.int64)
    if filt == BILINEAR:
        scaled = h                                  # denominator 2^16 -> h * 2^16 / 2^32
        thresholds = [wint[..., 0] * _TWO16]        # compare h >= (1-phi) 2^32
    else:
        scaled = h * (6 * _TWO16)                   # h * (6 * 2^48) / 2^32
        c = np.cumsum(wint, axis=-1)
        thresholds = [c[..., m] for m in range(3)]
    k = np.zeros(np.shape(h), dtype=np.int64)
    for t in thresholds:
        k += (scaled >= t).astype(np.int64)
    return k


# --------------------------------------------------------------------------
# a6: sharing footprints inside an 8x8 tile (Sec. 4.3)
# --------------------------------------------------------------------------

def footprint_members(kind: str, lut: np.ndarray | None = None) -> np.ndarray:
    """Member table [64, K] of row-major tile pixel ids (ly*8+lx) for every
    tile pixel. Every footprint contains the pixel itself (Sec. 4.5: each
    lane is always included in its own footprint).

      self       {c}
      quad2x2    the 2x2 quad with even origin (Sec. 2.3 quads; '2x2q')
      wave2x2    a 2x2 window whose origin is shifted by a per-pixel
                 checker pattern so neighbours differ ('2x2w', Sec. 4.3.1)
      square3x3  3x3 window, origin clamp(l-1, 0, 5) per axis
      square4x4  4x4 window, origin clamp(l-1, 0, 4) per axis
      tile8x8    all 64 pixels of the tile (the whole 64-lane wave)
      lut        caller table [64, K] of ids; entries equal to c are
                 dropped and c itself is always added (so K+1 members)
    Windows keep a constant size at tile edges by shifting inward, so every
    pixel shares with the same number of others (Sec. 4.3 criterion 2)."""
    ids = np.arange(64)
    lx, ly = ids % 8, ids // 8

    def window(ox, oy, n):
        a, b = np.meshgrid(np.arange(n), np.arange(n))
        mx = ox[:, None] + a.reshape(-1)[None, :]
        my = oy[:, None] + b.reshape(-1)[None, :]
        return my * 8 + mx

    if kind == "self":
        return ids[:, None].copy()
    if kind == "quad2x2":
        return window(lx & ~1, ly & ~1, 2)
    if kind == "wave2x2":
        ox = np.clip(lx - ((ly + (lx >> 1)) & 1), 0, 6)
        oy = np.clip(ly - ((lx + (ly >> 1)) & 1), 0, 6)
        return window(ox, oy, 2)
    if kind == "square3x3":
        return window(np.clip(lx - 1, 0, 5), np.clip(ly - 1, 0, 5), 3)
    if kind == "square4x4":
        return window(np.clip(lx - 1, 0, 4), np.clip(ly - 1, 0, 4), 4)
    if kind == "tile8x8":
        return np.tile(ids[None, :], (64, 1))
    if kind == "lut":
        lut = np.asarray(lut, dtype=np.int64) & 63
        rows = []
        for c in range(64):
            rows.append([c] + [int(j) for j in lut[c] if j != c])
        k = max(len(r) for r in rows)
        out = np.full((64, k), -1, dtype=np.int64)
        for c, r in enumerate(rows):
            out[c, : len(r)] = r
        return out
    raise ValueError(kind)


# --------------------------------------------------------------------------
# a1/a5: tiles, texel decode
# --------------------------------------------------------------------------

def all_tiles(width: int, height: int) -> np.ndarray:
    """All (tx, ty) tiles covering a width x height screen."""
    ty, tx = np.mgrid[0:(height + 7) // 8, 0:(width + 7) // 8]
    return np.stack([tx.reshape(-1), ty.reshape(-1)], axis=-1)


def _tile_pixels(tiles: np.ndarray):
    tiles = np.asarray(tiles, dtype=np.int64).reshape(-1, 2)
    ids = np.arange(64)
    px = tiles[:, 0:1] * 8 + (ids % 8)[None, :]
    py = tiles[:, 1:2] * 8 + (ids // 8)[None, :]
    return px, py                                   # [n, 64]


def tiles_to_image(values: np.ndarray, tiles: np.ndarray, width: int, height: int) -> np.ndarray:
    """Scatter per-tile values [n, 64, ...] back into an image [H, W, ...]."""
    px, py = _tile_pixels(tiles)
    img = np.zeros((height, width) + values.shape[2:], dtype=values.dtype)
    m = (px < width) & (py < height)
    img[py[m], px[m]] = values[m]
    return img


def decode_texels(raw: np.ndarray) -> np.ndarray:
    """Texel payload to FP64: UNORM8 -> byte/255, FP16/FP32 exact."""
    raw = np.asarray(raw)
    if raw.dtype == np.uint8:
        return raw.astype(np.float64) / 255.0
    if raw.dtype in (np.float16, np.float32, np.float64):
        return raw.astype(np.float64)
    raise TypeError(raw.dtype)


# --------------------------------------------------------------------------
# reduced-precision payloads and the latent decoder
# --------------------------------------------------------------------------

def fp8e4m3_value(codes) -> np.ndarray:
    """Value of OCP FP8 E4M3 (e4m3fn) codes: 1 sign bit, 4 exponent bits with
    bias 7, 3 mantissa bits; exponent 0 is subnormal (m/8 * 2^-6); the two
    codes S.1111.111 are NaN; there are no infinities (max finite 448)."""
    c = np.asarray(codes).astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = (c & 0x7).astype(np.float64)
    val = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1.0 + m / 8.0) * np.exp2(e.astype(np.float64) - 7.0))
    val = np.where((e == 0xF) & ((c & 0x7) == 0x7), np.nan, val)
    return sign * val


def bf16_value(bits) -> np.ndarray:
    """Value of bfloat16 bit patterns (the upper half of an FP32)."""
    b = np.asarray(bits).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def dequantize(stored: np.ndarray, kind: str, scale) -> np.ndarray:
    """Payload of kind 'unorm8' (bytes) | 'f16' | 'bf16' (uint16 bits) |
    'fp8' (uint8 codes) | 'f32' times its per-channel scale (last axis), in
    FP64."""
    if kind == "unorm8":
        v = np.asarray(stored).astype(np.float64) / 255.0
    elif kind == "f16":
        v = np.asarray(stored).view(np.float16).astype(np.float64) if np.asarray(stored).dtype != np.float16 \
            else np.asarray(stored).astype(np.float64)
    elif kind == "bf16":
        v = bf16_value(stored)
    elif kind == "fp8":
        v = fp8e4m3_value(stored)
    elif kind == "f32":
        v = np.asarray(stored, dtype=np.float64)
    else:
        raise ValueError(kind)
    if scale is None:
        return v
    return v * np.asarray(scale, dtype=np.float64)


def mlp_decode(latent: np.ndarray, layers) -> np.ndarray:
    """The latent decoder MLP in FP64: ReLU(W1 x + b1) -> ReLU(W2 . + b2) ->
    W3 . + b3, weights W_l [out, in] and biases b_l given in FP64 (already
    dequantized). latent [..., in]; returns [..., out]."""
    h = np.asarray(latent, dtype=np.float64)
    for li, (w, b) in enumerate(layers):
        h = h @ np.asarray(w, dtype=np.float64).T + np.asarray(b, dtype=np.float64)
        if li < len(layers) - 1:
            h = np.maximum(h, 0.0)
    return h


def decode_latent_texture(stored, kind, scale, layers) -> np.ndarray:
    """Every texel of a latent grid decoded once: [H, W, 8] -> [H, W, 4] FP64.
    Decoding is per texel, so filtering the decoded texture with one-tap STF,
    reuse or Eq. (3) equals decoding each texel the filter touches (the
    neural-texture setting of Sec. 1 and Sec. 5.6)."""
    return mlp_decode(dequantize(stored, kind, scale), layers)


def texture_values(tex) -> np.ndarray:
    """FP64 texel values [H, W, C] of a texture argument. A plain array is
    decoded by decode_texels; a tuple (stored, kind, scale) is dequantized
    (per-channel scale, None for 1); a tuple (stored, kind, scale, layers) is
    a latent grid decoded per texel by the MLP."""
    if isinstance(tex, tuple):
        if len(tex) == 4:
            return decode_latent_texture(*tex)
        stored, kind, scale = tex
        return dequantize(stored, kind, scale)
    return decode_texels(tex)


def _texture_scale(tex, channels: int) -> np.ndarray:
    """Per-channel factor applied after decoding a stored texel (1 for
    plain arrays and latent grids, whose scale precedes the decoder)."""
    if isinstance(tex, tuple) and len(tex) == 3 and tex[2] is not None:
        return np.asarray(tex[2], dtype=np.float64)
    return np.ones(channels)


# --------------------------------------------------------------------------
# one-tap STF samples for a batch of tiles
# --------------------------------------------------------------------------

def selection_slots(textures, share_selection: bool) -> list:
    """Slot whose random numbers each slot uses: itself, or with shared
    selection (Sec. 4.5: textures of the same UV and resolution may share
    one selection) the first slot of the same texture size."""
    keys = []
    sizes = [texture_values(t).shape[:2] for t in textures] if share_selection else None
    for i in range(len(textures)):
        k = i
        if share_selection:
            k = next(j for j in range(i + 1) if sizes[j] == sizes[i])
        keys.append(k)
    return keys


def stf_samples(tex: np.ndarray, uv: np.ndarray, tiles: np.ndarray, slot: int,
                filt: str, seed: int, frame: int) -> dict:
    """Per pixel of each tile: own coordinate split, own per-axis weights,
    the one-tap STF sample (integer texel coordinates, PMF p, texel value).

    Sec. 4.5: each lane first samples a single texel according to its own
    filter, exactly as one-tap STF does (Sec. 2.2; Sec. S1 shows the
    importance-sampling estimator then returns the texel unweighted)."""
    H, W = uv.shape[:2]
    values = texture_values(tex)
    th, tw = values.shape[:2]
    px, py = _tile_pixels(tiles)
    valid = (px < W) & (py < H)
    pxc = np.minimum(px, W - 1)
    pyc = np.minimum(py, H - 1)
    u = uv[pyc, pxc, 0]
    v = uv[pyc, pxc, 1]
    x = texel_float_coord(u, tw)
    y = texel_float_coord(v, th)
    i0x, Fx = split_coord(x)
    i0y, Fy = split_coord(y)
    wix = axis_weights_int(Fx, filt)
    wiy = axis_weights_int(Fy, filt)
    hx, hy = slot_hash(px, py, slot, seed, frame)
    kx = select_axis(hx, wix, filt)
    ky = select_axis(hy, wiy, filt)
    delta = 1 if filt == BICUBIC else 0
    sx = np.mod(i0x - delta + kx, tw)               # WRAP: canonical texel index
    sy = np.mod(i0y - delta + ky, th)
    wx = axis_weights(Fx, filt)
    wy = axis_weights(Fy, filt)
    p = np.take_along_axis(wx, kx[..., None], -1)[..., 0] * np.take_along_axis(wy, ky[..., None], -1)[..., 0]
    T = values[sy, sx]
    return dict(valid=valid, px=px, py=py, i0x=i0x, i0y=i0y, Fx=Fx, Fy=Fy, wx=wx, wy=wy,
                kx=kx, ky=ky, sx=sx, sy=sy, p=p, T=T, delta=delta, tw=tw, th=th)


def stf_filter(textures, uv, filt, seed, frame, tiles=None, share_selection=False):
    """One-tap STF (Sec. 2.2): each pixel returns its one sampled texel.
    Returns per slot (values [n, 64, C], selections [n, 64, 2] as (x, y))."""
    if tiles is None:
        tiles = all_tiles(uv.shape[1], uv.shape[0])
    keys = selection_slots(textures, share_selection)
    out = []
    for slot, tex in enumerate(textures):
        s = stf_samples(tex, uv, tiles, keys[slot], filt, seed, frame)
        out.append((s["T"], np.stack([s["sx"], s["sy"]], -1)))
    return out


# --------------------------------------------------------------------------
# a6/a7: sharing + weighted importance sampling, Eq. (14)
# --------------------------------------------------------------------------

def _own_weight_at(s: dict, sx_i: np.ndarray, sy_i: np.ndarray):
    """Pixel c's filter weight f_c at texel (sx_i, sy_i) (Sec. S6
    GetFilterPMF for bilinear; the B-spline analogue for bicubic), and
    whether that texel lies in c's support. Texel identity is taken modulo
    the texture size (WRAP)."""
    n = s["wx"].shape[-1]
    dx = np.mod(sx_i - (s["i0x"] - s["delta"]), s["tw"])
    dy = np.mod(sy_i - (s["i0y"] - s["delta"]), s["th"])
    inside = (dx < n) & (dy < n)
    dxc = np.minimum(dx, n - 1)
    dyc = np.minimum(dy, n - 1)
    f = np.take_along_axis(s["wx"], dxc[..., None], -1)[..., 0] * \
        np.take_along_axis(s["wy"], dyc[..., None], -1)[..., 0]
    return np.where(inside, f, 0.0), inside


def stf_filter_reuse(textures, uv, filt, seed, frame, footprint, lut=None, tiles=None, exact_filtering=False,
                     share_selection=False):
    """STF with sample reuse (Sec. 4), per slot.

    Pixel c combines the samples of the members i of its sharing footprint
    S(c) with the estimator of Eq. (14):
        out_c = sum_i w_i T_i / sum_j w_j,  w_i = f_c(x_i) / f_i(x_i),
    where x_i is the texel lane i sampled with its own PMF p_i = f_i
    (Sec. 4.2: for a normalised nonnegative filter p = f). A sample outside
    c's support has w_i = 0 and is skipped, never multiplied (Sec. 4.5), so
    the own sample (w_c = 1) always remains and with no useful neighbour the
    result is the one-tap STF value.

    exact_filtering (Sec. 4.2, "Exact Filtering"): when the samples of c's
    footprint include every texel of positive weight in c's own filter
    support, c returns the deterministic filter value of Eq. (3) instead.

    Returns per slot (values [n, 64, C], selections [n, 64, 2])."""
    if tiles is None:
        tiles = all_tiles(uv.shape[1], uv.shape[0])
    members = footprint_members(footprint, lut)
    keys = selection_slots(textures, share_selection)
    out = []
    for slot, tex in enumerate(textures):
        s = stf_samples(tex, uv, tiles, keys[slot], filt, seed, frame)
        C = s["T"].shape[-1]
        n_sup = s["wx"].shape[-1]
        seen = np.zeros(s["p"].shape + (n_sup, n_sup), dtype=bool)      # [tile, pixel, dy, dx]
        num = np.zeros(s["T"].shape, dtype=np.float64)
        den = np.zeros(s["p"].shape, dtype=np.float64)
        for k in range(members.shape[1]):
            j = members[:, k]                       # [64] member id per tile pixel
            present = (j >= 0)[None, :]
            jj = np.maximum(j, 0)
            sx_i = s["sx"][:, jj]
            sy_i = s["sy"][:, jj]
            p_i = s["p"][:, jj]
            T_i = s["T"][:, jj]
            use = present & s["valid"][:, jj] & s["valid"]
            f_c, inside = _own_weight_at(s, sx_i, sy_i)
            use = use & inside
            w = np.where(use, f_c / np.where(use, p_i, 1.0), 0.0)
            den += w
            num += np.where(use[..., None], w[..., None] * np.where(use[..., None], T_i, 0.0), 0.0)
            if exact_filtering:
                dx = np.mod(sx_i - (s["i0x"] - s["delta"]), s["tw"])
                dy = np.mod(sy_i - (s["i0y"] - s["delta"]), s["th"])
                t_i, p_i2 = np.nonzero(use)
                seen[t_i, p_i2, dy[t_i, p_i2], dx[t_i, p_i2]] = True
        with np.errstate(invalid="ignore", divide="ignore"):
            val = num / den[..., None]
        if exact_filtering:
            positive = (s["wy"][..., :, None] * s["wx"][..., None, :]) > 0          # [tile, pixel, dy, dx]
            covered = np.all(seen | ~positive, axis=(-2, -1))
            values = texture_values(tex)
            exact = np.zeros(s["T"].shape)
            for b in range(n_sup):
                yy = np.mod(s["i0y"] - s["delta"] + b, s["th"])
                for a in range(n_sup):
                    xx = np.mod(s["i0x"] - s["delta"] + a, s["tw"])
                    exact += (s["wx"][..., a] * s["wy"][..., b])[..., None] * values[yy, xx]
            val = np.where(covered[..., None], exact, val)
        val = np.where(s["valid"][..., None], val, 0.0)
        assert C == val.shape[-1]
        out.append((val, np.stack([s["sx"], s["sy"]], -1)))
    return out


# --------------------------------------------------------------------------
# ground truth, Eq. (3)
# --------------------------------------------------------------------------

def reference_filter(textures, uv, filt, tiles=None):
    """Deterministic filtered value, Eq. (3): t_r(u,v) = sum_i f_r(u-u_i,
    v-v_i) T_i over the filter support, with the same coordinates and
    quantised weights as the stochastic paths. Per slot [n, 64, C]."""
    if tiles is None:
        tiles = all_tiles(uv.shape[1], uv.shape[0])
    out = []
    for tex in textures:
        s = stf_samples(tex, uv, tiles, 0, filt, 0, 0)
        T = texture_values(tex)
        n = s["wx"].shape[-1]
        acc = np.zeros(s["T"].shape, dtype=np.float64)
        for b in range(n):
            yy = np.mod(s["i0y"] - s["delta"] + b, s["th"])
            for a in range(n):
                xx = np.mod(s["i0x"] - s["delta"] + a, s["tw"])
                acc += (s["wx"][..., a] * s["wy"][..., b])[..., None] * T[yy, xx]
        out.append(np.where(s["valid"][..., None], acc, 0.0))
    return out


# --------------------------------------------------------------------------
# adjoint of Eq. (14) with respect to the texels
# --------------------------------------------------------------------------

def stf_adjoint(textures, uv, filt, seed, frame, footprint, grads, lut=None, tiles=None, share_selection=False):
    """Gradient of L with respect to every texel, given dL/dout per pixel.

    The weights of Eq. (14) depend only on positions and random numbers, so
    out_c = sum_i a_ci T[x_i] with a_ci = w_i / sum_j w_j is linear in the
    texels and dL/dT[x] = sum_c sum_{i in S(c), x_i = x} a_ci dL/dout_c.
    grads: per slot [n, 64, C] (tile layout). Returns per slot [H_t, W_t, C],
    the gradient with respect to the texel before its per-channel scale
    (out is linear in it, with the scale as factor)."""
    if tiles is None:
        tiles = all_tiles(uv.shape[1], uv.shape[0])
    members = footprint_members(footprint, lut)
    keys = selection_slots(textures, share_selection)
    res = []
    for slot, (tex, g) in enumerate(zip(textures, grads)):
        s = stf_samples(tex, uv, tiles, keys[slot], filt, seed, frame)
        C = s["T"].shape[-1]
        ws, ids = [], []
        den = np.zeros(s["p"].shape)
        for k in range(members.shape[1]):
            j = members[:, k]
            jj = np.maximum(j, 0)
            use = (j >= 0)[None, :] & s["valid"][:, jj] & s["valid"]
            f_c, inside = _own_weight_at(s, s["sx"][:, jj], s["sy"][:, jj])
            use = use & inside
            w = np.where(use, f_c / np.where(use, s["p"][:, jj], 1.0), 0.0)
            den += w
            ws.append(w)
            ids.append(jj)
        grad = np.zeros((s["th"], s["tw"], C))
        gg = np.asarray(g, dtype=np.float64).reshape(s["T"].shape) * _texture_scale(tex, C)
        for w, jj in zip(ws, ids):
            a = np.where(den > 0, w / np.where(den > 0, den, 1.0), 0.0)
            contrib = a[..., None] * gg
            np.add.at(grad, (s["sy"][:, jj].reshape(-1), s["sx"][:, jj].reshape(-1)),
                      contrib.reshape(-1, C))
        res.append(grad)
    return res


# --------------------------------------------------------------------------
# adjoint through the latent decoder (the neural-texture setting)
# --------------------------------------------------------------------------

def mlp_backward(latent: np.ndarray, layers, g: np.ndarray):
    """Reverse-mode derivative of mlp_decode at n latents [n, in] for output
    gradients g [n, out], in FP64. Returns dL/dlatent [n, in] and, per layer,
    (dL/dW_l [out, in], dL/db_l [out]) summed over the n latents. The ReLU
    passes the gradient where its input is > 0 and blocks it elsewhere."""
    ws = [np.asarray(w, dtype=np.float64) for w, _ in layers]
    bs = [np.asarray(b, dtype=np.float64) for _, b in layers]
    acts = [np.asarray(latent, dtype=np.float64)]   # the input of each layer
    pre = []
    for li, (w, b) in enumerate(zip(ws, bs)):
        z = acts[-1] @ w.T + b
        pre.append(z)
        acts.append(np.maximum(z, 0.0) if li < len(ws) - 1 else z)
    d = np.asarray(g, dtype=np.float64)
    grads = [None] * len(ws)
    for li in reversed(range(len(ws))):
        if li < len(ws) - 1:
            d = d * (pre[li] > 0.0)
        grads[li] = (d.T @ acts[li], d.sum(axis=0))
        d = d @ ws[li]
    return d, grads


def stf_adjoint_decoder(textures, uv, filt, seed, frame, footprint, grads, lut=None, tiles=None,
                        share_selection=False):
    """Gradients of L through Eq. (14) and the latent decoder, given dL/dout
    per pixel, for latent textures (stored, kind, scale, layers) that share
    one decoder.

    The weights of Eq. (14) do not depend on the texel values, so the
    gradient with respect to each decoded texel is the texel adjoint
    (stf_adjoint); each texel's decode is independent, so the chain rule then
    runs through the decoder once per texel: dL/dlatent_x = J_x^T g_x, and
    the decoder's weight gradients sum over the texels. Returns (per slot
    dL/dstored latent [H_t, W_t, 8], the gradient with respect to the stored
    value before its per-channel scale; per layer (dL/dW_l, dL/db_l) summed
    over the slots)."""
    layers = textures[0][3]
    for t in textures:
        if not (isinstance(t, tuple) and len(t) == 4):
            raise ValueError("latent textures (stored, kind, scale, layers) expected")
        if t[3] is not layers:
            raise ValueError("every latent texture of a call shares one decoder")
    g_tex = stf_adjoint(textures, uv, filt, seed, frame, footprint, grads, lut=lut, tiles=tiles,
                        share_selection=share_selection)
    dlat = []
    total = [(np.zeros(np.shape(w)), np.zeros(np.shape(b))) for w, b in layers]
    for (stored, kind, scale, _), g in zip(textures, g_tex):
        lat = dequantize(stored, kind, scale)                  # [H_t, W_t, 8]
        hit = np.any(g != 0.0, axis=-1)
        d = np.zeros(lat.shape)
        if np.any(hit):
            dl, lg = mlp_backward(lat[hit], layers, g[hit])
            sc = np.ones(lat.shape[-1]) if scale is None else np.asarray(scale, dtype=np.float64)
            d[hit] = dl * sc                                   # latent = stored * scale
            total = [(tw + gw, tb + gb) for (tw, tb), (gw, gb) in zip(total, lg)]
        dlat.append(d)
    return dlat, total


# --------------------------------------------------------------------------
# metric
# --------------------------------------------------------------------------

def psnr(test: np.ndarray, ref: np.ndarray, peak: float = 1.0) -> float:
    """PSNR in dB over all pixels and channels in linear space (Sec. 5.1
    computes PSNR in linear RGB), FP64 host reduction."""
    d = np.asarray(test, np.float64) - np.asarray(ref, np.float64)
    mse = float(np.mean(d * d))
    if mse == 0.0:
        return float("inf")
    return 10.0 * np.log10(peak * peak / mse)
