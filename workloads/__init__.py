"""Seeded synthetic inputs for stochastic texture filtering workloads.

This module generates textures and screen-space UV buffers only. It holds none
of the filtering method's arithmetic (no coordinates, weights, hashing,
selection or estimators): the CPU oracle and the GPU path both receive what is
generated here as plain arrays.

The paper evaluates on material texture sets and scenes that are not available
here; the procedural stand-ins imitate what the paper says about texture
content (large flat / low-frequency regions plus high-contrast edges, Sec. 3)
and the magnification regime it targets (Sec. 5.1 zoom sweep, Sec. 5.6).

Workloads:
  * small:  256x256 RGBA8 value noise + hard-edged checkerboard, 512x512
            fronto-parallel quad at uniform 8x magnification.
  * plane:  2048x2048 RGBA16F multi-octave noise + sharp edges, RG16F normal
            map, 1920x1080 perspective ground plane spanning 2x..32x
            magnification with analytic UV derivatives.
  * four-texture 4K, latent-grid and view-set variants for the extensions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "value_noise", "small_texture", "small_screen", "plane_albedo", "plane_normal",
    "PlaneCamera", "perspective_plane", "tile_texture_rgba8", "r8_texture",
    "latent_grid", "mlp_weights", "view_set", "halton", "material_set", "frame_jitter",
]


# ----------------------------------------------------------------------------
# procedural texture content
# ----------------------------------------------------------------------------

def _smoothstep(t: np.ndarray) -> np.ndarray:
    return t * t * (3.0 - 2.0 * t)


def value_noise(rng: np.random.Generator, size: int, period: int, channels: int) -> np.ndarray:
    """Tileable value noise: random lattice values every `period` texels,
    smoothstep-interpolated. Returns float64 [size, size, channels] in [0, 1]."""
    period = min(period, size)
    assert size % period == 0
    n = size // period
    lat = rng.random((n, n, channels))
    c = (np.arange(size, dtype=np.float64) + 0.5) / period - 0.5
    i0 = np.floor(c).astype(np.int64)
    t = _smoothstep(c - i0)
    a = np.mod(i0, n)
    b = np.mod(i0 + 1, n)
    # rows (y) then columns (x)
    ty = t[:, None, None]
    tx = t[None, :, None]
    v00 = lat[a][:, a]
    v01 = lat[a][:, b]
    v10 = lat[b][:, a]
    v11 = lat[b][:, b]
    top = v00 * (1 - tx) + v01 * tx
    bot = v10 * (1 - tx) + v11 * tx
    return top * (1 - ty) + bot * ty


def small_texture(seed: int = 0, size: int = 256) -> np.ndarray:
    """256x256 RGBA8: 0.5 x value noise (lattice every 8 texels) + 0.5 x a
    checkerboard of 16-texel squares with random per-square colours."""
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = value_noise(rng, size, 8, 4)
    nsq = size // 16
    colours = rng.random((nsq, nsq, 4))
    sq = np.arange(size) // 16
    checker = colours[sq][:, sq]
    tex = 0.5 * noise + 0.5 * checker
    return np.ascontiguousarray(np.clip(np.rint(tex * 255.0), 0, 255).astype(np.uint8))


def small_screen(width: int = 512, height: int = 512, tex_size: int = 256, mag: float = 8.0,
                 offset_seed: int | None = None) -> np.ndarray:
    """Fronto-parallel quad at uniform magnification `mag`: pixel centre
    (px+1/2, py+1/2) maps to texel-space position (px+1/2)/mag (+ optional
    seeded sub-texel offset). Returns FP32 UV [height, width, 2]."""
    off = np.zeros(2)
    if offset_seed is not None:
        off = np.random.Generator(np.random.PCG64(offset_seed)).random(2)
    px = (np.arange(width, dtype=np.float64) + 0.5) / mag + off[0]
    py = (np.arange(height, dtype=np.float64) + 0.5) / mag + off[1]
    uv = np.empty((height, width, 2), np.float64)
    uv[..., 0] = px[None, :] / tex_size
    uv[..., 1] = py[:, None] / tex_size
    return uv.astype(np.float32)


def _edge_field(rng: np.random.Generator, size: int, n_lines: int = 12, checker: int = 32,
                max_freq: int = 24) -> np.ndarray:
    """Binary field with sharp edges: a rotated checkerboard XOR random
    half-planes (all periodic over the texture so it tiles)."""
    y, x = np.mgrid[0:size, 0:size].astype(np.float64)
    ang = rng.random() * math.pi
    ca, sa = math.cos(ang), math.sin(ang)
    # periodic rotated checker: use integer frequencies so it wraps seamlessly
    kx = max(1, int(round(size / checker * ca)))
    ky = max(1, int(round(size / checker * sa)))
    phase = np.sin(2 * math.pi * (kx * x + ky * y) / size) * np.sin(2 * math.pi * (-ky * x + kx * y) / size)
    field_ = phase > 0
    for _ in range(n_lines):
        fx, fy = rng.integers(-max_freq, max_freq + 1, 2)
        if fx == 0 and fy == 0:
            fx = 1
        ph = rng.random()
        field_ ^= np.sin(2 * math.pi * ((fx * x + fy * y) / size + ph)) > 0.6
    return field_.astype(np.float64)


_PLANE_CACHE: dict = {}


def _plane_content(seed: int, size: int):
    key = (seed, size)
    if key not in _PLANE_CACHE:
        rng = np.random.Generator(np.random.PCG64(seed))
        noise = np.zeros((size, size, 4))
        amp_sum = 0.0
        for o in range(5):
            period = max(2, 64 >> o)
            amp = 0.5 ** o
            noise += amp * value_noise(rng, size, period, 4)
            amp_sum += amp
        noise /= amp_sum
        edges = _edge_field(rng, size)
        tint_a = rng.random(4) * 0.3
        tint_b = 0.6 + rng.random(4) * 0.4
        albedo = 0.4 * noise + 0.6 * (tint_a + (tint_b - tint_a) * edges[..., None])
        albedo = np.clip(albedo, 0.0, 1.0)
        height = 0.7 * noise[..., 0] + 0.3 * edges
        _PLANE_CACHE.clear()
        _PLANE_CACHE[key] = (albedo, height)
    return _PLANE_CACHE[key]


def plane_albedo(seed: int = 0, size: int = 2048, dtype=np.float16) -> np.ndarray:
    """RGBA16F albedo: 5-octave value noise (base period 64 texels, gain 1/2)
    mixed with a sharp-edged binary field (edge contrast >= 0.5 per channel
    on average). Values in [0, 1], rounded to FP16 (or to `dtype`)."""
    albedo, _ = _plane_content(seed, size)
    return albedo.astype(dtype)


def plane_normal(seed: int = 0, size: int = 2048, strength: float = 8.0) -> np.ndarray:
    """RG16F tangent-space normal XY from the gradient of the same height
    field (periodic central differences), clamped to [-1, 1]."""
    _, h = _plane_content(seed, size)
    dx = (np.roll(h, -1, axis=1) - np.roll(h, 1, axis=1)) * 0.5
    dy = (np.roll(h, -1, axis=0) - np.roll(h, 1, axis=0)) * 0.5
    n = np.stack([-dx * strength, -dy * strength], axis=-1)
    return np.clip(n, -1.0, 1.0).astype(np.float16)


def tile_texture_rgba8(seed: int, size: int) -> np.ndarray:
    """RGBA8 texture with the same recipe as plane_albedo (UNORM8)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = np.zeros((size, size, 4))
    for o in range(4):
        noise += 0.5 ** o * value_noise(rng, size, max(2, 32 >> o), 4)
    noise /= sum(0.5 ** o for o in range(4))
    edges = _edge_field(rng, size, n_lines=8, checker=max(8, size // 16))
    tex = np.clip(0.4 * noise + 0.6 * edges[..., None] * rng.random(4), 0, 1)
    return np.clip(np.rint(tex * 255), 0, 255).astype(np.uint8)


def r8_texture(seed: int, size: int) -> np.ndarray:
    """Single-channel UNORM8 texture (roughness / mask)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = value_noise(rng, size, max(2, size // 32), 1)
    edges = _edge_field(rng, size, n_lines=6, checker=max(8, size // 8))
    tex = np.clip(0.5 * noise[..., 0] + 0.5 * edges, 0, 1)
    return np.clip(np.rint(tex * 255), 0, 255).astype(np.uint8)[..., None]


# ----------------------------------------------------------------------------
# perspective ground plane with analytic UV derivatives
# ----------------------------------------------------------------------------

@dataclass
class PlaneCamera:
    """Pinhole camera at height 1 above the plane y=0, pitched down by
    `pitch` radians; vertical field of view `fov_y`; the bottom screen row
    looks straight down when fov_y/2 = pi/2 - pitch."""
    width: int
    height: int
    pitch: float
    fov_y: float
    tile_len: float = 1.0          # world units per UV unit
    uv_offset: tuple = (0.25, 0.1)
    jitter: tuple = (0.0, 0.0)     # sub-pixel offset of the sample position
    info: dict = field(default_factory=dict)

    def rays(self, cols=None, rows=None):
        W, H = self.width, self.height
        cols = np.arange(W) if cols is None else np.asarray(cols)
        rows = np.arange(H) if rows is None else np.asarray(rows)
        px = cols.astype(np.float64) + 0.5 + self.jitter[0]
        py = rows.astype(np.float64) + 0.5 + self.jitter[1]
        sx = (px / W) * 2.0 - 1.0
        sy = 1.0 - (py / H) * 2.0
        return np.meshgrid(sx, sy)

    def evaluate(self, cols=None, rows=None):
        """Returns (uv, duv_dpx, duv_dpy) in float64, each [rows, cols, 2]
        (all pixels by default)."""
        sx, sy = self.rays(cols, rows)
        ty = math.tan(self.fov_y / 2)
        tx = ty * self.width / self.height
        cp, sp = math.cos(self.pitch), math.sin(self.pitch)
        dx = sx * tx
        dy = -sp + sy * ty * cp
        dz = cp + sy * ty * sp
        assert np.all(dy < 0), "horizon must lie above the screen"
        t = -1.0 / dy
        X = t * dx
        Z = t * dz
        dt_dsy = ty * cp / (dy * dy)
        dX_dsx = t * tx
        dX_dsy = dx * dt_dsy
        dZ_dsy = dt_dsy * dz + t * ty * sp
        L = self.tile_len
        u = X / L + self.uv_offset[0]
        v = Z / L + self.uv_offset[1]
        dsx_dpx = 2.0 / self.width
        dsy_dpy = -2.0 / self.height
        du_dpx = dX_dsx * dsx_dpx / L
        dv_dpx = np.zeros_like(du_dpx)
        du_dpy = dX_dsy * dsy_dpy / L
        dv_dpy = dZ_dsy * dsy_dpy / L
        uv = np.stack([u, v], -1)
        return uv, np.stack([du_dpx, dv_dpx], -1), np.stack([du_dpy, dv_dpy], -1)


def magnification(duv_dpx: np.ndarray, duv_dpy: np.ndarray, tex_size: int):
    """Per-pixel magnification along the least- and most-magnified screen
    axes: 1 / (tex_size * sigma_max(J)) and 1 / (tex_size * sigma_min(J))."""
    a = duv_dpx[..., 0]; c = duv_dpx[..., 1]
    b = duv_dpy[..., 0]; d = duv_dpy[..., 1]
    # singular values of [[a, b], [c, d]]
    s1 = a * a + b * b + c * c + d * d
    det = np.abs(a * d - b * c)
    disc = np.sqrt(np.maximum(s1 * s1 - 4 * det * det, 0))
    smax = np.sqrt((s1 + disc) / 2)
    smin = np.sqrt(np.maximum((s1 - disc) / 2, 0))
    return 1.0 / (tex_size * smax), 1.0 / (tex_size * np.maximum(smin, 1e-30))


def perspective_plane(width: int = 1920, height: int = 1080, tex_size: int = 2048,
                      mag_min: float = 2.0, mag_max: float = 32.0,
                      jitter: tuple = (0.0, 0.0), uv_offset: tuple = (0.25, 0.1)):
    """Perspective ground plane whose least-magnified axis spans
    [mag_min, mag_max] over the screen.

    The bottom row looks straight down (grazing angle 90 deg); the pitch is
    solved so that the ratio of largest to smallest min-axis magnification is
    mag_max/mag_min, then the UV scale is set so the minimum is mag_min.
    Returns (uv FP32 [H,W,2], duv_dpx, duv_dpy float64, info dict)."""
    # the extremes sit on the screen border and the centre column: a sparse
    # grid that contains them is enough to solve for the geometry
    cols = np.unique(np.r_[np.arange(0, width, 16), width - 1, width // 2 - 1, width // 2])
    rows = np.unique(np.r_[np.arange(0, height, 16), height - 1])

    def ratio(pitch):
        cam = PlaneCamera(width, height, pitch, 2 * (math.pi / 2 - pitch))
        _, jx, jy = cam.evaluate(cols, rows)
        mmin, _ = magnification(jx, jy, 1)
        return mmin.max() / mmin.min()

    target = mag_max / mag_min
    lo, hi = math.radians(46.0), math.radians(75.0)   # ratio decreases with pitch
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if ratio(mid) > target:
            lo = mid
        else:
            hi = mid
    pitch = 0.5 * (lo + hi)
    cam = PlaneCamera(width, height, pitch, 2 * (math.pi / 2 - pitch))
    _, jx, jy = cam.evaluate(cols, rows)
    mmin, _ = magnification(jx, jy, tex_size)
    scale = mag_min / mmin.min()          # magnification is proportional to tile_len
    cam = PlaneCamera(width, height, pitch, 2 * (math.pi / 2 - pitch), tile_len=scale,
                      uv_offset=uv_offset, jitter=jitter)
    uv, jx, jy = cam.evaluate()
    mmin, mmaj = magnification(jx, jy, tex_size)
    info = dict(pitch_deg=math.degrees(pitch), fov_y_deg=math.degrees(cam.fov_y), tile_len=scale,
                mag_min_axis=(float(mmin.min()), float(mmin.max())),
                anisotropy_max=float((mmaj / mmin).max()),
                texel_extent=float(np.abs(uv * tex_size).max()))
    return uv.astype(np.float32), jx, jy, info


# ----------------------------------------------------------------------------
# extension workloads: latent grid + decoder weights, view sets
# ----------------------------------------------------------------------------

def latent_grid(seed: int = 0, size: int = 1024, channels: int = 8) -> np.ndarray:
    """Float32 latent grid [size, size, channels]: smooth noise in [-1, 1]
    with edges, standing in for a trained neural-texture latent grid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lat = np.zeros((size, size, channels))
    for o in range(3):
        lat += 0.5 ** o * value_noise(rng, size, max(2, 32 >> o), channels)
    lat = lat / sum(0.5 ** o for o in range(3)) * 2.0 - 1.0
    edges = _edge_field(rng, size, n_lines=6, checker=max(8, size // 8))
    lat[..., : channels // 2] += 0.5 * (edges[..., None] - 0.5)
    return lat.astype(np.float32)


def mlp_weights(seed: int = 0, dims=(8, 64, 64, 4)):
    """He-initialised decoder weights [(W_l [out,in], b_l [out])] in float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    layers = []
    for din, dout in zip(dims[:-1], dims[1:]):
        w = rng.standard_normal((dout, din)) * math.sqrt(2.0 / din)
        b = rng.standard_normal(dout) * 0.05
        layers.append((w.astype(np.float32), b.astype(np.float32)))
    return layers


def view_set(n_views: int = 8, width: int = 1920, height: int = 1080, tex_size: int = 1024, seed: int = 0):
    """`n_views` perspective-plane views with seeded UV offsets and sub-pixel
    jitter (for texture optimisation from several views)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    views = []
    for _ in range(n_views):
        off = tuple(rng.random(2))
        jit = tuple(rng.random(2) - 0.5)
        uv, _, _, _ = perspective_plane(width, height, tex_size, 2.0, 16.0, jitter=jit, uv_offset=off)
        views.append(uv)
    return views


# ----------------------------------------------------------------------------
# four-texture 4K material workload
# ----------------------------------------------------------------------------

def halton(i: int, base: int) -> float:
    """i-th element (1-based) of the radical-inverse Halton sequence."""
    f, r = 1.0, 0.0
    while i > 0:
        f /= base
        r += f * (i % base)
        i //= base
    return r


def frame_jitter(frame: int) -> tuple:
    """Sub-pixel jitter of frame `frame`: Halton(2, 3) point minus 1/2."""
    return (halton(frame + 1, 2) - 0.5, halton(frame + 1, 3) - 0.5)


def material_set(seed: int = 0):
    """Four material textures sharing one UV set: albedo RGBA8 2048^2,
    normal RG16F 2048^2, roughness R8 1024^2, mask R8 512^2."""
    return [tile_texture_rgba8(seed, 2048), plane_normal(seed, 2048), r8_texture(seed + 1, 1024),
            r8_texture(seed + 2, 512)]


# ----------------------------------------------------------------------------
# reduced-precision payloads (inputs for the precision tests and benches)
# ----------------------------------------------------------------------------

def amax_scale(values: np.ndarray, kind: str) -> np.ndarray:
    """Per-channel scale that maps each channel's largest magnitude to the
    largest finite value of the format (448 for FP8 E4M3, 1 for BF16/FP16
    payloads, which keep their range)."""
    amax = np.abs(values.reshape(-1, values.shape[-1])).max(axis=0)
    top = {"fp8": 448.0}.get(kind, None)
    if top is None:
        return np.ones(values.shape[-1])
    return np.where(amax > 0, amax / top, 1.0).astype(np.float32).astype(np.float64)


def quantize(values: np.ndarray, kind: str, scale=None) -> np.ndarray:
    """Stored payload of values / scale in format `kind` (round to nearest
    even via torch's CPU casts): 'bf16' -> uint16 bits, 'fp8' -> uint8 E4M3
    codes, 'f16' -> float16."""
    import torch
    v = np.asarray(values, dtype=np.float64)
    if scale is not None:
        v = v / np.asarray(scale, dtype=np.float64)
    t = torch.from_numpy(np.ascontiguousarray(v.astype(np.float32)))
    if kind == "bf16":
        return t.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    if kind == "fp8":
        return t.to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    if kind == "f16":
        return t.to(torch.float16).numpy()
    raise ValueError(kind)


def bf16_representable(values: np.ndarray) -> np.ndarray:
    """values rounded to the nearest BF16 number, as float32."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(values, dtype=np.float32)))
    return t.to(torch.bfloat16).to(torch.float32).numpy()


def decoder_weights(seed: int = 0):
    """Decoder MLP 8 -> 64 -> 64 -> 4 (He-initialised) whose W1, b1, W2, W3 are
    BF16 numbers (the matrix cores take them exactly) and b2, b3 float32."""
    (w1, b1), (w2, b2), (w3, b3) = mlp_weights(seed)
    r = bf16_representable
    return [(r(w1), r(b1)), (r(w2), b2), (r(w3), b3)]
