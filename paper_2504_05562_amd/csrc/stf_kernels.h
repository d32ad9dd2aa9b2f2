// Kernels of the STF library (device code and forward launches), shared by
// the translation units of libstf.so.
//
// One wavefront processes one 8x8 screen tile at a time (the decoder
// kernels two tile rows, one after the other); a 256-thread workgroup holds
// four tiles side by side (32x8 pixels), so every UV row segment a group
// reads is 256 contiguous bytes. Per pixel and texture slot a kernel:
//   1. loads UV once (shared by all slots),
//   2. splits the texel-space coordinate and forms per-axis weights,
//   3. draws two uniforms from the pcg4d hash and picks one texel per axis
//      by exact integer CDF inversion (one-tap STF),
//   4. fetches and decodes that single texel,
//   5. (reuse) exchanges picks inside the tile and evaluates Eq. (14): the
//      pair and record exchanges in the difference form
//      out = T_c + sum_i w_i (T_i - T_c) / sum_i w_i (exact for constant
//      regions and the no-overlap fallback in FP32), the whole-tile bins as
//      sum_j f_c(j) N_j T_j / sum_j f_c(j) N_j (one FMA per channel and bin;
//      a wave whose picks all hold the same texel returns it exactly),
//   6. stores FP32 colours with non-temporal stores.
// Exchange strategies:
//   quad2x2  DPP quad_perm moves, no LDS;
//   tile8x8  texel bins in LDS: every lane adds its 1/p to the bin of its
//            texel (N_j = sum over picks of texel j of 1/p_i), then each
//            pixel visits only the N x N bins of its own support:
//            sum_i w_i T_i = sum_j f_c(j) N_j T_j;
//   others   per-lane records in LDS read through the footprint member
//            table (windows computed, or the caller's LUT).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>

#include "stf_device.h"
#include "stf_decoder.h"

namespace stf {

enum Mode { kModeStf = 0, kModeQuad = 1, kModeRecords = 2, kModeBins = 3 };

// f(std::integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time.
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// LDS per wavefront: bins (kBinRecords x 16 B records, or kBinRecords floats
// of N plus kBinRecords x 16 B of decoded texels) followed by kBinRecords
// 64-bit fixed-point accumulators, or records (64 x {s, r} + 64 x 16 B).
// Tables of at most kLutStageMax entries per pixel are staged in LDS.
constexpr int kLutStageMax = 16;
constexpr int kAccFloatOffset = kBinRecords * 5;
constexpr int kLdsFloatsPerWave = kAccFloatOffset + kBinRecords * 2;
static_assert(kLdsFloatsPerWave % 4 == 0, "16-byte aligned LDS records");

struct Pixel {
    int px, py;          // screen pixel
    int lx, ly;          // pixel inside the tile
    int q;               // row-major tile pixel id ly*8+lx
    bool valid;          // inside the screen
    float u, v;
};

// Per-pixel selection state for one texture size: both axes plus the
// products of their weights (the 2D filter weights f_c over the support).
template <int FILT>
struct SelCtx {
    static constexpr int N = AxisCtx<FILT>::N;
    AxisCtx<FILT> x, y;
    float wxy[N * N];
    int tw = 0, th = 0;
    __device__ __forceinline__ void update(const Pixel& P, int w, int h) {
        if (w == tw && h == th) return;                  // wave-uniform
        if (w != tw) x.init(P.u, w);
        if (h != th) y.init(P.v, h);
        tw = w;
        th = h;
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int a = 0; a < N; ++a) wxy[b * N + a] = x.w(a) * y.w(b);
    }
};

// Footprint member m of tile pixel (lx, ly) as a row-major tile pixel id.
__device__ __forceinline__ int member_id(int fp, int lx, int ly, int m, const uint8_t* lut, int lut_k, int q) {
    switch (fp) {
    case STF_FP_QUAD2X2:
        return ((ly & ~1) + (m >> 1)) * 8 + (lx & ~1) + (m & 1);
    case STF_FP_WAVE2X2: {
        const int ox = min(max(lx - ((ly + (lx >> 1)) & 1), 0), 6);
        const int oy = min(max(ly - ((lx + (ly >> 1)) & 1), 0), 6);
        return (oy + (m >> 1)) * 8 + ox + (m & 1);
    }
    case STF_FP_SQUARE3X3: {
        const int ox = min(max(lx - 1, 0), 5), oy = min(max(ly - 1, 0), 5);
        const int my = m / 3;
        return (oy + my) * 8 + ox + (m - 3 * my);
    }
    case STF_FP_SQUARE4X4: {
        const int ox = min(max(lx - 1, 0), 4), oy = min(max(ly - 1, 0), 4);
        return (oy + (m >> 2)) * 8 + ox + (m & 3);
    }
    case STF_FP_LUT:
        return lut[q * lut_k + m] & 63;
    default:  // STF_FP_TILE8X8
        return m;
    }
}

// Window footprints as origin (ox, oy) and size n on the tile: the members
// are the n x n tile pixels from the origin (member_id in row-major order).
__device__ __forceinline__ void window_of(int fp, int lx, int ly, int& ox, int& oy, int& n) {
    switch (fp) {
    case STF_FP_QUAD2X2: ox = lx & ~1; oy = ly & ~1; n = 2; break;
    case STF_FP_WAVE2X2:
        ox = min(max(lx - ((ly + (lx >> 1)) & 1), 0), 6);
        oy = min(max(ly - ((lx + (ly >> 1)) & 1), 0), 6);
        n = 2;
        break;
    case STF_FP_SQUARE3X3: ox = min(max(lx - 1, 0), 5); oy = min(max(ly - 1, 0), 5); n = 3; break;
    case STF_FP_SQUARE4X4: ox = min(max(lx - 1, 0), 4); oy = min(max(ly - 1, 0), 4); n = 4; break;
    default: ox = 0; oy = 0; n = 8; break;     // STF_FP_TILE8X8
    }
}

__device__ __forceinline__ int footprint_size(int fp, int lut_k) {
    switch (fp) {
    case STF_FP_QUAD2X2: case STF_FP_WAVE2X2: return 4;
    case STF_FP_SQUARE3X3: return 9;
    case STF_FP_SQUARE4X4: return 16;
    case STF_FP_LUT: return lut_k;
    default: return 64;
    }
}

// Offset of texel s (packed sx | sy << 16) inside the support starting at
// (bx, by), modulo the texture size; inside iff both offsets are < N.
template <int N>
__device__ __forceinline__ bool support_offset(uint32_t s, int bx, int by, uint32_t mx, uint32_t my,
                                               uint32_t& dx, uint32_t& dy) {
    dx = ((s & 0xFFFFu) - (uint32_t)bx) & mx;
    dy = ((s >> 16) - (uint32_t)by) & my;
    return dx < (uint32_t)N && dy < (uint32_t)N;
}

// Accumulate one shared pick (texel s, reciprocal PMF r, decoded texel Ti)
// into pixel c's sums; picks outside c's support are skipped.
template <int FILT, int C>
__device__ __forceinline__ void accumulate(const SelCtx<FILT>& ctx, uint32_t s, float r, const float* Ti,
                                           uint32_t mx, uint32_t my, const float* Tc, float& B, float* acc) {
    constexpr int N = SelCtx<FILT>::N;
    uint32_t dx, dy;
    if (support_offset<N>(s, ctx.x.base, ctx.y.base, mx, my, dx, dy)) {
        const float w = ctx.x.wsel(dx) * ctx.y.wsel(dy) * r;
        B += w;
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = fmaf(w, Ti[c] - Tc[c], acc[c]);
    }
}

// Exact filtering (Sec. 4.2): which texels of pixel c's support the shared
// picks hit (bit dy * N + dx) and the Eq. (3) sum over those texels, each
// counted once.
template <int FILT, int C>
struct Coverage {
    static constexpr int N = SelCtx<FILT>::N;
    uint32_t seen = 0u;
    float sum[C];
    __device__ __forceinline__ Coverage() {
#pragma unroll
        for (int c = 0; c < C; ++c) sum[c] = 0.0f;
    }
    __device__ __forceinline__ void add(const SelCtx<FILT>& ctx, uint32_t dx, uint32_t dy, const float* T) {
        const uint32_t bit = 1u << (dy * N + dx);
        if (!(seen & bit)) {
            seen |= bit;
            const float f = ctx.x.wsel(dx) * ctx.y.wsel(dy);
#pragma unroll
            for (int c = 0; c < C; ++c) sum[c] = fmaf(f, T[c], sum[c]);
        }
    }
    __device__ __forceinline__ void add_pick(const SelCtx<FILT>& ctx, uint32_t s, const float* T, uint32_t mx,
                                             uint32_t my) {
        uint32_t dx, dy;
        if (support_offset<N>(s, ctx.x.base, ctx.y.base, mx, my, dx, dy)) add(ctx, dx, dy, T);
    }
    // every support texel of positive weight was picked
    __device__ __forceinline__ bool covered(const SelCtx<FILT>& ctx) const {
        uint32_t need = 0u;
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int a = 0; a < N; ++a)
                if (ctx.wxy[b * N + a] > 0.0f) need |= 1u << (b * N + a);
        return (seen & need) == need;
    }
};

// ---------------------------------------------------------------- texel bins

// One bin per texel of a kBinG x kBinG window: N = sum of 1/p over the picks
// of that texel, plus the texel itself (raw half bits or decoded floats).
// gather() adds one bin's term of  sum_j f_c(j) N_j T_j  to acc and
// f_c(j) N_j to B (half channels enter the FMA unconverted: v_fma_mix_f32).
template <int P> struct Bins;

typedef unsigned int u3 __attribute__((ext_vector_type(3)));

template <> struct Bins<kF16x4> {             // record {raw.x, raw.y, N, pad}, 16-byte aligned
    __device__ static void clear_one(float* l, int rec) {
        *reinterpret_cast<u3*>(__builtin_assume_aligned(&l[rec * 4], 16)) = u3{0u, 0u, 0u};
    }
    __device__ static void put(float* l, int bin, float r, const Texel<kF16x4>& T) {
        atomicAdd(&l[bin * 4 + 2], r);
        *reinterpret_cast<uint2*>(&l[bin * 4]) = T.raw;
    }
    __device__ static void put_texel(float* l, int bin, const Texel<kF16x4>& T) {
        *reinterpret_cast<uint2*>(&l[bin * 4]) = T.raw;
    }
    __device__ static void finalize(float* l, int rec, float n) {
        if (n == 0.0f) clear_one(l, rec);
        else l[rec * 4 + 2] = n;
    }
    __device__ static void gather(const float* l, int bin, float f, float& B, float* acc) {
        const u3 q = *reinterpret_cast<const u3*>(__builtin_assume_aligned(&l[bin * 4], 16));   // 12 of 16 bytes
        const float n = __uint_as_float(q.z);
        const float w = f * n;
        B = fmaf(f, n, B);
        acc[0] = fmaf(w, h2f(q.x), acc[0]);
        acc[1] = fmaf(w, h2f(q.x >> 16), acc[1]);
        acc[2] = fmaf(w, h2f(q.y), acc[2]);
        acc[3] = fmaf(w, h2f(q.y >> 16), acc[3]);
    }
    // Eq. (3) term of the bin (zero texel when empty) and its coverage
    __device__ static void exact(const float* l, int bin, float f, float* ex, bool& cov) {
        const u3 q = *reinterpret_cast<const u3*>(__builtin_assume_aligned(&l[bin * 4], 16));
        cov = cov && (f == 0.0f || __uint_as_float(q.z) != 0.0f);
        ex[0] = fmaf(f, h2f(q.x), ex[0]);
        ex[1] = fmaf(f, h2f(q.x >> 16), ex[1]);
        ex[2] = fmaf(f, h2f(q.y), ex[2]);
        ex[3] = fmaf(f, h2f(q.y >> 16), ex[3]);
    }
};

template <> struct Bins<kF16x2> {             // record {raw, N}
    __device__ static void clear_one(float* l, int rec) { reinterpret_cast<uint2*>(l)[rec] = make_uint2(0u, 0u); }
    __device__ static void put(float* l, int bin, float r, const Texel<kF16x2>& T) {
        atomicAdd(&l[bin * 2 + 1], r);
        reinterpret_cast<uint32_t*>(l)[bin * 2] = T.raw;
    }
    __device__ static void put_texel(float* l, int bin, const Texel<kF16x2>& T) {
        reinterpret_cast<uint32_t*>(l)[bin * 2] = T.raw;
    }
    __device__ static void finalize(float* l, int rec, float n) {
        if (n == 0.0f) clear_one(l, rec);
        else l[rec * 2 + 1] = n;
    }
    __device__ static void gather(const float* l, int bin, float f, float& B, float* acc) {
        const uint2 q = reinterpret_cast<const uint2*>(l)[bin];
        const float n = __uint_as_float(q.y);
        const float w = f * n;
        B = fmaf(f, n, B);
        acc[0] = fmaf(w, h2f(q.x), acc[0]);
        acc[1] = fmaf(w, h2f(q.x >> 16), acc[1]);
    }
    __device__ static void exact(const float* l, int bin, float f, float* ex, bool& cov) {
        const uint2 q = reinterpret_cast<const uint2*>(l)[bin];
        cov = cov && (f == 0.0f || __uint_as_float(q.y) != 0.0f);
        ex[0] = fmaf(f, h2f(q.x), ex[0]);
        ex[1] = fmaf(f, h2f(q.x >> 16), ex[1]);
    }
};

template <> struct Bins<kF32x1> {             // record {T, N}
    __device__ static void clear_one(float* l, int rec) { reinterpret_cast<uint2*>(l)[rec] = make_uint2(0u, 0u); }
    __device__ static void put(float* l, int bin, float r, const Texel<kF32x1>& T) {
        atomicAdd(&l[bin * 2 + 1], r);
        l[bin * 2] = T.v[0];
    }
    __device__ static void put_texel(float* l, int bin, const Texel<kF32x1>& T) { l[bin * 2] = T.v[0]; }
    __device__ static void finalize(float* l, int rec, float n) {
        if (n == 0.0f) clear_one(l, rec);
        else l[rec * 2 + 1] = n;
    }
    __device__ static void gather(const float* l, int bin, float f, float& B, float* acc) {
        const float2 q = reinterpret_cast<const float2*>(l)[bin];
        const float w = f * q.y;
        B = fmaf(f, q.y, B);
        acc[0] = fmaf(w, q.x, acc[0]);
    }
    __device__ static void exact(const float* l, int bin, float f, float* ex, bool& cov) {
        const float2 q = reinterpret_cast<const float2*>(l)[bin];
        cov = cov && (f == 0.0f || q.y != 0.0f);
        ex[0] = fmaf(f, q.x, ex[0]);
    }
};

template <> struct Bins<kF32x4> {             // float4 T[kBinRecords], then float N[kBinRecords]
    __device__ static void clear_one(float* l, int rec) {
        reinterpret_cast<uint4*>(l)[rec] = make_uint4(0u, 0u, 0u, 0u);
        l[4 * kBinRecords + rec] = 0.0f;
    }
    __device__ static void put(float* l, int bin, float r, const Texel<kF32x4>& T) {
        atomicAdd(&l[4 * kBinRecords + bin], r);
        reinterpret_cast<float4*>(l)[bin] = make_float4(T.v[0], T.v[1], T.v[2], T.v[3]);
    }
    __device__ static void put_texel(float* l, int bin, const Texel<kF32x4>& T) {
        reinterpret_cast<float4*>(l)[bin] = make_float4(T.v[0], T.v[1], T.v[2], T.v[3]);
    }
    __device__ static void finalize(float* l, int rec, float n) {
        if (n == 0.0f) clear_one(l, rec);
        else l[4 * kBinRecords + rec] = n;
    }
    __device__ static void gather(const float* l, int bin, float f, float& B, float* acc) {
        const float4 q = reinterpret_cast<const float4*>(l)[bin];
        const float n = l[4 * kBinRecords + bin];
        const float w = f * n;
        B = fmaf(f, n, B);
        acc[0] = fmaf(w, q.x, acc[0]);
        acc[1] = fmaf(w, q.y, acc[1]);
        acc[2] = fmaf(w, q.z, acc[2]);
        acc[3] = fmaf(w, q.w, acc[3]);
    }
    __device__ static void exact(const float* l, int bin, float f, float* ex, bool& cov) {
        const float4 q = reinterpret_cast<const float4*>(l)[bin];
        cov = cov && (f == 0.0f || l[4 * kBinRecords + bin] != 0.0f);
        ex[0] = fmaf(f, q.x, ex[0]);
        ex[1] = fmaf(f, q.y, ex[1]);
        ex[2] = fmaf(f, q.z, ex[2]);
        ex[3] = fmaf(f, q.w, ex[3]);
    }
};

// Offset of support start b from lane 0's b0 modulo the texture size m + 1,
// taken in [-(m + 1) / 2, (m + 1) / 2).
__device__ __forceinline__ int wrapped_offset(int b, int b0, uint32_t m) {
    const int d = (int)((uint32_t)(b - b0) & m);
    return d > (int)(m >> 1) ? d - (int)m - 1 : d;
}

// Bin window of the wave: kBinG x kBinG texels, first with its corner
// `margin` texels before lane 0's support (no reduction: the common case at
// magnification); if some pixel's support leaves that, from the wave's
// smallest support start (two wave reductions per axis), which holds every
// tile whose support starts spread over at most kBinG - N texels per axis
// (about 1x magnification for the B-spline, 0.8x for bilinear). Returns
// false (wave-uniformly) when neither placement holds every support. Lanes
// off the screen read the UV of their nearest on-screen pixel, so their
// supports are among the on-screen ones.
template <int N>
__device__ __forceinline__ bool bin_window(const Pixel& P, int bx, int by, uint32_t mx, uint32_t my, int tw, int th,
                                           int& base_x, int& base_y, uint32_t& rx, uint32_t& ry) {
    constexpr int margin = (kBinG - N) / 2;
    constexpr int span = kBinG - N;
    if (tw < kBinG || th < kBinG) return false;
    const int x0 = __builtin_amdgcn_readfirstlane(bx), y0 = __builtin_amdgcn_readfirstlane(by);
    base_x = x0 - margin;
    base_y = y0 - margin;
    rx = (uint32_t)(bx - base_x) & mx;
    ry = (uint32_t)(by - base_y) & my;
    const bool fits = !P.valid || (rx <= (uint32_t)span && ry <= (uint32_t)span);
    if (__builtin_amdgcn_ballot_w64(!fits) == 0) return true;
    const int dx = wrapped_offset(bx, x0, mx), dy = wrapped_offset(by, y0, my);
    const int lo_x = wave_min(dx), hi_x = -wave_min(-dx);
    const int lo_y = wave_min(dy), hi_y = -wave_min(-dy);
    if (hi_x - lo_x > span || hi_y - lo_y > span) return false;
    base_x = x0 + lo_x;
    base_y = y0 + lo_y;
    rx = (uint32_t)(dx - lo_x);
    ry = (uint32_t)(dy - lo_y);
    return true;
}

// Bounding box, in window coordinates, of every on-screen pixel's support:
// one bit per support start column / row, OR-reduced over the wave.
struct BinBox {
    int x0, x1, y0, y1;
};

template <int N>
__device__ __forceinline__ BinBox support_box(const Pixel& P, uint32_t rx, uint32_t ry) {
    const uint32_t bits = wave_or(P.valid ? ((1u << rx) | (1u << (16u + ry))) : 0u);
    BinBox b;
    b.x0 = __builtin_ctz(bits & 0xFFFFu);
    b.x1 = 31 - __builtin_clz(bits & 0xFFFFu) + N - 1;
    b.y0 = __builtin_ctz(bits >> 16);
    b.y1 = 31 - __builtin_clz(bits >> 16) + N - 1;
    return b;
}

// Calls f(record) for every bin of the box, one 8x8 block of bins per step
// (lane -> (lane & 7, lane >> 3)); wave-uniform trip counts.
template <typename F>
__device__ __forceinline__ void for_box(const BinBox& b, int lane, F f) {
    const int x = b.x0 + (lane & 7), y = b.y0 + (lane >> 3);
    if (b.x1 - b.x0 < 8 && b.y1 - b.y0 < 8) {          // one block (magnification >= ~1.6x)
        if (x <= b.x1 && y <= b.y1) f(y * kBinStride + x);
        return;
    }
    for (int by = b.y0; by <= b.y1; by += 8)
        for (int bx = b.x0; bx <= b.x1; bx += 8) {
            const int x = bx + (lane & 7), y = by + (lane >> 3);
            if (x <= b.x1 && y <= b.y1) f(y * kBinStride + x);
        }
}

// Exact sums of 1/p per bin at a fixed scale. p <= 1, so every reciprocal PMF
// r >= 1 is an integer multiple of 2^-23 (its last significand bit is worth
// at least that); for r < 2^34 the integer r * 2^23 is below 2^57, and 64 of
// them sum below 2^63: the 64-bit sums are exact and independent of the
// order of the atomic adds, and no wave-wide scale is needed. Each bin is
// converted to FP32 within 2 ulp, deterministically. A wave holding an r
// outside [1, 2^34) (probability below 2^-34 per pick) takes FP32 atomics.
__device__ __forceinline__ bool fixed_range(float r) {
    return (__float_as_uint(r) >> 23) - 127u <= 33u;      // also false for r < 1
}

__device__ __forceinline__ uint64_t fixed_r(float r) {
    const uint32_t b = __float_as_uint(r);
    return (uint64_t)((b & 0x7FFFFFu) | 0x800000u) << ((b >> 23) - 127u);
}

__device__ __forceinline__ float float_r(uint64_t n) {
    // n < 2^63, so its high word is below 2^31 and converts as a signed int
    return fmaf((float)(int32_t)(n >> 32), 4294967296.0f, (float)(uint32_t)n) * 0x1p-23f;   // within 2 ulp
}

// Bin window and support box of the wave for one texture size (shared by
// every texture of that size).
template <int N>
struct BinGeom {
    bool ok = false;         // every on-screen support fits the window
    bool clean = false;      // the 64-bit sums of the box are zero (left so by the last finalize)
    uint32_t rx = 0, ry = 0; // this pixel's support start inside the window
    BinBox box;
    int tw = 0, th = 0;
};

template <int FILT>
__device__ __forceinline__ void update_geom(BinGeom<AxisCtx<FILT>::N>& g, const Pixel& P, const SelCtx<FILT>& ctx,
                                            int tw, int th) {
    constexpr int N = AxisCtx<FILT>::N;
    if (g.tw == tw && g.th == th) return;                // wave-uniform
    int base_x, base_y;
    g.ok = bin_window<N>(P, ctx.x.base, ctx.y.base, (uint32_t)tw - 1u, (uint32_t)th - 1u, tw, th, base_x, base_y,
                         g.rx, g.ry);
    if (g.ok) g.box = support_box<N>(P, g.rx, g.ry);
    g.clean = false;
    g.tw = tw;
    g.th = th;
}

// Receive the pick of quad partner lane^X through DPP and accumulate it.
template <int X, int FILT, int C, bool EF, int CC>
__device__ __forceinline__ void quad_step(const SelCtx<FILT>& ctx, uint32_t s, float r, const float* Tv, uint32_t mx,
                                          uint32_t my, float& B, float* acc, Coverage<FILT, CC>& cov) {
    float Ti[C];
    const uint32_t si = quad_xor<X>(s);
    const float ri = quad_xor<X>(r);
#pragma unroll
    for (int c = 0; c < C; ++c) Ti[c] = quad_xor<X>(Tv[c]);
    accumulate<FILT, C>(ctx, si, ri, Ti, mx, my, Tv, B, acc);
    if constexpr (EF) {
        if (ri != 0.0f) cov.add_pick(ctx, si, Ti, mx, my);   // off-screen partners carry r = 0
    }
}

// The one-tap pick of one texture slot: per-axis offsets, texel, and the
// 16-byte block holding the texel (extracted after every load is issued).
struct SlotPick {
    int kx, ky;
    uint32_t sx, sy;
    uint4 raw;
};

template <int FILT>
__device__ __forceinline__ SlotPick pick_slot(const TexArg& t, const SelCtx<FILT>& ctx, uint32_t hx, uint32_t hy) {
    SlotPick k;
    k.kx = ctx.x.pick(hx);
    k.ky = ctx.y.pick(hy);
    k.sx = (uint32_t)(ctx.x.base + k.kx) & ((uint32_t)t.w - 1u);
    k.sy = (uint32_t)(ctx.y.base + k.ky) & ((uint32_t)t.h - 1u);
    k.raw = fetch_block(t, k.sx, k.sy, format_bytes(t.fmt));
    return k;
}

// True when every on-screen lane holds the same texel payload (bit for bit).
template <int PL>
__device__ __forceinline__ bool wave_same_texel(const Texel<PL>& T, bool valid) {
    const uint64_t on = __builtin_amdgcn_ballot_w64(valid);
    const int first = on ? (int)__builtin_ctzll(on) : 0;
    bool same = true;
#pragma unroll
    for (int k = 0; k < Texel<PL>::W; ++k) {
        const uint32_t x = T.word(k);
        same = same && x == (uint32_t)__builtin_amdgcn_readlane((int)x, first);
    }
    return __builtin_amdgcn_ballot_w64(valid && !same) == 0;
}

// Exchange and estimator for one texture slot of one pixel. LAT: the texture
// holds latents; the picked texel is decoded by the MLP in `dec` (LDS) before
// it is shared, so every pixel decodes exactly one texel.
// EF: exact filtering (Sec. 4.2) replaces the estimate by the Eq. (3) value
// whenever the shared picks cover the pixel's support.
template <int FILT, int MODE, int PL, bool LAT = false, bool EF = false>
__device__ __forceinline__ void slot_pass(const Args& a, const TexArg& t, int slot, const Pixel& P,
                                          const SelCtx<FILT>& ctx, BinGeom<AxisCtx<FILT>::N>& geom,
                                          const SlotPick& pk, float* lds, const uint8_t* dec = nullptr,
                                          const uint8_t* lut_lds = nullptr) {
    static_assert(!LAT || PL == kF32x4, "decoded latents are RGBA FP32");
    constexpr int N = SelCtx<FILT>::N;
    constexpr int C = Texel<PL>::C;
    const int lane = lane_id();
    const int kx = pk.kx, ky = pk.ky;
    const uint32_t mx = (uint32_t)t.w - 1u, my = (uint32_t)t.h - 1u;
    // reuse modes recompute the picked texel from the offsets, so that the
    // pick's copies are not kept live across the other slots' passes
    const uint32_t sx = MODE == kModeStf ? pk.sx : (uint32_t)(ctx.x.base + kx) & mx;
    const uint32_t sy = MODE == kModeStf ? pk.sy : (uint32_t)(ctx.y.base + ky) & my;
    Texel<PL> T;
    if constexpr (LAT)
        decode_latent_dedup(dec, latent_operand(dec, block_texel(pk.raw, sx, format_bytes(t.fmt)), t), sx, sy, mx, my,
                            reinterpret_cast<uint8_t*>(lds), T.v);
    else
        T = decode<PL>(block_texel(pk.raw, sx, format_bytes(t.fmt)), t.fmt);
    const bool scale_out = !LAT && t.has_scale;       // a latent scale precedes the decoder
    const int64_t pix = (int64_t)P.py * a.sw + P.px;

    if (a.sel != nullptr && P.valid) {
        int2* sp = reinterpret_cast<int2*>(a.sel) + ((int64_t)slot * a.sh * a.sw + pix);
        *sp = make_int2((int)sx, (int)sy);
    }
    float Tv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) Tv[c] = T.ch(c);
    if constexpr (MODE == kModeStf) {
        if (scale_out) {
#pragma unroll
            for (int c = 0; c < C; ++c) Tv[c] *= t.scale[c];
        }
        if (P.valid) store_out<C>(a.out[slot], pix, Tv);
        return;
    } else {
        // 1/p of the own pick; off-screen pixels share a pick of weight zero
        const float pc = ctx.x.wsel(kx) * ctx.y.wsel(ky);
        const float r = P.valid ? fast_rcp(pc) : 0.0f;
        if (!P.valid) {
#pragma unroll
            for (int c = 0; c < C; ++c) Tv[c] = 0.0f;
        }
        const uint32_t s = sx | (sy << 16);
        float B = 1.0f;            // own pick: w_c = f_c / p_c = 1 (Sec. 4.5)
        float acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0.0f;
        Coverage<FILT, EF ? C : 1> cov;            // used only with EF
        bool covered = false;
        bool lone = false;                         // whole tile: no other pick in the support

        if constexpr (MODE == kModeQuad) {
            if constexpr (EF) cov.add(ctx, (uint32_t)kx, (uint32_t)ky, Tv);
            quad_step<1, FILT, C, EF>(ctx, s, r, Tv, mx, my, B, acc, cov);
            quad_step<2, FILT, C, EF>(ctx, s, r, Tv, mx, my, B, acc, cov);
            quad_step<3, FILT, C, EF>(ctx, s, r, Tv, mx, my, B, acc, cov);
            if constexpr (EF) covered = cov.covered(ctx);
        } else {
            bool use_bins = false;
            if constexpr (MODE == kModeBins) {
                use_bins = geom.ok;
                if (use_bins) {
                    // every on-screen pick of the wave holds the same texel: Eq. (14) returns it
                    const bool flat = wave_same_texel<PL>(T, P.valid);
                    if (!flat || EF) {               // exact filtering still needs the coverage
                        const uint32_t rx = geom.rx, ry = geom.ry;
                        const BinBox& box = geom.box;
                        const int my_bin = (int)(ry + ky) * kBinStride + (int)(rx + kx);
                        const bool fixed = !(a.flags & kFlagFloatBinSums) &&
                                           __builtin_amdgcn_ballot_w64(P.valid && !fixed_range(r)) == 0;
                        if (fixed) {
                            uint64_t* acc64 = reinterpret_cast<uint64_t*>(lds + kAccFloatOffset);
                            if (!geom.clean) {
                                for_box(box, lane, [&](int rec) { acc64[rec] = 0ull; });
                                wave_lds_sync();
                            }
                            if (P.valid) {
                                atomicAdd(reinterpret_cast<unsigned long long*>(&acc64[my_bin]),
                                          (unsigned long long)fixed_r(r));
                                Bins<PL>::put_texel(lds, my_bin, T);
                            }
                            wave_lds_sync();
                            // N of every bin; the sums are left zero for the next texture of this size
                            for_box(box, lane, [&](int rec) {
                                const uint64_t n = acc64[rec];
                                acc64[rec] = 0ull;
                                Bins<PL>::finalize(lds, rec, float_r(n));
                            });
                            geom.clean = true;
                        } else {
                            for_box(box, lane, [&](int rec) { Bins<PL>::clear_one(lds, rec); });
                            wave_lds_sync();
                            if (P.valid) Bins<PL>::put(lds, my_bin, r, T);
                        }
                        wave_lds_sync();
                        B = 0.0f;                    // the own pick is in the bins
                        const int bin0 = (int)ry * kBinStride + (int)rx;
                        bool all_in = true;
#pragma unroll
                        for (int b = 0; b < N; ++b) {
                            const float wyb = ctx.y.w(b);
#pragma unroll
                            for (int aa = 0; aa < N; ++aa) {
                                const float f = ctx.x.w(aa) * wyb;
                                Bins<PL>::gather(lds, bin0 + b * kBinStride + aa, f, B, acc);
                                // same weights and order as the Eq. (3) kernel: bit-identical sums
                                if constexpr (EF) Bins<PL>::exact(lds, bin0 + b * kBinStride + aa, f, cov.sum, all_in);
                            }
                        }
                        if constexpr (EF) covered = all_in;
                        wave_lds_sync();             // reads done before the next slot reuses LDS
                    }
                    if (flat) {                      // out = T_c exactly
                        B = 1.0f;
#pragma unroll
                        for (int c = 0; c < C; ++c) acc[c] = 0.0f;
                    } else {
                        // No other pick of positive weight in the support: B is then exactly
                        // the own bin's term p_c r_c (the other bins add exact zeros), and
                        // Eq. (14) is the own texel, returned as one-tap STF returns it.
                        // Otherwise out = acc / B, with no T_c term.
                        lone = B == pc * r;
#pragma unroll
                        for (int c = 0; c < C; ++c) Tv[c] = lone ? Tv[c] : 0.0f;
                    }
                }
            }
            if (!use_bins) {
                uint2* meta = reinterpret_cast<uint2*>(lds);        // [64] {s, r}
                float4* val = reinterpret_cast<float4*>(lds + 128);  // [64] texel
                meta[P.q] = make_uint2(s, __float_as_uint(r));
                float pad[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int c = 0; c < C; ++c) pad[c] = Tv[c];
                val[P.q] = make_float4(pad[0], pad[1], pad[2], pad[3]);
                wave_lds_sync();
                if constexpr (EF) cov.add(ctx, (uint32_t)kx, (uint32_t)ky, Tv);
                auto member = [&](int j) {
                    if (j == P.q) return;            // the own pick is already counted
                    const uint2 mj = meta[j];
                    const float4 vj = val[j];
                    const float Ti[4] = {vj.x, vj.y, vj.z, vj.w};
                    accumulate<FILT, C>(ctx, mj.x, __uint_as_float(mj.y), Ti, mx, my, Tv, B, acc);
                    if constexpr (EF) {
                        if (__uint_as_float(mj.y) != 0.0f) cov.add_pick(ctx, mj.x, Ti, mx, my);
                    }
                };
                if constexpr (MODE == kModeBins) {   // record fallback of the whole tile
                    for (int m = 0; m < 64; ++m) {
                        if (m == P.q) continue;
                        const uint2 mj = meta[m];
                        const float4 vj = val[m];
                        const float Ti[4] = {vj.x, vj.y, vj.z, vj.w};
                        accumulate<FILT, C>(ctx, mj.x, __uint_as_float(mj.y), Ti, mx, my, Tv, B, acc);
                        if constexpr (EF) {
                            if (__uint_as_float(mj.y) != 0.0f) cov.add_pick(ctx, mj.x, Ti, mx, my);
                        }
                    }
                } else if (a.footprint == STF_FP_LUT && lut_lds != nullptr) {
                    for (int m = 0; m < a.lut_k; ++m) member(lut_lds[P.q * a.lut_k + m] & 63);   // staged
                } else if (a.footprint == STF_FP_LUT) {
                    for (int m = 0; m < a.lut_k; ++m) member(a.lut[P.q * a.lut_k + m] & 63);
                } else {
                    // square windows: origin and size once per pixel, then the rows and
                    // columns of the window (wave-uniform trip counts)
                    int ox, oy, n;
                    window_of(a.footprint, P.lx, P.ly, ox, oy, n);
                    for (int wy = 0; wy < n; ++wy)
                        for (int wx = 0; wx < n; ++wx) member((oy + wy) * 8 + ox + wx);
                }
                if constexpr (EF) covered = cov.covered(ctx);
                wave_lds_sync();
            }
        }
        if (P.valid) {
            float o[C];
            const float inv = lone ? 0.0f : fast_rcp(B);
#pragma unroll
            for (int c = 0; c < C; ++c) o[c] = fmaf(acc[c], inv, Tv[c]);
            if constexpr (EF) {
                if (covered) {
#pragma unroll
                    for (int c = 0; c < C; ++c) o[c] = cov.sum[c];
                }
            }
            if (scale_out) {                     // Eq. (14) is linear in the texels
#pragma unroll
                for (int c = 0; c < C; ++c) o[c] *= t.scale[c];
            }
            store_out<C>(a.out[slot], pix, o);
        }
    }
}

// This lane's pixel of screen tile (tx, ty); UV not loaded.
__device__ __forceinline__ void place_pixel(const Args& a, int tx, int ty, Pixel& P) {
    lane_pixel(lane_id(), P.lx, P.ly);
    P.q = P.ly * 8 + P.lx;
    P.px = tx * kTile + P.lx;
    P.py = ty * kTile + P.ly;
    P.valid = (P.px < a.sw) && (P.py < a.sh);
}

// UV of screen pixel (px, py), clamped to the screen (off-screen lanes of
// edge tiles read their nearest on-screen pixel).
__device__ __forceinline__ v2f load_uv(const Args& a, int px, int py) {
    const int cx = min(px, a.sw - 1), cy = min(py, a.sh - 1);
    return __builtin_nontemporal_load(reinterpret_cast<const v2f*>(a.uv) + ((int64_t)cy * a.sw + cx));
}

// Pixel and UV of this lane for one-tile-per-wave kernels; false when the
// wave's whole tile is off screen.
__device__ __forceinline__ bool setup_pixel(const Args& a, Pixel& P) {
    const int tx = blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6);
    if (tx * kTile >= a.sw) return false;
    place_pixel(a, tx, blockIdx.y, P);
    const v2f uv = load_uv(a, P.px, P.py);
    P.u = uv.x;
    P.v = uv.y;
    return true;
}

// Random numbers of the slot whose selection slot `slot` uses (itself, or
// with shared selection the first slot of the same texture size), computed
// on their own.
__device__ __forceinline__ void keyed_uniforms(const Args& a, const Pixel& P, int slot, uint32_t& hx, uint32_t& hy) {
    const int key = a.leader[slot];
    const uint4 h = pcg4d(make_uint4((uint32_t)P.px, (uint32_t)P.py, a.frame, a.seed + (uint32_t)(key >> 1) * kGolden));
    hx = (key & 1) ? h.z : h.x;
    hy = (key & 1) ? h.w : h.y;
}

// Random numbers of texture slot `slot`: slots 2q and 2q+1 share one pcg4d
// evaluation keyed with seed + q * golden (first / last two outputs).
__device__ __forceinline__ void slot_uniforms(const Args& a, const Pixel& P, int slot, uint4& hq, uint32_t& hx,
                                              uint32_t& hy) {
    if ((slot & 1) == 0)
        hq = pcg4d(make_uint4((uint32_t)P.px, (uint32_t)P.py, a.frame, a.seed + (uint32_t)(slot >> 1) * kGolden));
    hx = (slot & 1) ? hq.z : hq.x;
    hy = (slot & 1) ? hq.w : hq.y;
}

__device__ __forceinline__ int payload_of(int fmt) {
    switch (fmt) {
    case STF_RGBA16F: return kF16x4;
    case STF_RG16F: return kF16x2;
    case STF_R8_UNORM: case STF_R32F: return kF32x1;
    case STF_LATENT8_F16: case STF_LATENT8_BF16: case STF_LATENT8_FP8: return kLatent;
    default: return kF32x4;          // RGBA8, RGBA32F, RGBA BF16, RGBA FP8
    }
}

// The picked texel of one slot as four floats (channels past the payload's
// are zero).
template <int PL>
__device__ __forceinline__ void texel_floats(const TexArg& t, const SlotPick& pk, uint32_t sx, float (&v)[4]) {
    const Texel<PL> T = decode<PL>(block_texel(pk.raw, sx, format_bytes(t.fmt)), t.fmt);
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = 0.0f;
#pragma unroll
    for (int c = 0; c < Texel<PL>::C; ++c) v[c] = T.ch(c);
}

// LDS floats per wave of the one-size record kernel: {s, r}[64], then one
// float4 texel per lane and slot.
template <int NT>
constexpr int kSharedRecordFloats = 128 + NT * 256;

// Record footprints under shared selection, every slot led by slot 0 (one
// texture size, Sec. 4.5): all slots pick the same texel, so the support
// test and weight w_i = f_c(x_i) / p_i of a member are formed once and
// applied to every slot's texel. Per slot the sums are the ones slot_pass
// forms, operation for operation, so the outputs are the same bits. LDS:
// {s, r}[64], then one float4 texel per lane and slot.
template <int FILT, int NT>
__device__ __forceinline__ void shared_records_pass(const Args& a, const TexArg (&t)[NT], const Pixel& P,
                                                    const SelCtx<FILT>& ctx, const SlotPick (&pk)[NT], float* lds,
                                                    const uint8_t* lut_lds) {
    static_assert(NT >= 2 && NT <= 4, "two to four slots");
    constexpr int N = SelCtx<FILT>::N;
    const uint32_t mx = (uint32_t)t[0].w - 1u, my = (uint32_t)t[0].h - 1u;
    const int kx = pk[0].kx, ky = pk[0].ky;
    const uint32_t sx = (uint32_t)(ctx.x.base + kx) & mx;
    const uint32_t sy = (uint32_t)(ctx.y.base + ky) & my;
    const int64_t pix = (int64_t)P.py * a.sw + P.px;
    float Tv[NT][4];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        switch (payload_of(t[i].fmt)) {
        case kF16x4: texel_floats<kF16x4>(t[i], pk[i], sx, Tv[i]); break;
        case kF16x2: texel_floats<kF16x2>(t[i], pk[i], sx, Tv[i]); break;
        case kF32x1: texel_floats<kF32x1>(t[i], pk[i], sx, Tv[i]); break;
        case kLatent: Tv[i][0] = Tv[i][1] = Tv[i][2] = Tv[i][3] = 0.0f; break;   // the decoder kernels' case
        default: texel_floats<kF32x4>(t[i], pk[i], sx, Tv[i]); break;
        }
        if (a.sel != nullptr && P.valid)
            reinterpret_cast<int2*>(a.sel)[(int64_t)i * a.sh * a.sw + pix] = make_int2((int)sx, (int)sy);
    }
    // 1/p of the own pick; off-screen pixels share a pick of weight zero
    const float pc = ctx.x.wsel(kx) * ctx.y.wsel(ky);
    const float r = P.valid ? fast_rcp(pc) : 0.0f;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) Tv[i][c] = P.valid ? Tv[i][c] : 0.0f;
    uint2* meta = reinterpret_cast<uint2*>(lds);          // [64] {s, r}
    float4* val = reinterpret_cast<float4*>(lds + 128);   // [NT][64] texel
    meta[P.q] = make_uint2(sx | (sy << 16), __float_as_uint(r));
#pragma unroll
    for (int i = 0; i < NT; ++i) val[i * 64 + P.q] = make_float4(Tv[i][0], Tv[i][1], Tv[i][2], Tv[i][3]);
    wave_lds_sync();
    float B = 1.0f;            // own pick: w_c = 1
    float acc[NT][4];
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[i][c] = 0.0f;
    auto member = [&](int j) {
        if (j == P.q) return;                // the own pick is already counted
        const uint2 mj = meta[j];
        float4 vj[NT];
#pragma unroll
        for (int i = 0; i < NT; ++i) vj[i] = val[i * 64 + j];
        uint32_t dx, dy;
        if (support_offset<N>(mj.x, ctx.x.base, ctx.y.base, mx, my, dx, dy)) {
            const float w = ctx.x.wsel(dx) * ctx.y.wsel(dy) * __uint_as_float(mj.y);
            B += w;
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                const float Ti[4] = {vj[i].x, vj[i].y, vj[i].z, vj[i].w};
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[i][c] = fmaf(w, Ti[c] - Tv[i][c], acc[i][c]);
            }
        }
    };
    if (a.footprint == STF_FP_LUT && lut_lds != nullptr) {
        for (int m = 0; m < a.lut_k; ++m) member(lut_lds[P.q * a.lut_k + m] & 63);   // staged
    } else if (a.footprint == STF_FP_LUT) {
        for (int m = 0; m < a.lut_k; ++m) member(a.lut[P.q * a.lut_k + m] & 63);
    } else {
        int ox, oy, n;
        window_of(a.footprint, P.lx, P.ly, ox, oy, n);
        for (int wy = 0; wy < n; ++wy)
            for (int wx = 0; wx < n; ++wx) member((oy + wy) * 8 + ox + wx);
    }
    wave_lds_sync();                         // reads done before the wave's next tile reuses LDS
    if (P.valid) {
        const float inv = fast_rcp(B);
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            float o[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) o[c] = fmaf(acc[i][c], inv, Tv[i][c]);
            if (t[i].has_scale) {            // Eq. (14) is linear in the texels
#pragma unroll
                for (int c = 0; c < 4; ++c) o[c] *= t[i].scale[c];
            }
            switch (payload_of(t[i].fmt)) {
            case kF16x2: store_out<2>(a.out[i], pix, o); break;
            case kF32x1: store_out<1>(a.out[i], pix, o); break;
            case kLatent: break;
            default: store_out<4>(a.out[i], pix, o); break;
            }
        }
    }
}

// One slot's quad sums under shared selection: the partners' weights wq
// (support test inq) are the slot-independent part; each slot moves its own
// C channels. Same operations, in the same order, as quad_step.
template <int C>
__device__ __forceinline__ void quad_slot_sums(const float (&wq)[3], const bool (&inq)[3], const float (&Tc)[4],
                                               float (&acc)[4]) {
    static_for<3>([&](auto X) {
        constexpr int x = decltype(X)::value + 1;
        float Ti[C];
#pragma unroll
        for (int c = 0; c < C; ++c) Ti[c] = quad_xor<x>(Tc[c]);
        if (inq[x - 1]) {
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = fmaf(wq[x - 1], Ti[c] - Tc[c], acc[c]);
        }
    });
}

// 2x2 quads under shared selection, every slot led by slot 0: each
// partner's pick, reciprocal PMF, support test and weight cross the quad
// and are formed once for all slots; per slot the sums are quad_step's.
template <int FILT, int NT>
__device__ __forceinline__ void shared_quad_pass(const Args& a, const TexArg (&t)[NT], const Pixel& P,
                                                 const SelCtx<FILT>& ctx, const SlotPick (&pk)[NT]) {
    constexpr int N = SelCtx<FILT>::N;
    const uint32_t mx = (uint32_t)t[0].w - 1u, my = (uint32_t)t[0].h - 1u;
    const int kx = pk[0].kx, ky = pk[0].ky;
    const uint32_t sx = (uint32_t)(ctx.x.base + kx) & mx;
    const uint32_t sy = (uint32_t)(ctx.y.base + ky) & my;
    const int64_t pix = (int64_t)P.py * a.sw + P.px;
    float Tv[NT][4];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        switch (payload_of(t[i].fmt)) {
        case kF16x4: texel_floats<kF16x4>(t[i], pk[i], sx, Tv[i]); break;
        case kF16x2: texel_floats<kF16x2>(t[i], pk[i], sx, Tv[i]); break;
        case kF32x1: texel_floats<kF32x1>(t[i], pk[i], sx, Tv[i]); break;
        case kLatent: Tv[i][0] = Tv[i][1] = Tv[i][2] = Tv[i][3] = 0.0f; break;   // the decoder kernels' case
        default: texel_floats<kF32x4>(t[i], pk[i], sx, Tv[i]); break;
        }
        if (a.sel != nullptr && P.valid)
            reinterpret_cast<int2*>(a.sel)[(int64_t)i * a.sh * a.sw + pix] = make_int2((int)sx, (int)sy);
    }
    const float pc = ctx.x.wsel(kx) * ctx.y.wsel(ky);
    const float r = P.valid ? fast_rcp(pc) : 0.0f;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) Tv[i][c] = P.valid ? Tv[i][c] : 0.0f;
    const uint32_t s = sx | (sy << 16);
    float B = 1.0f;            // own pick: w_c = 1
    float wq[3];
    bool inq[3];
    static_for<3>([&](auto X) {
        constexpr int x = decltype(X)::value + 1;
        const uint32_t si = quad_xor<x>(s);
        const float ri = quad_xor<x>(r);
        uint32_t dx, dy;
        inq[x - 1] = support_offset<N>(si, ctx.x.base, ctx.y.base, mx, my, dx, dy);
        wq[x - 1] = 0.0f;
        if (inq[x - 1]) {
            wq[x - 1] = ctx.x.wsel(dx) * ctx.y.wsel(dy) * ri;
            B += wq[x - 1];
        }
    });
    const float inv = fast_rcp(B);
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        const int pl = payload_of(t[i].fmt);
        if (pl == kF16x2) quad_slot_sums<2>(wq, inq, Tv[i], acc);
        else if (pl == kF32x1) quad_slot_sums<1>(wq, inq, Tv[i], acc);
        else quad_slot_sums<4>(wq, inq, Tv[i], acc);
        if (P.valid) {
            float o[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) o[c] = fmaf(acc[c], inv, Tv[i][c]);
            if (t[i].has_scale) {            // Eq. (14) is linear in the texels
#pragma unroll
                for (int c = 0; c < 4; ++c) o[c] *= t[i].scale[c];
            }
            switch (pl) {
            case kF16x2: store_out<2>(a.out[i], pix, o); break;
            case kF32x1: store_out<1>(a.out[i], pix, o); break;
            case kLatent: break;
            default: store_out<4>(a.out[i], pix, o); break;
            }
        }
    }
}

// Waves per SIMD the forward kernels are register-budgeted for (VGPRs per
// lane: 512 / waves, in steps of 8). The whole-tile kernel issues VALU most
// of the time and hides its memory and LDS latency with occupancy: with up
// to two textures it fits 64 VGPRs (eight waves; two textures spill a few
// registers there, which ran 4 % faster than seven waves at 72 VGPRs without
// spills), three textures fit 72 (seven waves), four keep 80 (six waves;
// they spill a few registers, and at 72 more of them, which ran 15 % slower;
// 96 without spills, five waves, measured no faster); with the latent
// decoder it keeps 128 (four waves; its slots run one after another).
template <int MODE, int NT, bool DEC, bool EF>
constexpr int kForwardWaves = (MODE == kModeBins && !EF) ? (DEC ? 4 : NT <= 2 ? 8 : NT == 3 ? 7 : 6) : 1;

// Screen tile rows each forward wave filters one after the other (one tile
// column): the next row's UV is loaded while the current row is filtered,
// and a workgroup stages the decoder once for all its rows. Only the
// decoder kernels take more than one row: in the others the extra live
// registers cost more occupancy than the prefetch hides.
template <bool DEC>
constexpr int kForwardRows = DEC ? 2 : 1;

// One screen tile, NT textures unrolled: descriptors are loaded once, and
// every pick and texel fetch is issued before the first exchange so their
// latencies overlap; then the UV of the wave's next tile (more = true) is
// requested into uv_next.
// SHR: record footprints with every slot led by slot 0 (shared_records_pass).
template <int FILT, int MODE, int NT, bool DEC, bool EF, bool SHR = false>
__device__ __forceinline__ void forward_tile(const Args& a, Pixel& P, float* lds, const uint8_t* dec, bool more,
                                             v2f& uv_next, const uint8_t* lut_lds = nullptr) {
    TexArg t[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) t[i] = a.tex[i];
    if constexpr ((DEC && MODE != kModeStf) || (EF && NT >= 3)) {
        // With a decoder the exchanging slots run one after another, each
        // from its pick to its stores: the decode and exchange dominate a
        // slot, and carrying every slot's pick through the others' passes (as
        // below) kept them in scratch memory once the compiler left the slot
        // loop rolled (one-tap STF keeps the overlapped fetches below). The
        // same holds for exact filtering with three or four textures (four:
        // 361 -> 153 us at 1080p; two keep the overlapped form, 68 vs 90 us).
        SelCtx<FILT> ctx;
        BinGeom<AxisCtx<FILT>::N> geom;
        uint4 hq;
        uint32_t hxs[NT], hys[NT];
        static_for<NT>([&](auto I) {
            constexpr int i = decltype(I)::value;
            uint32_t hx, hy;
            slot_uniforms(a, P, i, hq, hx, hy);
            ctx.update(P, t[i].w, t[i].h);
#pragma unroll
            for (int j = 0; j < i; ++j) {            // shared selection, as below
                const bool lead = a.leader[i] == j;
                hx = lead ? hxs[j] : hx;
                hy = lead ? hys[j] : hy;
            }
            hxs[i] = hx;
            hys[i] = hy;
            const SlotPick pk = pick_slot<FILT>(t[i], ctx, hx, hy);
            if (i == 0 && more) uv_next = load_uv(a, P.px, P.py + kTile);
            if constexpr (MODE == kModeBins) update_geom<FILT>(geom, P, ctx, t[i].w, t[i].h);
            switch (payload_of(t[i].fmt)) {
            case kF16x4: slot_pass<FILT, MODE, kF16x4, false, EF>(a, t[i], i, P, ctx, geom, pk, lds); break;
            case kF16x2: slot_pass<FILT, MODE, kF16x2, false, EF>(a, t[i], i, P, ctx, geom, pk, lds); break;
            case kF32x1: slot_pass<FILT, MODE, kF32x1, false, EF>(a, t[i], i, P, ctx, geom, pk, lds); break;
            case kLatent: slot_pass<FILT, MODE, kF32x4, true, EF>(a, t[i], i, P, ctx, geom, pk, lds, dec); break;
            default: slot_pass<FILT, MODE, kF32x4, false, EF>(a, t[i], i, P, ctx, geom, pk, lds); break;
            }
        });
        return;
    }
    SelCtx<FILT> ctx;
    SlotPick pk[NT];
    uint4 hq;
    uint32_t hxs[NT], hys[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        uint32_t hx, hy;
        slot_uniforms(a, P, i, hq, hx, hy);
        ctx.update(P, t[i].w, t[i].h);
        // shared selection: the leader, an earlier slot of this texture's
        // size, picks the same texel here with its own random numbers. They
        // are selected value by value (copying the leader's whole pick under
        // a runtime slot index made the compiler keep every pick in scratch
        // memory).
#pragma unroll
        for (int j = 0; j < i; ++j) {
            const bool lead = a.leader[i] == j;
            hx = lead ? hxs[j] : hx;
            hy = lead ? hys[j] : hy;
        }
        hxs[i] = hx;
        hys[i] = hy;
        pk[i] = pick_slot<FILT>(t[i], ctx, hx, hy);
    }
    if (more) uv_next = load_uv(a, P.px, P.py + kTile);
    if constexpr (SHR) {                             // ctx: slot 0's size, every slot's
        static_assert((MODE == kModeRecords || MODE == kModeQuad) && !DEC && !EF, "shared selection kernels");
        if constexpr (MODE == kModeQuad) shared_quad_pass<FILT, NT>(a, t, P, ctx, pk);
        else shared_records_pass<FILT, NT>(a, t, P, ctx, pk, lds, lut_lds);
        return;
    }
    BinGeom<AxisCtx<FILT>::N> geom;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        ctx.update(P, t[i].w, t[i].h);
        if constexpr (MODE == kModeBins) update_geom<FILT>(geom, P, ctx, t[i].w, t[i].h);
        switch (payload_of(t[i].fmt)) {
        case kF16x4: slot_pass<FILT, MODE, kF16x4, false, EF>(a, t[i], i, P, ctx, geom, pk[i], lds, nullptr, lut_lds); break;
        case kF16x2: slot_pass<FILT, MODE, kF16x2, false, EF>(a, t[i], i, P, ctx, geom, pk[i], lds, nullptr, lut_lds); break;
        case kF32x1: slot_pass<FILT, MODE, kF32x1, false, EF>(a, t[i], i, P, ctx, geom, pk[i], lds, nullptr, lut_lds); break;
        case kLatent:
            if constexpr (DEC) slot_pass<FILT, MODE, kF32x4, true, EF>(a, t[i], i, P, ctx, geom, pk[i], lds, dec);
            break;
        default: slot_pass<FILT, MODE, kF32x4, false, EF>(a, t[i], i, P, ctx, geom, pk[i], lds, nullptr, lut_lds); break;
        }
    }
}

// One-tap STF without a decoder exchanges nothing between lanes, so it does
// not need 8x8 tiles: its waves take kOneTapPixels<NT> runs of 64 consecutive
// pixels of one screen row, whose UV reads and output writes are contiguous
// (whole cache lines, where an 8x8 tile writes 8-pixel row pieces: half lines
// of RG32F). Each lane carries its pixels through the phases together --
// every UV, then every pick and texel request, then every decode and store
// -- so that a wave has that many times the loads of one pixel in flight.
// Two pixels per lane, one with four textures, whose picks already keep four
// texel requests per pixel in flight (3840x2160: 124 instead of 128 us).
template <int MODE, bool DEC>
constexpr bool kRowLinear = MODE == kModeStf && !DEC;
template <int NT>
constexpr int kOneTapPixels = NT >= 4 ? 1 : 2;
inline int onetap_pixels(int ntex) { return ntex >= 4 ? 1 : 2; }

template <int FILT, int NT, int K>
__device__ __forceinline__ void onetap_pixels(const Args& a, const Pixel (&P)[K]) {
    TexArg t[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) t[i] = a.tex[i];
    SlotPick pk[K][NT];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        SelCtx<FILT> ctx;
        uint4 hq;
        uint32_t hxs[NT], hys[NT];
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            uint32_t hx, hy;
            slot_uniforms(a, P[k], i, hq, hx, hy);
            ctx.update(P[k], t[i].w, t[i].h);
#pragma unroll
            for (int j = 0; j < i; ++j) {            // shared selection, as in forward_tile
                const bool lead = a.leader[i] == j;
                hx = lead ? hxs[j] : hx;
                hy = lead ? hys[j] : hy;
            }
            hxs[i] = hx;
            hys[i] = hy;
            pk[k][i] = pick_slot<FILT>(t[i], ctx, hx, hy);
        }
    }
    SelCtx<FILT> unused;                             // one-tap passes read only the pick
    BinGeom<AxisCtx<FILT>::N> geom;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            switch (payload_of(t[i].fmt)) {
            case kF16x4: slot_pass<FILT, kModeStf, kF16x4>(a, t[i], i, P[k], unused, geom, pk[k][i], nullptr); break;
            case kF16x2: slot_pass<FILT, kModeStf, kF16x2>(a, t[i], i, P[k], unused, geom, pk[k][i], nullptr); break;
            case kF32x1: slot_pass<FILT, kModeStf, kF32x1>(a, t[i], i, P[k], unused, geom, pk[k][i], nullptr); break;
            case kLatent: break;                     // latents need the decoder kernels
            default: slot_pass<FILT, kModeStf, kF32x4>(a, t[i], i, P[k], unused, geom, pk[k][i], nullptr); break;
            }
        }
}

// Workgroup (x, y) filters tile columns 4x .. 4x+3 (one per wave) over tile
// rows kForwardRows<DEC> * y onward; row-linear kernels: pixels
// 256 K x .. 256 K (x + 1) - 1 of screen row y (K = kOneTapPixels<NT>).
template <int FILT, int MODE, int NT, bool DEC, bool EF>
__global__ __launch_bounds__(kThreads, (kForwardWaves<MODE, NT, DEC, EF>)) void forward_kernel(Args a) {
    // per-wave LDS: records or bins; with a decoder also the deduplicating decode's scratch
    constexpr bool kLds = MODE == kModeRecords || MODE == kModeBins || DEC;
    static_assert(kDedupBytes <= kLdsFloatsPerWave * 4, "decode scratch exceeds the wave's LDS");
    __shared__ __align__(16) float lds_all[kLds ? kWavesPerGroup * kLdsFloatsPerWave : 4];
    __shared__ __align__(16) uint8_t dec[DEC ? kDecBytes : 16];
    // record footprints without a decoder: a table of at most kLutStageMax
    // entries per pixel is read from LDS
    constexpr bool kStageLut = MODE == kModeRecords && !DEC;
    __shared__ uint8_t lut_lds[kStageLut ? 64 * kLutStageMax : 1];
    const bool staged = kStageLut && a.footprint == STF_FP_LUT && a.lut_k <= kLutStageMax;
    if constexpr (DEC) {                       // before any wave of the group can leave
        stage_decoder(a.dec, dec);
        __syncthreads();
    }
    if (staged) {                              // uniform over the launch; before any wave can leave
        for (int i = threadIdx.x; i < 64 * a.lut_k; i += kThreads) lut_lds[i] = a.lut[i];
        __syncthreads();
    }
    if constexpr (kRowLinear<MODE, DEC>) {
        constexpr int K = kOneTapPixels<NT>;
        const int x0 = (blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6)) * (64 * K);
        if (x0 >= a.sw) return;                // whole wave off screen
        Pixel P[K];
        v2f uv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            P[k].px = x0 + 64 * k + lane_id();
            P[k].py = blockIdx.y;
            P[k].lx = P[k].ly = P[k].q = 0;    // no tile: nothing is exchanged
            P[k].valid = P[k].px < a.sw;
            uv[k] = load_uv(a, P[k].px, P[k].py);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            P[k].u = uv[k].x;
            P[k].v = uv[k].y;
        }
        onetap_pixels<FILT, NT, K>(a, P);
        return;
    }
    constexpr int kRows = kForwardRows<DEC>;
    const int tx = blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6);
    if (tx * kTile >= a.sw) return;            // whole tile column off screen
    float* lds = lds_all + (kLds ? (threadIdx.x >> 6) * kLdsFloatsPerWave : 0);
    const int ty0 = blockIdx.y * kRows;
    Pixel P;
    place_pixel(a, tx, ty0, P);
    v2f uv = load_uv(a, P.px, P.py);
    if constexpr (kRows == 1) {
        P.u = uv.x;
        P.v = uv.y;
        forward_tile<FILT, MODE, NT, DEC, EF>(a, P, lds, DEC ? dec : nullptr, false, uv, staged ? lut_lds : nullptr);
    } else {
#pragma unroll 1
        for (int k = 0; k < kRows; ++k) {
            const int ty = ty0 + k;
            if (ty * kTile >= a.sh) break;     // wave-uniform
            if (k > 0) place_pixel(a, tx, ty, P);
            P.u = uv.x;
            P.v = uv.y;
            const bool more = k + 1 < kRows && (ty + 1) * kTile < a.sh;
            forward_tile<FILT, MODE, NT, DEC, EF>(a, P, lds, DEC ? dec : nullptr, more, uv, staged ? lut_lds : nullptr);
        }
    }
}

// Record footprints (2x2w, 3x3, 4x4, tables) over two to four textures of
// one size under shared selection: one support test and weight per member
// for every slot. A kernel of its own, so that the independent-selection
// kernels keep their register counts, with its own LDS share per wave; one
// tile per wave, laid out as in forward_kernel.
template <int FILT, int NT>
__global__ __launch_bounds__(kThreads) void shared_records_kernel(Args a) {
    __shared__ __align__(16) float lds_all[kWavesPerGroup * kSharedRecordFloats<NT>];
    __shared__ uint8_t lut_lds[64 * kLutStageMax];
    const bool staged = a.footprint == STF_FP_LUT && a.lut_k <= kLutStageMax;
    if (staged) {                              // uniform over the launch; before any wave can leave
        for (int i = threadIdx.x; i < 64 * a.lut_k; i += kThreads) lut_lds[i] = a.lut[i];
        __syncthreads();
    }
    Pixel P;
    if (!setup_pixel(a, P)) return;
    float* lds = lds_all + (threadIdx.x >> 6) * kSharedRecordFloats<NT>;
    v2f next;                                  // no next tile
    forward_tile<FILT, kModeRecords, NT, false, false, true>(a, P, lds, nullptr, false, next,
                                                             staged ? lut_lds : nullptr);
}

// 2x2 quads over two to four textures of one size under shared selection:
// one support test and weight per partner for every slot (a kernel of its
// own for the same reason).
template <int FILT, int NT>
__global__ __launch_bounds__(kThreads) void shared_quad_kernel(Args a) {
    Pixel P;
    if (!setup_pixel(a, P)) return;
    v2f next;                                  // no next tile
    forward_tile<FILT, kModeQuad, NT, false, false, true>(a, P, nullptr, nullptr, false, next);
}

// ---------------------------------------------------------------- comparison estimators
//
// The estimators Sec. 4.1 evaluates before proposing Eq. (14), over the same
// shared picks: pixel c holds the picks x_i of its footprint's on-screen
// members i (itself included), each drawn from member i's PMF p_i = f_i.
// With w_i = f_c(x_i) / p_i(x_i) and n the number of picks:
//   IS          (1/n) sum_i w_i T_i                                   Eq. (6)
//   MIS         sum_i f_c(x_i) T_i / sum_j p_j(x_i)   (balance heuristic, n^2 PMFs)
//   pairwise    sum_i m_i(x_i) w_i T_i, canonical c:  (2n PMFs)
//     m_i(x) = p_i(x) / ((n-1) p_i(x) + p_c(x)),  m_c(x) = 1/(n-1) sum_{i!=c} p_c(x) / (p_c(x) + (n-1) p_i(x))
//   regression  (1/n) sum_i [w_i T_i - beta (w_i - 1)],
//     beta = sum_i (w_i - wbar) w_i T_i / sum_i (w_i - wbar)^2   (0 when all w_i are equal)   Eq. (7)
//   WIS         Eq. (14) written out plainly (used for its clamped form)
// Clamping limits the result per channel to the range of the texels with
// f_c(x_i) > 0. One wave per tile; each lane publishes its pick, PMF,
// support start, per-axis weights and decoded texel in LDS and every pixel
// walks its members. Comparison only: not the optimised path.

template <int N>
struct PickRecord {                  // LDS record of one lane, 16-byte aligned
    uint32_t s;                      // texel sx | sy << 16
    float p;                         // own PMF at the pick; 0 for off-screen pixels
    int bx, by;                      // support start
    float T[4];
    float wx[N], wy[N];
};

template <int N>
__device__ __forceinline__ float pmf_at(const PickRecord<N>& r, uint32_t s, uint32_t mx, uint32_t my) {
    uint32_t dx, dy;
    if (!support_offset<N>(s, r.bx, r.by, mx, my, dx, dy)) return 0.0f;
    return r.wx[dx] * r.wy[dy];
}

// Texel of any non-latent format as four floats (zero-padded).
__device__ __forceinline__ void texel_f4(const TexArg& t, uint4 raw, float* T) {
#pragma unroll
    for (int c = 0; c < 4; ++c) T[c] = 0.0f;
    switch (payload_of(t.fmt)) {
    case kF16x4: { const Texel<kF16x4> x = decode<kF16x4>(raw, t.fmt); for (int c = 0; c < 4; ++c) T[c] = x.ch(c); break; }
    case kF16x2: { const Texel<kF16x2> x = decode<kF16x2>(raw, t.fmt); T[0] = x.ch(0); T[1] = x.ch(1); break; }
    case kF32x1: { const Texel<kF32x1> x = decode<kF32x1>(raw, t.fmt); T[0] = x.ch(0); break; }
    default: { const Texel<kF32x4> x = decode<kF32x4>(raw, t.fmt); for (int c = 0; c < 4; ++c) T[c] = x.ch(c); break; }
    }
}

template <int FILT>
__device__ __forceinline__ void estimator_slot(const Args& a, int slot, const Pixel& P, const SelCtx<FILT>& ctx,
                                               uint32_t hx, uint32_t hy, float* lds) {
    constexpr int N = SelCtx<FILT>::N;
    const TexArg t = a.tex[slot];
    const uint32_t mx = (uint32_t)t.w - 1u, my = (uint32_t)t.h - 1u;
    const SlotPick pk = pick_slot<FILT>(t, ctx, hx, hy);
    PickRecord<N>* rec = reinterpret_cast<PickRecord<N>*>(lds);
    PickRecord<N> mine;
    mine.s = pk.sx | (pk.sy << 16);
    mine.p = P.valid ? ctx.x.wsel(pk.kx) * ctx.y.wsel(pk.ky) : 0.0f;
    mine.bx = ctx.x.base;
    mine.by = ctx.y.base;
    texel_f4(t, block_texel(pk.raw, pk.sx, format_bytes(t.fmt)), mine.T);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        mine.wx[i] = ctx.x.w(i);
        mine.wy[i] = ctx.y.w(i);
    }
    const int64_t pix = (int64_t)P.py * a.sw + P.px;
    if (a.sel != nullptr && P.valid) {
        int2* sp = reinterpret_cast<int2*>(a.sel) + ((int64_t)slot * a.sh * a.sw + pix);
        *sp = make_int2((int)pk.sx, (int)pk.sy);
    }
    rec[P.q] = mine;
    wave_lds_sync();

    const int fp = a.footprint;
    const int K = fp == STF_FP_SELF ? 0 : footprint_size(fp, a.lut_k);
    const int est = a.estimator;
    // member iteration: the pixel itself first, then the others
    auto member = [&](int m) -> int {                     // m = -1: the pixel itself; -2: skip
        if (m < 0) return P.q;
        const int j = member_id(fp, P.lx, P.ly, m, a.lut, a.lut_k, P.q);
        return j == P.q ? -2 : j;
    };
    // pass 1: n, sum of w, clamp range
    float n = 0.0f, sw = 0.0f;
    float lo[4], hi[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        lo[c] = __builtin_huge_valf();
        hi[c] = -__builtin_huge_valf();
    }
    for (int m = -1; m < K; ++m) {
        const int j = member(m);
        if (j < 0) continue;
        const PickRecord<N>& r = rec[j];
        if (r.p == 0.0f) continue;                        // off-screen member
        n += 1.0f;
        uint32_t dx, dy;
        if (support_offset<N>(r.s, ctx.x.base, ctx.y.base, mx, my, dx, dy)) {
            const float f = ctx.x.wsel(dx) * ctx.y.wsel(dy);
            sw += f / r.p;
            if (f > 0.0f) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    lo[c] = fminf(lo[c], r.T[c]);
                    hi[c] = fmaxf(hi[c], r.T[c]);
                }
            }
        }
    }
    const float wbar = sw / fmaxf(n, 1.0f);
    const float nm1 = fmaxf(n - 1.0f, 1.0f);
    // pairwise MIS: canonical weight m_c(x_c)
    float m_c = 1.0f;
    if (est == STF_EST_PAIRWISE_MIS && n > 1.0f) {
        m_c = 0.0f;
        for (int m = 0; m < K; ++m) {
            const int j = member(m);
            if (j < 0 || rec[j].p == 0.0f) continue;
            m_c += mine.p / (mine.p + nm1 * pmf_at<N>(rec[j], mine.s, mx, my));
        }
        m_c /= nm1;
    }
    // pass 2
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    float dw2 = 0.0f, cv = 0.0f;
    float dwt[4] = {0.f, 0.f, 0.f, 0.f};
    for (int m = -1; m < K; ++m) {
        const int j = member(m);
        if (j < 0) continue;
        const PickRecord<N>& r = rec[j];
        if (r.p == 0.0f) continue;
        uint32_t dx, dy;
        const float f = support_offset<N>(r.s, ctx.x.base, ctx.y.base, mx, my, dx, dy)
                            ? ctx.x.wsel(dx) * ctx.y.wsel(dy) : 0.0f;
        const float w = f / r.p;
        float coef;
        switch (est) {
        case STF_EST_IS: coef = w; break;
        case STF_EST_MIS: {
            float den = 0.0f;                              // sum over all members k of p_k(x_i)
            for (int mm = -1; mm < K; ++mm) {
                const int k = member(mm);
                if (k < 0 || rec[k].p == 0.0f) continue;
                den += pmf_at<N>(rec[k], r.s, mx, my);
            }
            coef = f / den;                                // den >= p_i(x_i) > 0
            break;
        }
        case STF_EST_PAIRWISE_MIS:
            coef = (m < 0 ? m_c : r.p / (nm1 * r.p + f)) * w;
            break;
        case STF_EST_REGRESSION: {
            const float d = w - wbar;
            dw2 = fmaf(d, d, dw2);
            cv += w - 1.0f;
#pragma unroll
            for (int c = 0; c < 4; ++c) dwt[c] = fmaf(d * w, r.T[c], dwt[c]);
            coef = w;
            break;
        }
        default: coef = w; break;                          // WIS numerator
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = fmaf(coef, r.T[c], acc[c]);
    }
    float o[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        switch (est) {
        case STF_EST_IS: o[c] = acc[c] / n; break;
        case STF_EST_MIS: case STF_EST_PAIRWISE_MIS: o[c] = acc[c]; break;
        case STF_EST_REGRESSION: {
            const float beta = dw2 > 0.0f ? dwt[c] / dw2 : 0.0f;
            o[c] = fmaf(-beta, cv, acc[c]) / n;
            break;
        }
        default: o[c] = acc[c] / sw; break;
        }
        if (a.flags & STF_REUSE_CLAMP) o[c] = fminf(fmaxf(o[c], lo[c]), hi[c]);
        if (t.has_scale) o[c] *= t.scale[c];
    }
    wave_lds_sync();                                       // records read before the next slot
    if (P.valid) {
        switch (t.ch) {
        case 4: store_out<4>(a.out[slot], pix, o); break;
        case 2: store_out<2>(a.out[slot], pix, o); break;
        default: store_out<1>(a.out[slot], pix, o); break;
        }
    }
}

template <int FILT>
__global__ __launch_bounds__(kThreads) void estimator_kernel(Args a) {
    __shared__ __align__(16) float lds_all[kWavesPerGroup * kLdsFloatsPerWave];
    static_assert(64 * sizeof(PickRecord<SelCtx<FILT>::N>) <= kLdsFloatsPerWave * sizeof(float),
                  "pick records exceed the wave's LDS");
    Pixel P;
    if (!setup_pixel(a, P)) return;
    float* lds = lds_all + (threadIdx.x >> 6) * kLdsFloatsPerWave;
    SelCtx<FILT> ctx;
    for (int slot = 0; slot < a.ntex; ++slot) {
        uint32_t hx, hy;
        keyed_uniforms(a, P, slot, hx, hy);
        ctx.update(P, a.tex[slot].w, a.tex[slot].h);
        estimator_slot<FILT>(a, slot, P, ctx, hx, hy, lds);
    }
}

// Deterministic filter, Eq. (3): sum over the support of f_c * T.
template <int FILT, int PL, bool LAT = false>
__device__ __forceinline__ void reference_slot(const Args& a, int slot, const Pixel& P, const SelCtx<FILT>& ctx,
                                               const uint8_t* dec = nullptr, uint8_t* scratch = nullptr) {
    constexpr int N = SelCtx<FILT>::N;
    constexpr int C = Texel<PL>::C;
    const TexArg t = a.tex[slot];
    const uint32_t mx = (uint32_t)t.w - 1u, my = (uint32_t)t.h - 1u;
    const int bpp = format_bytes(t.fmt);
    float acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0f;
#pragma unroll
    for (int b = 0; b < N; ++b) {
        const uint32_t y = (uint32_t)(ctx.y.base + b) & my;
#pragma unroll
        for (int aa = 0; aa < N; ++aa) {
            const uint32_t x = (uint32_t)(ctx.x.base + aa) & mx;
            Texel<PL> T;
            if constexpr (LAT)                       // every tap decodes (the full-filter cost)
                decode_latent_dedup(dec, latent_operand(dec, block_texel(fetch_block(t, x, y, bpp), x, bpp), t), x, y, mx, my,
                                    scratch, T.v);
            else
                T = decode<PL>(block_texel(fetch_block(t, x, y, bpp), x, bpp), t.fmt);
            const float w = ctx.wxy[b * N + aa];
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = fmaf(w, T.ch(c), acc[c]);
        }
    }
    if (P.valid) {
        if (!LAT && t.has_scale) {
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] *= t.scale[c];
        }
        store_out<C>(a.out[slot], (int64_t)P.py * a.sw + P.px, acc);
    }
}

template <int FILT, bool DEC>
__global__ __launch_bounds__(kThreads) void reference_kernel(Args a) {
    __shared__ __align__(16) uint8_t dec[DEC ? kDecBytes : 16];
    __shared__ __align__(16) uint8_t dscratch[DEC ? kWavesPerGroup * kDedupBytes : 16];
    if constexpr (DEC) {
        stage_decoder(a.dec, dec);
        __syncthreads();
    }
    Pixel P;
    if (!setup_pixel(a, P)) return;
    SelCtx<FILT> ctx;
    for (int slot = 0; slot < a.ntex; ++slot) {
        ctx.update(P, a.tex[slot].w, a.tex[slot].h);
        switch (payload_of(a.tex[slot].fmt)) {
        case kF16x4: reference_slot<FILT, kF16x4>(a, slot, P, ctx); break;
        case kF16x2: reference_slot<FILT, kF16x2>(a, slot, P, ctx); break;
        case kF32x1: reference_slot<FILT, kF32x1>(a, slot, P, ctx); break;
        case kLatent:
            if constexpr (DEC)
                reference_slot<FILT, kF32x4, true>(a, slot, P, ctx, dec, dscratch + (threadIdx.x >> 6) * kDedupBytes);
            break;
        default: reference_slot<FILT, kF32x4>(a, slot, P, ctx); break;
        }
    }
}


// ---------------------------------------------------------------- launches

// One workgroup per kWavesPerGroup tiles side by side.
inline dim3 grid_of(const Args& a) {
    return dim3((unsigned)((a.sw + kTile * kWavesPerGroup - 1) / (kTile * kWavesPerGroup)),
                (unsigned)((a.sh + kTile - 1) / kTile));
}

// Forward kernels: kForwardRows<DEC> tile rows per workgroup, or 256
// kOneTapPixels<NT> pixels of one screen row.
template <int MODE, bool DEC>
inline dim3 grid_forward(const Args& a) {
    if constexpr (kRowLinear<MODE, DEC>) {
        const int k = onetap_pixels(a.ntex);
        return dim3((unsigned)((a.sw + kThreads * k - 1) / (kThreads * k)), (unsigned)a.sh);
    }
    const int rows = (a.sh + kTile - 1) / kTile;
    return dim3((unsigned)((a.sw + kTile * kWavesPerGroup - 1) / (kTile * kWavesPerGroup)),
                (unsigned)((rows + kForwardRows<DEC> - 1) / kForwardRows<DEC>));
}

template <int FILT, int MODE, bool DEC, bool EF>
void launch_nt(const Args& a, hipStream_t s) {
    const dim3 g = grid_forward<MODE, DEC>(a), b(kThreads);
    if constexpr (MODE == kModeRecords && !DEC && !EF) {
        bool one_pick = a.ntex >= 2;                      // every slot takes slot 0's selection
        for (int i = 1; i < a.ntex; ++i) one_pick = one_pick && a.leader[i] == 0;
        if (one_pick) {
            if (a.ntex == 2) hipLaunchKernelGGL((shared_records_kernel<FILT, 2>), g, b, 0, s, a);
            else if (a.ntex == 3) hipLaunchKernelGGL((shared_records_kernel<FILT, 3>), g, b, 0, s, a);
            else hipLaunchKernelGGL((shared_records_kernel<FILT, 4>), g, b, 0, s, a);
            return;
        }
    }
    if constexpr (MODE == kModeQuad && !DEC && !EF) {
        bool one_pick = a.ntex >= 2;
        for (int i = 1; i < a.ntex; ++i) one_pick = one_pick && a.leader[i] == 0;
        if (one_pick) {
            if (a.ntex == 2) hipLaunchKernelGGL((shared_quad_kernel<FILT, 2>), g, b, 0, s, a);
            else if (a.ntex == 3) hipLaunchKernelGGL((shared_quad_kernel<FILT, 3>), g, b, 0, s, a);
            else hipLaunchKernelGGL((shared_quad_kernel<FILT, 4>), g, b, 0, s, a);
            return;
        }
    }
    switch (a.ntex) {
    case 1: hipLaunchKernelGGL((forward_kernel<FILT, MODE, 1, DEC, EF>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((forward_kernel<FILT, MODE, 2, DEC, EF>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((forward_kernel<FILT, MODE, 3, DEC, EF>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((forward_kernel<FILT, MODE, 4, DEC, EF>), g, b, 0, s, a); break;
    }
}

// Forward launch for one filter and exchange mode. Explicitly instantiated
// in stf_forward_bilinear.hip and stf_forward_bicubic.hip, so the 112
// forward kernels compile in two translation units of their own.
template <int FILT, int MODE>
void launch_forward(const Args& a, hipStream_t s) {
    const bool dec = a.dec != nullptr;
    if constexpr (MODE == kModeStf) {          // one pick: exact filtering changes nothing
        dec ? launch_nt<FILT, MODE, true, false>(a, s) : launch_nt<FILT, MODE, false, false>(a, s);
    } else {
        const bool ef = (a.flags & STF_REUSE_EXACT_FILTERING) != 0;
        if (dec) ef ? launch_nt<FILT, MODE, true, true>(a, s) : launch_nt<FILT, MODE, true, false>(a, s);
        else ef ? launch_nt<FILT, MODE, false, true>(a, s) : launch_nt<FILT, MODE, false, false>(a, s);
    }
}

#define STF_EXTERN_FORWARD(F) \
    extern template void launch_forward<F, kModeStf>(const Args&, hipStream_t); \
    extern template void launch_forward<F, kModeQuad>(const Args&, hipStream_t); \
    extern template void launch_forward<F, kModeRecords>(const Args&, hipStream_t); \
    extern template void launch_forward<F, kModeBins>(const Args&, hipStream_t);
STF_EXTERN_FORWARD(0)
STF_EXTERN_FORWARD(1)
#undef STF_EXTERN_FORWARD

}  // namespace stf
