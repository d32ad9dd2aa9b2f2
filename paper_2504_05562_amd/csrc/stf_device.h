// Device-side building blocks of the STF kernels for gfx950 (wave64).
//
// Tile mapping: one wavefront = one 8x8 screen tile. Lanes are in Morton
// order inside the tile, so lanes 4k..4k+3 form a 2x2 quad (DPP quad_perm
// exchanges) and lanes 16k..16k+15 a 4x4 block.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "stf.h"

namespace stf {

constexpr int kTile = 8;
constexpr int kWavesPerGroup = 4;          // 256-thread workgroup = 4 tiles side by side (32x8 px)
constexpr int kThreads = 64 * kWavesPerGroup;
#ifndef STF_BIN_G
#define STF_BIN_G 12
#endif
constexpr int kBinG = STF_BIN_G;           // texel bins per axis for whole-tile reuse
constexpr int kBins = kBinG * kBinG;
constexpr int kBinStride = kBinG + 1;      // records per bin row (padded: rows fall on different LDS banks)
constexpr int kBinRecords = kBinG * kBinStride;
constexpr uint32_t kGolden = 0x9E3779B9u;

struct TexArg {
    const uint8_t* data;
    int64_t pitch;
    int32_t w, h;
    int32_t fmt;
    int32_t ch;              // channels of the filtered (decoded) texel
    int32_t has_scale;       // per-channel dequantization scale present
    float scale[8];
};

// Args::flags: the stf_reuse flags plus kernel-internal bits.
constexpr int32_t kFlagFloatBinSums = 1 << 8;   // STF_FLOAT_BIN_SUMS: FP32 atomics for the whole-tile sums

struct Args {
    TexArg tex[STF_MAX_TEXTURES];
    float* out[STF_MAX_TEXTURES];
    const float* dout[STF_MAX_TEXTURES];
    const float* uv;
    int32_t* sel;
    const uint8_t* lut;
    const uint8_t* dec;      // packed latent decoder (device), shared by the latent textures
    int32_t ntex, sw, sh, lut_k, footprint, flags, estimator;
    int32_t leader[STF_MAX_TEXTURES];   // slot whose selection each slot uses
    uint32_t seed, frame;
};

// ---------------------------------------------------------------- lanes

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Morton lane -> tile pixel (lx, ly): lx takes lane bits 0,2,4; ly bits 1,3,5.
__device__ __forceinline__ void lane_pixel(int lane, int& lx, int& ly) {
    lx = (lane & 1) | ((lane >> 1) & 2) | ((lane >> 2) & 4);
    ly = ((lane >> 1) & 1) | ((lane >> 2) & 2) | ((lane >> 3) & 4);
}

// Wave-local LDS ordering: LDS instructions of one wavefront execute in
// order, so a compiler fence at wavefront scope is all that is needed
// between a store by one lane and a load of the same word by another lane.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- hash

// pcg4d of Jarzynski and Olano (JCGT 2020), all arithmetic modulo 2^32.
__device__ __forceinline__ uint4 pcg4d(uint4 v) {
    v.x = v.x * 1664525u + 1013904223u;
    v.y = v.y * 1664525u + 1013904223u;
    v.z = v.z * 1664525u + 1013904223u;
    v.w = v.w * 1664525u + 1013904223u;
    v.x += v.y * v.w; v.y += v.z * v.x; v.z += v.x * v.y; v.w += v.y * v.z;
    v.x ^= v.x >> 16; v.y ^= v.y >> 16; v.z ^= v.z >> 16; v.w ^= v.w >> 16;
    v.x += v.y * v.w; v.y += v.z * v.x; v.z += v.x * v.y; v.w += v.y * v.z;
    return v;
}

// ---------------------------------------------------------------- coordinates

// Texel-space coordinate x = u * size - 0.5 in FP32 with two roundings
// (Sec. 4.5 listing), split into integer texel i0 = floor(x) and the 16-bit
// fraction F = floor(2^16 (x - i0)) computed exactly as
// floor(2^16 x) - 2^16 floor(x) (both terms are exact FP32 integers).
__device__ __forceinline__ void texel_split(float u, int size, int& i0, int& F) {
#pragma clang fp contract(off)
    const float x = u * (float)size - 0.5f;
    const float fl = floorf(x);
    const float X = floorf(__fmul_rn(x, 65536.0f));
    F = (int)__fsub_rn(X, __fmul_rn(fl, 65536.0f)) & 0xFFFF;
    i0 = (int)fl;
}

// ---------------------------------------------------------------- filters

// Per-axis selection context of one pixel for one texture size: first
// texel of the filter support, per-axis weights and the integer CDF
// thresholds. Textures of equal size share it.
template <int FILT> struct AxisCtx;

// Bilinear (tent): texels i0, i0+1 with weights 1-phi, phi (the per-axis
// factor of GetFilterPMF, Sec. S6). Offset 1 is picked iff
// h >= (1-phi) 2^32, i.e. (h >> 16) >= 2^16 - F: probability exactly phi.
template <> struct AxisCtx<STF_BILINEAR> {
    static constexpr int N = 2;
    int base;            // first texel of the support (unwrapped)
    uint32_t G;          // 2^16 - F
    float w0, w1;        // scalars, not an array: lane-varying selection stays in registers
    __device__ __forceinline__ void init(float u, int size) {
        int i0, F;
        texel_split(u, size, i0, F);
        base = i0;
        G = 65536u - (uint32_t)F;
        w0 = (float)G * (1.0f / 65536.0f);
        w1 = (float)F * (1.0f / 65536.0f);
    }
    __device__ __forceinline__ int pick(uint32_t h) const { return (int)((h >> 16) >= G); }
    __device__ __forceinline__ float w(int i) const { return i == 0 ? w0 : w1; }       // constant i
    __device__ __forceinline__ float wsel(uint32_t k) const { return k ? w1 : w0; }   // lane-varying k
};

// Uniform cubic B-spline (Sec. 5.4): texels i0-1..i0+2. Multiplied by
// 6 * 2^48 the weights are the integers
//   G^3, 3F^3 - 6*2^16 F^2 + 4*2^48, 6*2^48 - (others), F^3   (G = 2^16 - F),
// all below 2^53 and therefore exact in FP64. The offset is the number of
// cumulative weights that h * 6 * 2^16 (exact, < 2^51) reaches.
template <> struct AxisCtx<STF_BICUBIC_BSPLINE> {
    static constexpr int N = 4;
    int base;
    double c0, c01, c012;   // cumulative integer weights
    float w0, w1, w2, w3;
    __device__ __forceinline__ void init(float u, int size) {
        int i0, F;
        texel_split(u, size, i0, F);
        base = i0 - 1;
        const double f = (double)F;
        const double g = 65536.0 - f;
        const double f2 = f * f;
        const double c3 = f2 * f;
        c0 = g * g * g;
        const double c1 = fma(3.0, c3, fma(-393216.0, f2, 1125899906842624.0));   // + 4 * 2^48
        const double total = 1688849860263936.0;                                  // 6 * 2^48
        c01 = c0 + c1;
        c012 = total - c3;
        const double s = 1.0 / total;
        w0 = (float)(c0 * s);
        w1 = (float)(c1 * s);
        w2 = (float)((c012 - c01) * s);
        w3 = (float)(c3 * s);
    }
    __device__ __forceinline__ int pick(uint32_t h) const {
        const double hs = (double)h * 393216.0;
        return (int)(hs >= c0) + (int)(hs >= c01) + (int)(hs >= c012);
    }
    __device__ __forceinline__ float w(int i) const { return i == 0 ? w0 : i == 1 ? w1 : i == 2 ? w2 : w3; }
    __device__ __forceinline__ float wsel(uint32_t k) const {
        const float lo = (k & 1u) ? w1 : w0;
        const float hi = (k & 1u) ? w3 : w2;
        return (k & 2u) ? hi : lo;
    }
};

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------- texels

// clang vector types for the non-temporal load/store builtins
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

// Half-precision value of the low 16 bits (exact in FP32). Written as a
// conversion of a _Float16 so that fmaf(w, h2f(x), acc) compiles to one
// v_fma_mix_f32 that reads the half operand directly.
__device__ __forceinline__ float h2f(uint32_t bits16) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(bits16 & 0xFFFFu));
}

// Texel payload kinds. F16x4 / F16x2 keep the raw half bits (exchanged and
// binned as stored); F32x4 / F32x1 decode at fetch (RGBA8, RGBA32F, BF16,
// FP8 / R8, R32F). Latent textures are decoded by the MLP to F32x4.
enum Payload { kF16x4 = 0, kF16x2 = 1, kF32x4 = 2, kF32x1 = 3, kLatent = 4 };

template <int P> struct Texel;
// C channels; W 32-bit words of payload (word(k) its bits).
template <> struct Texel<kF16x4> {
    static constexpr int C = 4, W = 2;
    uint2 raw;
    __device__ __forceinline__ float ch(int c) const {
        return h2f(c < 2 ? (raw.x >> (16 * c)) : (raw.y >> (16 * (c - 2))));
    }
    __device__ __forceinline__ uint32_t word(int k) const { return k ? raw.y : raw.x; }
};
template <> struct Texel<kF16x2> {
    static constexpr int C = 2, W = 1;
    uint32_t raw;
    __device__ __forceinline__ float ch(int c) const { return h2f(raw >> (16 * c)); }
    __device__ __forceinline__ uint32_t word(int) const { return raw; }
};
template <> struct Texel<kF32x4> {
    static constexpr int C = 4, W = 4;
    float v[4];
    __device__ __forceinline__ float ch(int c) const { return v[c]; }
    __device__ __forceinline__ uint32_t word(int k) const { return __float_as_uint(v[k]); }
};
template <> struct Texel<kF32x1> {
    static constexpr int C = 1, W = 1;
    float v[1];
    __device__ __forceinline__ float ch(int) const { return v[0]; }
    __device__ __forceinline__ uint32_t word(int) const { return __float_as_uint(v[0]); }
};

__device__ __forceinline__ int format_bytes(int fmt) {
    switch (fmt) {
    case STF_R8_UNORM: return 1;
    case STF_RGBA16F: case STF_RGBA_BF16: case STF_LATENT8_FP8: return 8;
    case STF_RGBA32F: case STF_LATENT8_F16: case STF_LATENT8_BF16: return 16;
    default: return 4;               // RGBA8, RG16F, R32F, RGBA FP8
    }
}

// OCP FP8 E4M3 code (low 8 bits) to FP32, from the format definition:
// exponent bias 7, exponent 0 subnormal (m * 2^-9), S.1111.111 NaN.
__device__ __forceinline__ float fp8_e4m3(uint32_t code) {
    const uint32_t c = code & 0xFFu;
    const uint32_t e = (c >> 3) & 0xFu, m = c & 7u;
    const uint32_t sign = (c & 0x80u) << 24;
    const float normal = __uint_as_float(sign | ((e + 120u) << 23) | (m << 20));
    const float sub = __uint_as_float(__float_as_uint((float)m * 0.001953125f) | sign);
    const float v = (e == 0u) ? sub : normal;
    return (e == 15u && m == 7u) ? __uint_as_float(0x7FC00000u) : v;
}

__device__ __forceinline__ float bf16_bits(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

// One texel's payload as stored (1, 4, 8 or 16 bytes), zero-extended.
__device__ __forceinline__ uint4 fetch_raw(const TexArg& t, uint32_t x, uint32_t y) {
    const uint8_t* row = t.data + (int64_t)y * t.pitch;
    switch (format_bytes(t.fmt)) {
    case 1: return make_uint4(row[x], 0u, 0u, 0u);
    case 8: { const uint2 q = *reinterpret_cast<const uint2*>(row + (size_t)x * 8); return make_uint4(q.x, q.y, 0u, 0u); }
    case 16: return *reinterpret_cast<const uint4*>(row + (size_t)x * 16);
    default: return make_uint4(*reinterpret_cast<const uint32_t*>(row + (size_t)x * 4), 0u, 0u, 0u);
    }
}

// The aligned 16-byte block holding texel (x, y): one load instruction for
// every format, so the loads of several textures issue back to back with
// no control flow between them. In bounds because pitch and base address
// are multiples of 16 (validated on the host): the block starts at the
// largest multiple of 16 not above the texel's row offset, which is at
// most pitch - 16.
__device__ __forceinline__ uint4 fetch_block(const TexArg& t, uint32_t x, uint32_t y, int bpp) {
    const uint32_t off = (x * (uint32_t)bpp) & ~15u;
    return *reinterpret_cast<const uint4*>(t.data + (int64_t)y * t.pitch + off);
}

// The texel's payload inside its block (zero-extended).
__device__ __forceinline__ uint4 block_texel(uint4 b, uint32_t x, int bpp) {
    const uint32_t o = (x * (uint32_t)bpp) & 15u;
    const uint32_t lo = (o & 8u) ? b.z : b.x;
    const uint32_t hi = (o & 8u) ? b.w : b.y;
    switch (bpp) {
    case 16: return b;
    case 8: return make_uint4(lo, hi, 0u, 0u);
    case 4: return make_uint4((o & 4u) ? hi : lo, 0u, 0u, 0u);
    default: return make_uint4((((o & 4u) ? hi : lo) >> (8u * (o & 3u))) & 0xFFu, 0u, 0u, 0u);
    }
}

// Texel of payload kind P from the raw payload of a texel of format fmt.
template <int P>
__device__ __forceinline__ Texel<P> decode(uint4 q, int fmt) {
    Texel<P> r;
    if constexpr (P == kF16x4) {
        r.raw = make_uint2(q.x, q.y);
    } else if constexpr (P == kF16x2) {
        r.raw = q.x;
    } else if constexpr (P == kF32x4) {
        if (fmt == STF_RGBA8_UNORM) {
            r.v[0] = (float)(q.x & 0xFF) * (1.0f / 255.0f);
            r.v[1] = (float)((q.x >> 8) & 0xFF) * (1.0f / 255.0f);
            r.v[2] = (float)((q.x >> 16) & 0xFF) * (1.0f / 255.0f);
            r.v[3] = (float)(q.x >> 24) * (1.0f / 255.0f);
        } else if (fmt == STF_RGBA_BF16) {
            r.v[0] = bf16_bits(q.x & 0xFFFFu); r.v[1] = bf16_bits(q.x >> 16);
            r.v[2] = bf16_bits(q.y & 0xFFFFu); r.v[3] = bf16_bits(q.y >> 16);
        } else if (fmt == STF_RGBA_FP8) {
            r.v[0] = fp8_e4m3(q.x); r.v[1] = fp8_e4m3(q.x >> 8);
            r.v[2] = fp8_e4m3(q.x >> 16); r.v[3] = fp8_e4m3(q.x >> 24);
        } else {
            r.v[0] = __uint_as_float(q.x); r.v[1] = __uint_as_float(q.y);
            r.v[2] = __uint_as_float(q.z); r.v[3] = __uint_as_float(q.w);
        }
    } else {
        r.v[0] = (fmt == STF_R8_UNORM) ? (float)(q.x & 0xFF) * (1.0f / 255.0f) : __uint_as_float(q.x);
    }
    return r;
}

template <int P>
__device__ __forceinline__ Texel<P> fetch(const TexArg& t, uint32_t x, uint32_t y) {
    return decode<P>(fetch_raw(t, x, y), t.fmt);
}

template <int C>
__device__ __forceinline__ void store_out(float* out, int64_t pix, const float* v) {
    float* p = out + pix * C;
    if constexpr (C == 4) {
        v4f q = {v[0], v[1], v[2], v[3]};
        __builtin_nontemporal_store(q, reinterpret_cast<v4f*>(p));
    } else if constexpr (C == 2) {
        v2f q = {v[0], v[1]};
        __builtin_nontemporal_store(q, reinterpret_cast<v2f*>(p));
    } else {
        __builtin_nontemporal_store(v[0], p);
    }
}

// ---------------------------------------------------------------- DPP

// Bitwise OR of v over the 64 lanes of the wavefront (DPP within rows of
// 16 lanes, then the four row results).
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);   // row_half_mirror
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);   // row_mirror
    return (uint32_t)(__builtin_amdgcn_readlane((int)v, 0) | __builtin_amdgcn_readlane((int)v, 16) |
                      __builtin_amdgcn_readlane((int)v, 32) | __builtin_amdgcn_readlane((int)v, 48));
}

// Minimum of v over the 64 lanes of the wavefront (same pattern).
__device__ __forceinline__ int wave_min(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Value of `v` held by lane (lane ^ X) within the same quad of 4 lanes.
template <int X>
__device__ __forceinline__ float quad_xor(float v) {
    constexpr int ctrl = (X == 1) ? 0xB1 : (X == 2) ? 0x4E : 0x1B;   // quad_perm patterns
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xF, 0xF, false));
}
template <int X>
__device__ __forceinline__ uint32_t quad_xor(uint32_t v) {
    constexpr int ctrl = (X == 1) ? 0xB1 : (X == 2) ? 0x4E : 0x1B;
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, 0xF, 0xF, false);
}

}  // namespace stf
