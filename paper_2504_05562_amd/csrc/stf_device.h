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
constexpr int kBinG = 16;                  // texel bins per axis for whole-tile reuse
constexpr int kBins = kBinG * kBinG;
constexpr uint32_t kGolden = 0x9E3779B9u;

struct TexArg {
    const uint8_t* data;
    int64_t pitch;
    int32_t w, h;
    int32_t fmt;
    int32_t ch;
};

struct Args {
    TexArg tex[STF_MAX_TEXTURES];
    float* out[STF_MAX_TEXTURES];
    const float* dout[STF_MAX_TEXTURES];
    const float* uv;
    int32_t* sel;
    const uint8_t* lut;
    int32_t ntex, sw, sh, lut_k, footprint;
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

// Two uniforms for pixel (px, py) and texture slot `slot`: slots 2q and
// 2q+1 share one pcg4d evaluation keyed with seed + q * golden.
__device__ __forceinline__ uint2 slot_hash(uint32_t px, uint32_t py, int slot, uint32_t seed, uint32_t frame) {
    uint4 h = pcg4d(make_uint4(px, py, frame, seed + (uint32_t)(slot >> 1) * kGolden));
    return (slot & 1) ? make_uint2(h.z, h.w) : make_uint2(h.x, h.y);
}

// ---------------------------------------------------------------- coordinates

// Texel-space coordinate x = u * size - 0.5 in FP32 with two roundings
// (Sec. 4.5 listing), split into integer texel i0 = floor(x) and the 16-bit
// fraction F = floor(2^16 (x - i0)) computed exactly as
// floor(2^16 x) - 2^16 floor(x) (both terms are exact FP32 integers).
__device__ __forceinline__ void texel_split(float u, int size, int& i0, int& F) {
    const float x = __fsub_rn(__fmul_rn(u, (float)size), 0.5f);
    const float fl = floorf(x);
    const float X = floorf(__fmul_rn(x, 65536.0f));
    F = (int)__fsub_rn(X, __fmul_rn(fl, 65536.0f)) & 0xFFFF;
    i0 = (int)fl;
}

// ---------------------------------------------------------------- filters

// Per-axis support size, offset of the first texel, selection and weights.
template <int FILT> struct Filter;

// Bilinear (tent): texels i0, i0+1 with weights 1-phi, phi (the per-axis
// factor of GetFilterPMF, Sec. S6). Offset 1 is picked iff
// h >= (1-phi) 2^32, i.e. (h >> 16) >= 2^16 - F: probability exactly phi.
template <> struct Filter<STF_BILINEAR> {
    static constexpr int N = 2;
    static constexpr int DELTA = 0;
    __device__ __forceinline__ static int pick(uint32_t h, int F, float* w) {
        const int G = 65536 - F;
        w[0] = (float)G * (1.0f / 65536.0f);
        w[1] = (float)F * (1.0f / 65536.0f);
        return (int)((h >> 16) >= (uint32_t)G);
    }
};

// Uniform cubic B-spline (Sec. 5.4): texels i0-1..i0+2. Multiplied by
// 6 * 2^48 the weights are the integers
//   G^3, 3F^3 - 6*2^16 F^2 + 4*2^48, 6*2^48 - (others), F^3   (G = 2^16 - F),
// all below 2^53 and therefore exact in FP64. The offset is the number of
// cumulative weights that h * 6 * 2^16 (exact, < 2^51) reaches.
template <> struct Filter<STF_BICUBIC_BSPLINE> {
    static constexpr int N = 4;
    static constexpr int DELTA = 1;
    __device__ __forceinline__ static int pick(uint32_t h, int F, float* w) {
        const double f = (double)F;
        const double g = (double)(65536 - F);
        const double f2 = f * f;
        const double c3 = f2 * f;
        const double c0 = g * g * g;
        const double c1 = 3.0 * c3 - 393216.0 * f2 + 1125899906842624.0;   // + 4 * 2^48
        const double total = 1688849860263936.0;                             // 6 * 2^48
        const double c01 = c0 + c1;
        const double c012 = total - c3;
        const double hs = (double)h * 393216.0;
        const int k = (int)(hs >= c0) + (int)(hs >= c01) + (int)(hs >= c012);
        const double s = 1.0 / total;
        w[0] = (float)(c0 * s);
        w[1] = (float)(c1 * s);
        w[2] = (float)((c012 - c01) * s);
        w[3] = (float)(c3 * s);
        return k;
    }
};

// ---------------------------------------------------------------- texels

template <int C> struct Texel { float v[C]; };

// clang vector types for the non-temporal load/store builtins
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

// Decode one texel of slot descriptor t at canonical (x, y). C is the
// channel count of the format (validated on the host).
template <int C>
__device__ __forceinline__ Texel<C> fetch(const TexArg& t, uint32_t x, uint32_t y) {
    Texel<C> r;
    const uint8_t* row = t.data + (int64_t)y * t.pitch;
    if constexpr (C == 4) {
        if (t.fmt == STF_RGBA16F) {
            const uint2 q = *reinterpret_cast<const uint2*>(row + (size_t)x * 8);
            r.v[0] = __half2float(__ushort_as_half((unsigned short)(q.x & 0xFFFF)));
            r.v[1] = __half2float(__ushort_as_half((unsigned short)(q.x >> 16)));
            r.v[2] = __half2float(__ushort_as_half((unsigned short)(q.y & 0xFFFF)));
            r.v[3] = __half2float(__ushort_as_half((unsigned short)(q.y >> 16)));
        } else if (t.fmt == STF_RGBA8_UNORM) {
            const uint32_t q = *reinterpret_cast<const uint32_t*>(row + (size_t)x * 4);
            r.v[0] = (float)(q & 0xFF) * (1.0f / 255.0f);
            r.v[1] = (float)((q >> 8) & 0xFF) * (1.0f / 255.0f);
            r.v[2] = (float)((q >> 16) & 0xFF) * (1.0f / 255.0f);
            r.v[3] = (float)(q >> 24) * (1.0f / 255.0f);
        } else {
            const float4 q = *reinterpret_cast<const float4*>(row + (size_t)x * 16);
            r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
        }
    } else if constexpr (C == 2) {
        const uint32_t q = *reinterpret_cast<const uint32_t*>(row + (size_t)x * 4);
        r.v[0] = __half2float(__ushort_as_half((unsigned short)(q & 0xFFFF)));
        r.v[1] = __half2float(__ushort_as_half((unsigned short)(q >> 16)));
    } else {
        if (t.fmt == STF_R8_UNORM) {
            r.v[0] = (float)row[x] * (1.0f / 255.0f);
        } else {
            r.v[0] = *reinterpret_cast<const float*>(row + (size_t)x * 4);
        }
    }
    return r;
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
