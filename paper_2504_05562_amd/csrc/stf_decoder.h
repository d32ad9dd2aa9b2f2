// Latent-texture decoder on the gfx950 matrix cores.
//
// A latent texel (8 channels) is decoded to RGBA by the MLP
//     h1 = ReLU(W1 x + b1)   (8 -> 64)
//     h2 = ReLU(W2 h1 + b2)  (64 -> 64)
//     y  = W3 h2 + b3        (64 -> 4)
// the neural-texture setting the paper motivates stochastic filtering with
// (Sec. 1, Sec. 5.6): each pixel decodes only the one texel it picked, and
// sample reuse then shares the decoded colours (Sec. 4).
//
// One wavefront decodes the 64 texels its lanes picked at once, as three
// matrix products with the pixels as columns: H^T = W X^T. Every product
// is a chain of v_mfma_f32_32x32x16_bf16 (BF16 operands, FP32 accumulation)
// over two column tiles of 32 pixels:
//   - layer 1: K = 16 = 8 latents (lanes 0-31 of the B operand) + a
//     constant 1 that carries b1 (lanes 32-63); 2 row tiles;
//   - layer 2: K = 64 in 4 steps, 2 row tiles, b2 preloaded in the
//     accumulators;
//   - layer 3: the 4 outputs padded to one 32-row tile, b3 preloaded.
// The accumulator layout of one product (lane l holds rows 8i + 4(l/32) + r,
// i, r in 0..3, of column l % 32) is consumed directly as the B operand of
// the next: lane l contributes the 8 rows it holds as its 8 K-values, which
// permutes K; the packed weights carry the same permutation, so activations
// never move between lanes. Activations are rounded to BF16 (RN) between
// layers; ReLU commutes with that rounding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Packed decoder (device memory written by the pack kernel, staged into LDS
// by every workgroup that decodes): a 16-byte header (precision, per-layer
// weight scales), then the A operands stored lane-major (operand o occupies
// 64 lanes x 16 bytes for BF16, 64 lanes x 8 bytes for FP8) and the FP32
// accumulator start values (biases).
struct DecHeader {
    uint32_t precision;                          // STF_DECODER_BF16 or STF_DECODER_FP8
    float scale[3];                              // FP8: W_l = scale_l * W_l(stored); BF16: 1
};
constexpr int kDecHead = 16;
// BF16 layout
constexpr int kDecA1 = kDecHead;                 // [2 row tiles]; b1 folded in as K index 8
constexpr int kDecA2 = kDecA1 + 2 * 1024;        // [2 row tiles][4 K steps]
constexpr int kDecA3 = kDecA2 + 8 * 1024;        // [4 K steps]
constexpr int kDecC2 = kDecA3 + 4 * 1024;        // f32 [2 row tiles][2 lane halves][16] layer-2 bias
constexpr int kDecC3 = kDecC2 + 2 * 2 * 16 * 4;  // f32 [2 lane halves][16] layer-3 bias
constexpr int kDecBytes = kDecC3 + 2 * 16 * 4;   // 14736
// FP8 layout (biases over the layer's weight scale, so s * (C + W x) = b + s W x)
constexpr int kF8A1 = kDecHead;                  // [2 row tiles]
constexpr int kF8A2 = kF8A1 + 2 * 512;           // [2 row tiles][4 K steps]
constexpr int kF8A3 = kF8A2 + 8 * 512;           // [4 K steps]
constexpr int kF8C1 = kF8A3 + 4 * 512;           // f32 [2][2][16] layer-1 bias / s1
constexpr int kF8C2 = kF8C1 + 2 * 2 * 16 * 4;    // f32 [2][2][16] layer-2 bias / s2
constexpr int kF8C3 = kF8C2 + 2 * 2 * 16 * 4;    // f32 [2][16] layer-3 bias / s3
constexpr int kF8Bytes = kF8C3 + 2 * 16 * 4;
static_assert(kDecBytes % 16 == 0 && kF8Bytes <= kDecBytes, "packed decoder layout");

// Hidden unit carried by K index k of K step s of layers 2 and 3: step
// s = 2 m + g reads accumulator registers 8g..8g+7 of row tile m, and the
// lane half h = k / 8 holds rows 8i + 4h + r there (t = k % 8 = 4q + r,
// i = 2g + q).
__host__ __device__ constexpr int dec_unit(int s, int k) {
    return 32 * (s >> 1) + 16 * (s & 1) + 8 * ((k & 7) >> 2) + 4 * (k >> 3) + (k & 3);
}

// Row of accumulator register j held by lane half h (32x32 output tile).
__host__ __device__ constexpr int acc_row(int j, int h) { return 8 * (j >> 2) + 4 * h + (j & 3); }

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    const f32x2 f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
}

__device__ __forceinline__ f32x16 mfma_bf16(u32x4 a, u32x4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// Value of v held by lane l ^ 32.
__device__ __forceinline__ uint32_t from_other_half(uint32_t v) { return (uint32_t)__shfl_xor((int)v, 32, 64); }

typedef short i16x2 __attribute__((ext_vector_type(2)));

// B operand of the next layer from accumulators: round to BF16, ReLU, and
// take registers 8g..8g+7 as the lane's 8 K values. ReLU acts on the BF16
// bit patterns as a signed 16-bit maximum with 0 (every value with the sign
// bit set, -0 included, becomes +0; others are unchanged), one packed
// instruction per two values; rounding first is equivalent because round to
// nearest preserves the sign.
__device__ __forceinline__ u32x4 relu_pack(const f32x16& d, int g) {
    u32x4 r;
    const i16x2 zero = {0, 0};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const i16x2 v = __builtin_bit_cast(i16x2, pack_bf16(d[8 * g + 2 * t], d[8 * g + 2 * t + 1]));
        r[t] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, zero));
    }
    return r;
}

// One column tile (32 pixels) through the three layers; returns the tile's
// output accumulators (rows 0-3 are the outputs).
__device__ __forceinline__ f32x16 decode_columns(const uint8_t* dec, u32x4 x, int lane, bool hi) {
    const u32x4* A = reinterpret_cast<const u32x4*>(dec);
    const f32x16 zero = {};
    u32x4 b2[4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const f32x16 d = mfma_bf16(A[(kDecA1 >> 4) + m * 64 + lane], x, zero);
        b2[2 * m] = relu_pack(d, 0);
        b2[2 * m + 1] = relu_pack(d, 1);
    }
    const float* C2 = reinterpret_cast<const float*>(dec + kDecC2);
    u32x4 b3[4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const float* cb = C2 + (m * 2 + (hi ? 1 : 0)) * 16;
        f32x16 d;
#pragma unroll
        for (int j = 0; j < 16; ++j) d[j] = cb[j];
#pragma unroll
        for (int s = 0; s < 4; ++s) d = mfma_bf16(A[(kDecA2 >> 4) + (m * 4 + s) * 64 + lane], b2[s], d);
        b3[2 * m] = relu_pack(d, 0);
        b3[2 * m + 1] = relu_pack(d, 1);
    }
    const float* C3 = reinterpret_cast<const float*>(dec + kDecC3) + (hi ? 16 : 0);
    f32x16 y;
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = C3[j];
#pragma unroll
    for (int s = 0; s < 4; ++s) y = mfma_bf16(A[(kDecA3 >> 4) + s * 64 + lane], b3[s], y);
    return y;
}

typedef uint64_t u64;

__device__ __forceinline__ f32x16 mfma_fp8(u64 a, u64 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8((long)a, (long)b, c, 0, 0, 0);
}

// FP8 B operand from accumulators: scale, ReLU, round to FP8 E4M3 (RN), and
// take registers 8g..8g+7 as the lane's 8 K values (byte t = K value t).
__device__ __forceinline__ u64 relu_pack_fp8(const f32x16& d, int g, float s) {
    uint32_t w[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = 8 * g + 4 * h;
        int v = __builtin_amdgcn_cvt_pk_fp8_f32(fmaxf(d[j] * s, 0.0f), fmaxf(d[j + 1] * s, 0.0f), 0, false);
        v = __builtin_amdgcn_cvt_pk_fp8_f32(fmaxf(d[j + 2] * s, 0.0f), fmaxf(d[j + 3] * s, 0.0f), v, true);
        w[h] = (uint32_t)v;
    }
    return (u64)w[0] | ((u64)w[1] << 32);
}

__device__ __forceinline__ f32x16 load_acc(const float* c) {
    f32x16 d;
#pragma unroll
    for (int j = 0; j < 16; ++j) d[j] = c[j];
    return d;
}

// One column tile through the three layers on v_mfma_f32_32x32x16_fp8_fp8
// (same operand layouts as the BF16 path, 8 one-byte K values per lane):
// x holds the 8 FP8 latents in lanes 0-31 and zeros in lanes 32-63 (b1 is
// a start value here). Returns y = s3 (C3 + W3 h2) in rows 0-3.
__device__ __forceinline__ f32x16 decode_columns_fp8(const uint8_t* dec, u64 x, int lane, bool hi) {
    const DecHeader* hd = reinterpret_cast<const DecHeader*>(dec);
    const u64* A1 = reinterpret_cast<const u64*>(dec + kF8A1);
    const u64* A2 = reinterpret_cast<const u64*>(dec + kF8A2);
    const u64* A3 = reinterpret_cast<const u64*>(dec + kF8A3);
    const int half = hi ? 1 : 0;
    u64 b2[4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const f32x16 d = mfma_fp8(A1[m * 64 + lane], x,
                                  load_acc(reinterpret_cast<const float*>(dec + kF8C1) + (m * 2 + half) * 16));
        b2[2 * m] = relu_pack_fp8(d, 0, hd->scale[0]);
        b2[2 * m + 1] = relu_pack_fp8(d, 1, hd->scale[0]);
    }
    u64 b3[4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        f32x16 d = load_acc(reinterpret_cast<const float*>(dec + kF8C2) + (m * 2 + half) * 16);
#pragma unroll
        for (int s = 0; s < 4; ++s) d = mfma_fp8(A2[(m * 4 + s) * 64 + lane], b2[s], d);
        b3[2 * m] = relu_pack_fp8(d, 0, hd->scale[1]);
        b3[2 * m + 1] = relu_pack_fp8(d, 1, hd->scale[1]);
    }
    f32x16 y = load_acc(reinterpret_cast<const float*>(dec + kF8C3) + half * 16);
#pragma unroll
    for (int s = 0; s < 4; ++s) y = mfma_fp8(A3[s * 64 + lane], b3[s], y);
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] *= hd->scale[2];
    return y;
}

__device__ __forceinline__ bool decoder_is_fp8(const uint8_t* dec) {
    return reinterpret_cast<const DecHeader*>(dec)->precision == STF_DECODER_FP8;
}

// One column tile in the decoder's precision: `x` is the operand of the
// lanes 0-31 (8 BF16 latents, or 8 FP8 latents in its low 8 bytes).
__device__ __forceinline__ f32x16 decode_tile(const uint8_t* dec, u32x4 x, int lane, bool hi) {
    if (decoder_is_fp8(dec)) {
        const u64 b = hi ? 0ull : ((u64)x[0] | ((u64)x[1] << 32));
        return decode_columns_fp8(dec, b, lane, hi);
    }
    const u32x4 one = {0x3F80u, 0u, 0u, 0u};      // BF16 1.0 at k = 8: the b1 column
    return decode_columns(dec, hi ? one : x, lane, hi);
}

// Decode the latent texels of all 64 lanes (`lat`: the lane's 8 latents as
// BF16, element k in bits 16(k%2) of dword k/2). `dec` is the packed
// decoder in LDS. Must be called by all 64 lanes in uniform control flow.
// The two column tiles go through the layers one after the other, which
// keeps one tile's activations live at a time.
__device__ __forceinline__ void decode_latent(const uint8_t* dec, u32x4 lat, float out[4]) {
    const int lane = threadIdx.x & 63;
    const bool hi = lane >= 32;
    u32x4 other;
#pragma unroll
    for (int i = 0; i < 4; ++i) other[i] = from_other_half(lat[i]);
    // column tile 0: pixels of lanes 0-31; column tile 1: pixels of lanes 32-63
    const f32x16 y0 = decode_tile(dec, lat, lane, hi);
    // an empty asm that claims to read tile 0's result and rewrite tile 1's
    // input: the compiler cannot start tile 1 before tile 0 is done, which
    // keeps the kernel at about 80 VGPRs (6 waves per SIMD) instead of 120
    u32x4 x1 = other;
    float y00 = y0[0];
    asm volatile("" : "+v"(x1[0]), "+v"(y00));
    const f32x16 y1 = decode_tile(dec, x1, lane, hi);
    // rows 0-3 (the outputs) sit in registers 0-3 of lanes 0-31; lane l + 32
    // takes column l of tile 1 from lane l
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float t1 = __uint_as_float(from_other_half(__float_as_uint(y1[i])));
        out[i] = hi ? t1 : (i == 0 ? y00 : y0[i]);
    }
}

// LDS the deduplicating decode needs per wavefront (bytes).
constexpr int kDedupBytes = 256 * 4 + 32 * 16 + 32 * 16;

// Decode with duplicates removed: the texels picked by the wave usually
// repeat (a magnified tile picks from a few texels), and each distinct
// texel decodes alike in any column. When the picks lie within 16x16
// texels of lane 0's pick and at most 32 are distinct, one lane per distinct
// texel hands its latents to a compact column tile, the wave runs one column
// tile through the MLP instead of two, and every lane takes the result of its
// texel. Otherwise it falls back to decode_latent. The outputs are identical
// either way. `scratch` is kDedupBytes of the wave's LDS; all 64 lanes call
// in uniform control flow.
__device__ __forceinline__ void decode_latent_dedup(const uint8_t* dec, u32x4 lat, uint32_t sx, uint32_t sy,
                                                    uint32_t mx, uint32_t my, uint8_t* scratch, float out[4]) {
    const int lane = threadIdx.x & 63;
    const bool hi = lane >= 32;
    const uint32_t sx0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)sx);
    const uint32_t sy0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)sy);
    const uint32_t rx = (sx - sx0 + 8u) & mx, ry = (sy - sy0 + 8u) & my;
    if (__builtin_amdgcn_ballot_w64(rx >= 16u || ry >= 16u) == 0) {
        int* owner = reinterpret_cast<int*>(scratch);                         // [256]
        u32x4* latbuf = reinterpret_cast<u32x4*>(scratch + 256 * 4);          // [32]
        float4* rgba = reinterpret_cast<float4*>(scratch + 256 * 4 + 32 * 16); // [32]
        const int key = (int)(rx | (ry << 4));                                // injective on the texels
        owner[key] = lane;                                                    // any writer wins
        wave_lds_sync();
        const int o = owner[key];
        const uint64_t reps = __builtin_amdgcn_ballot_w64(o == lane);
        const int n = __popcll(reps);
        if (n <= 32) {
            if (o == lane) latbuf[__popcll(reps & ((1ull << lane) - 1ull))] = lat;
            wave_lds_sync();
            const u32x4 zero4 = {0u, 0u, 0u, 0u};
            const u32x4 x = (!hi && lane < n) ? latbuf[lane] : zero4;
            const f32x16 y = decode_tile(dec, x, lane, hi);
            if (!hi && lane < n) rgba[lane] = make_float4(y[0], y[1], y[2], y[3]);
            wave_lds_sync();
            const float4 v = rgba[__popcll(reps & ((1ull << o) - 1ull))];
            out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
            wave_lds_sync();                                                  // scratch free again
            return;
        }
        wave_lds_sync();
    }
    decode_latent(dec, lat, out);
}

// The lane's 8 latents as BF16 from the raw texel payload (16 bytes for
// F16/BF16 latents, the low 8 bytes for FP8), times the optional
// per-channel scale (in FP32, then RN to BF16).
__device__ __forceinline__ float latent_channel(uint4 q, int fmt, int k) {
    const uint32_t w = (k < 2) ? q.x : (k < 4) ? q.y : (k < 6) ? q.z : q.w;
    if (fmt == STF_LATENT8_FP8) {
        const uint32_t d = (k < 4) ? q.x : q.y;
        return fp8_e4m3(d >> (8 * (k & 3)));
    }
    const uint32_t half = (w >> (16 * (k & 1))) & 0xFFFFu;
    return fmt == STF_LATENT8_F16 ? h2f(half) : bf16_bits(half);
}

// The lane's 8 latents as FP8 E4M3 bytes (low 8 bytes of the result):
// FP8 latents without a scale as stored, others times the scale, RN.
__device__ __forceinline__ u32x4 latent_fp8(uint4 q, const TexArg& t) {
    u32x4 r = {0u, 0u, 0u, 0u};
    if (t.fmt == STF_LATENT8_FP8 && !t.has_scale) {
        r[0] = q.x; r[1] = q.y;
        return r;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = latent_channel(q, t.fmt, 4 * i + k);
            if (t.has_scale) v[k] *= t.scale[4 * i + k];
        }
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
        r[i] = (uint32_t)w;
    }
    return r;
}

// The lane's latents as the decoder's operand type.
__device__ __forceinline__ u32x4 latent_operand(const uint8_t* dec, uint4 q, const TexArg& t);

__device__ __forceinline__ u32x4 latent_bf16(uint4 q, const TexArg& t) {
    u32x4 r;
    if (t.fmt == STF_LATENT8_BF16 && !t.has_scale) {
        r[0] = q.x; r[1] = q.y; r[2] = q.z; r[3] = q.w;
        return r;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float a = latent_channel(q, t.fmt, 2 * i), b = latent_channel(q, t.fmt, 2 * i + 1);
        if (t.has_scale) {
            a *= t.scale[2 * i];
            b *= t.scale[2 * i + 1];
        }
        r[i] = pack_bf16(a, b);
    }
    return r;
}

// Copy the packed decoder into LDS (all threads of the workgroup; the caller
// synchronises).
__device__ __forceinline__ void stage_decoder(const uint8_t* src, uint8_t* lds) {
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < kDecBytes / 16; i += blockDim.x) d[i] = s[i];
}

__device__ __forceinline__ u32x4 latent_operand(const uint8_t* dec, uint4 q, const TexArg& t) {
    return decoder_is_fp8(dec) ? latent_fp8(q, t) : latent_bf16(q, t);
}

}  // namespace stf
