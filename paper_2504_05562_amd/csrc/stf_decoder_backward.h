// Adjoint of Eq. (14) through the latent decoder MLP (the neural-texture
// setting of Sec. 1 and Sec. 5.6): gradients with respect to the latents and
// to the decoder's weights and biases.
//
// The weights of Eq. (14) do not depend on texel values, so the gradient
// with respect to each decoded texel, g_x = dL/dD(x), is the texel adjoint
// (backward_kernel with four channels, into a dense FP32 buffer). Each
// texel's decode is independent, so the chain rule then runs through the
// decoder once per texel x with g_x != 0:
//     z1 = W1 l + b1, h1 = ReLU(z1), z2 = W2 h1 + b2, h2 = ReLU(z2), y = W3 h2 + b3
//     d2 = (W3^T g) * [z2 > 0],  d1 = (W2^T d2) * [z1 > 0],  dL/dl = W1^T d1
//     dW3 = sum g h2^T,  dW2 = sum d2 h1^T,  dW1 = sum d1 l^T,  db = sums of g, d2, d1
// in FP32 with the FP32 weights (the forward pass's BF16 or FP8 rounding of
// weights and activations is passed straight through, as in mixed-precision
// training). One wavefront takes kDbN consecutive texels of the grid at a
// time: their activations live in LDS with the texels as columns, and every
// product above -- the per-texel layers as well as the weight gradients,
// which contract over the texels -- runs on v_mfma_f32_16x16x4_f32, with the
// weights read from one LDS copy per workgroup. Only blocks that some
// gradient reaches are visited: a view covers a small part of the grid, so
// the blocks with g != 0 are first listed in increasing order and dealt out
// round-robin, which gives every wave the same number of blocks to within
// one. A wave's weight gradients accumulate in registers over its blocks;
// the waves of a workgroup add them into one slot in wave order, and the
// last kernels sum the slots in a fixed order, so the result does not
// depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stf_device.h"

namespace stf {

constexpr int kDbN = 16;                           // texels per block (the columns of the products)
constexpr int kDbLd = kDbN + 1;                    // LDS row stride (floats) of the [unit][texel] arrays
constexpr int kDbWaves = 4;                        // waves per workgroup, sharing one LDS copy of the weights
constexpr int kGradW1 = 0, kGradB1 = kGradW1 + 64 * 8, kGradW2 = kGradB1 + 64, kGradB2 = kGradW2 + 64 * 64,
              kGradW3 = kGradB2 + 64, kGradB3 = kGradW3 + 4 * 64, kGradFloats = kGradB3 + 4;   // 4996
constexpr int kDecBwdMaxWaves = 2048;                       // per texture, in workgroups of kDbWaves
constexpr int kListThreads = 1024;                 // the one workgroup that lists the active blocks

struct DecBwdArgs {
    const uint8_t* data;     // latent grid, row pitch `pitch`
    int64_t pitch;
    int32_t tw, th, fmt;
    int32_t nblocks;         // ceil(tw * th / kDbN)
    const int32_t* list;     // indices of the blocks with some g != 0, increasing
    const int32_t* count;    // their number
    float scale[8];          // latent = stored * scale
    const float* g;          // dL/d(decoded texel), [th * tw][4]
    const float* w1;         // [64][8]
    const float* b1;         // [64]
    const float* w2;         // [64][64]
    const float* b2;         // [64]
    const float* w3;         // [4][64]
    float* dlat;             // [th * tw][8], accumulated
    float* partial;          // [gridDim.x][kGradFloats], written
};

// Latent channels of texel t (row-major index) times their scales.
__device__ __forceinline__ void load_latent(const DecBwdArgs& a, int64_t t, float* x) {
    const int64_t y = t / a.tw, xx = t % a.tw;
    const uint8_t* p = a.data + y * a.pitch;
    if (a.fmt == STF_LATENT8_FP8) {
        const uint2 q = *reinterpret_cast<const uint2*>(p + xx * 8);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            x[c] = fp8_e4m3(q.x >> (8 * c));
            x[4 + c] = fp8_e4m3(q.y >> (8 * c));
        }
    } else {
        const uint4 q = *reinterpret_cast<const uint4*>(p + xx * 16);
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t bits = (w[c >> 1] >> (16 * (c & 1))) & 0xFFFFu;
            x[c] = a.fmt == STF_LATENT8_BF16 ? bf16_bits(bits) : h2f(bits);
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] *= a.scale[c];
}

// acc[i * NT + j] += A(16 i .., k) B(k, 16 j ..) over k in [0, K), K a
// multiple of 4: MT x NT tiles of 16 x 16 on v_mfma_f32_16x16x4_f32. Lane l
// feeds A(16 i + l % 16, k0 + l / 16) and B(k0 + l / 16, 16 j + l % 16) and
// holds rows 16 i + 4 (l / 16) + v, v < 4, of column 16 j + l % 16 of each
// tile. The accessors return 0 outside the operands.
template <int MT, int NT, typename FA, typename FB>
__device__ __forceinline__ void mfma_tiles(v4f (&acc)[MT * NT], FA A, FB B, int K) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
#pragma unroll 2
    for (int k0 = 0; k0 < K; k0 += 4) {
        float av[MT], bv[NT];
#pragma unroll
        for (int i = 0; i < MT; ++i) av[i] = A(16 * i + r, k0 + q);
#pragma unroll
        for (int j = 0; j < NT; ++j) bv[j] = B(k0 + q, 16 * j + r);
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[i * NT + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i * NT + j], 0, 0, 0);
    }
}

template <int T>
__device__ __forceinline__ void zero_tiles(v4f (&acc)[T]) {
#pragma unroll
    for (int i = 0; i < T; ++i) acc[i] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
}

// Calls f(row, col, value) for every element a lane holds of MT x NT tiles.
template <int MT, int NT, typename F>
__device__ __forceinline__ void tiles_out(const v4f (&acc)[MT * NT], F f) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) f(16 * i + 4 * q + v, 16 * j + r, acc[i * NT + j][v]);
}

// Marks the blocks of kDbN texels that some gradient reaches: one bit per
// block in `mask` (cleared beforehand). Each quarter wave reads one block's
// g (16 bytes per texel); a wave's four blocks share a mask word, set with
// one atomic OR. Grid: ceil(nblocks / 16) workgroups of 256.
__global__ __launch_bounds__(256) void decoder_block_mask_kernel(const float* g, int64_t ntex, int nblocks,
                                                                 uint32_t* mask) {
    static_assert(kDbN == 16, "one block per quarter wave");
    const int lane = threadIdx.x & 63;
    const int blk0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 4;     // a multiple of 4: one mask word
    const int blk = blk0 + (lane >> 4);
    const int64_t t = (int64_t)blk * kDbN + (lane & 15);
    bool any = false;
    if (blk < nblocks && t < ntex) {
        const float4 v = reinterpret_cast<const float4*>(g)[t];
        any = v.x != 0.0f || v.y != 0.0f || v.z != 0.0f || v.w != 0.0f;
    }
    const uint64_t m = __builtin_amdgcn_ballot_w64(any);
    uint32_t bits = 0u;
#pragma unroll
    for (int q = 0; q < 4; ++q) bits |= ((m >> (16 * q)) & 0xFFFFull) != 0ull ? 1u << q : 0u;
    if (lane == 0 && bits != 0u) atomicOr(&mask[blk0 >> 5], bits << (blk0 & 31));
}

// Indices of the marked blocks in increasing order, and their number: one
// workgroup of kListThreads. Thread i takes the i-th contiguous run of mask
// words (one word per thread up to 32 768 blocks), the runs' bit counts are
// scanned in LDS, then every thread writes its run's indices at its offset.
__global__ __launch_bounds__(kListThreads) void decoder_block_list_kernel(const uint32_t* mask, int nblocks,
                                                                          int32_t* list, int32_t* count) {
    __shared__ int32_t scan[kListThreads];
    const int i = threadIdx.x;
    const int nwords = (nblocks + 31) / 32;
    const int run = (nwords + kListThreads - 1) / kListThreads;
    const int lo = min(i * run, nwords), hi = min(lo + run, nwords);
    int n = 0;
#pragma unroll 4
    for (int j = lo; j < hi; ++j) n += __builtin_popcount(mask[j]);
    scan[i] = n;
    __syncthreads();
    for (int d = 1; d < kListThreads; d <<= 1) {      // inclusive scan (Hillis-Steele)
        const int v = i >= d ? scan[i - d] : 0;
        __syncthreads();
        scan[i] += v;
        __syncthreads();
    }
    int o = scan[i] - n;
    for (int j = lo; j < hi; ++j)
        for (uint32_t m = mask[j]; m != 0u; m &= m - 1u) list[o++] = j * 32 + __builtin_ctz(m);
    if (i == kListThreads - 1) *count = scan[i];
}

// Workgroups of kDbWaves waves; wave w of the launch (workgroup-major) takes
// the listed blocks w, w + kDbWaves * gridDim.x, ... The workgroup stages the
// decoder's FP32 weights in LDS once (the operands of every per-texel
// product), and each wave keeps its block's activations there with the
// texels as columns. A wave's weight gradients accumulate in registers over
// its blocks; at the end the waves add them into one slot per workgroup, in
// wave order, through LDS.
constexpr int kW1Ld = 9, kW2Ld = 65, kW3Ld = 65;   // padded LDS rows of the weights
constexpr int kDbWeightFloats = 64 * kW1Ld + 64 * kW2Ld + 4 * kW3Ld + 64 + 64;
constexpr int kDbWaveFloats = 2 * 64 * kDbLd + 4 * kDbLd + 8 * kDbLd;    // H1, H2, GT, XT
static_assert(kDbWaves * kDbWaveFloats + kDbWeightFloats >= kGradFloats, "the slot sum fits the LDS");

__global__ __launch_bounds__(64 * kDbWaves, 2) void decoder_backward_kernel(DecBwdArgs a) {
    __shared__ float lds[kDbWeightFloats + kDbWaves * kDbWaveFloats];
    float* W1s = lds;                                  // [64][kW1Ld]   W1 (64 x 8)
    float* W2s = W1s + 64 * kW1Ld;                     // [64][kW2Ld]   W2 (64 x 64)
    float* W3s = W2s + 64 * kW2Ld;                     // [4][kW3Ld]    W3 (4 x 64)
    float* B1s = W3s + 4 * kW3Ld;                      // [64]
    float* B2s = B1s + 64;                             // [64]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* H1 = lds + kDbWeightFloats + wave * kDbWaveFloats;   // h1, then d1; [unit][texel]
    float* H2 = H1 + 64 * kDbLd;                                 // h2, then d2
    float* GT = H2 + 64 * kDbLd;                                 // g
    float* XT = GT + 4 * kDbLd;                                  // latents
    const int nlisted = *a.count;
    if ((int)blockIdx.x * kDbWaves >= nlisted) return;          // no block for the workgroup: no slot
    for (int i = threadIdx.x; i < 64 * 64; i += 64 * kDbWaves) W2s[(i >> 6) * kW2Ld + (i & 63)] = a.w2[i];
    for (int i = threadIdx.x; i < 64 * 8; i += 64 * kDbWaves) W1s[(i >> 3) * kW1Ld + (i & 7)] = a.w1[i];
    for (int i = threadIdx.x; i < 4 * 64; i += 64 * kDbWaves) W3s[(i >> 6) * kW3Ld + (i & 63)] = a.w3[i];
    if (threadIdx.x < 64) {
        B1s[threadIdx.x] = a.b1[threadIdx.x];
        B2s[threadIdx.x] = a.b2[threadIdx.x];
    }
    __syncthreads();
    constexpr int NT = kDbN / 16;      // column tiles of the per-texel products
    v4f dw2[16], dw1[4], dw3[4];
    zero_tiles(dw2);
    zero_tiles(dw1);
    zero_tiles(dw3);
    float db1 = 0.0f, db2 = 0.0f, db3 = 0.0f;      // unit `lane` (db3: lanes 0-3)
    const int64_t ntex = (int64_t)a.tw * a.th;
    const int stride = (int)gridDim.x * kDbWaves;
#pragma unroll 1
    for (int k = (int)blockIdx.x * kDbWaves + wave; k < nlisted; k += stride) {
        const int blk = a.list[k];
        const int64_t t = (int64_t)blk * kDbN + lane;
        const bool in = lane < kDbN && t < ntex;
        float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (in) g = reinterpret_cast<const float4*>(a.g)[t];
        float x[8];
        if (in) {
            load_latent(a, t, x);
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) x[c] = 0.0f;
        }
        if (lane < kDbN) {
            GT[0 * kDbLd + lane] = g.x;
            GT[1 * kDbLd + lane] = g.y;
            GT[2 * kDbLd + lane] = g.z;
            GT[3 * kDbLd + lane] = g.w;
#pragma unroll
            for (int c = 0; c < 8; ++c) XT[c * kDbLd + lane] = x[c];
        }
        wave_lds_sync();
        {   // h1 = ReLU(W1 l + b1)
            v4f acc[4 * NT];
            zero_tiles(acc);
            mfma_tiles<4, NT>(acc, [&](int m, int k) { return W1s[m * kW1Ld + k]; },
                              [&](int k, int n) { return XT[k * kDbLd + n]; }, 8);
            tiles_out<4, NT>(acc, [&](int m, int n, float v) { H1[m * kDbLd + n] = fmaxf(v + B1s[m], 0.0f); });
        }
        wave_lds_sync();
        {   // h2 = ReLU(W2 h1 + b2)
            v4f acc[4 * NT];
            zero_tiles(acc);
            mfma_tiles<4, NT>(acc, [&](int m, int k) { return W2s[m * kW2Ld + k]; },
                              [&](int k, int n) { return H1[k * kDbLd + n]; }, 64);
            tiles_out<4, NT>(acc, [&](int m, int n, float v) { H2[m * kDbLd + n] = fmaxf(v + B2s[m], 0.0f); });
        }
        wave_lds_sync();
        // dW3 += g h2^T (texels contracted; rows 4-15 of the tile are padding)
        mfma_tiles<1, 4>(dw3, [&](int m, int k) { return m < 4 ? GT[m * kDbLd + k] : 0.0f; },
                         [&](int k, int n) { return H2[n * kDbLd + k]; }, kDbN);
        if (lane < 4)
            for (int k = 0; k < kDbN; ++k) db3 += GT[lane * kDbLd + k];
        wave_lds_sync();
        {   // d2 = (W3^T g) * [z2 > 0], in place of h2
            v4f acc[4 * NT];
            zero_tiles(acc);
            mfma_tiles<4, NT>(acc, [&](int m, int k) { return W3s[k * kW3Ld + m]; },
                              [&](int k, int n) { return GT[k * kDbLd + n]; }, 4);
            tiles_out<4, NT>(acc, [&](int m, int n, float v) {
                float& h = H2[m * kDbLd + n];
                h = h > 0.0f ? v : 0.0f;
            });
        }
        wave_lds_sync();
        // dW2 += d2 h1^T, db2 += sum d2
        mfma_tiles<4, 4>(dw2, [&](int m, int k) { return H2[m * kDbLd + k]; },
                         [&](int k, int n) { return H1[n * kDbLd + k]; }, kDbN);
        for (int k = 0; k < kDbN; ++k) db2 += H2[lane * kDbLd + k];
        wave_lds_sync();
        {   // d1 = (W2^T d2) * [z1 > 0], in place of h1
            v4f acc[4 * NT];
            zero_tiles(acc);
            mfma_tiles<4, NT>(acc, [&](int m, int k) { return W2s[k * kW2Ld + m]; },
                              [&](int k, int n) { return H2[k * kDbLd + n]; }, 64);
            tiles_out<4, NT>(acc, [&](int m, int n, float v) {
                float& h = H1[m * kDbLd + n];
                h = h > 0.0f ? v : 0.0f;
            });
        }
        wave_lds_sync();
        // dW1 += d1 l^T (columns 8-15 of the tile are padding), db1 += sum d1
        mfma_tiles<4, 1>(dw1, [&](int m, int k) { return H1[m * kDbLd + k]; },
                         [&](int k, int n) { return n < 8 ? XT[n * kDbLd + k] : 0.0f; }, kDbN);
        for (int k = 0; k < kDbN; ++k) db1 += H1[lane * kDbLd + k];
        {   // dL/dl = W1^T d1 (rows 8-15 padding); dL/dstored = dL/dl * scale
            v4f acc[NT];
            zero_tiles(acc);
            mfma_tiles<1, NT>(acc, [&](int m, int k) { return m < 8 ? W1s[k * kW1Ld + m] : 0.0f; },
                              [&](int k, int n) { return H1[k * kDbLd + n]; }, 64);
            const int64_t base = (int64_t)blk * kDbN;
            tiles_out<1, NT>(acc, [&](int m, int n, float v) {
                if (m < 8 && base + n < ntex) a.dlat[(base + n) * 8 + m] += v * a.scale[m];
            });
        }
        wave_lds_sync();                                              // LDS reads done before the next block
    }
    // the workgroup's slot: wave 0's sums, then waves 1, 2, 3 add theirs in turn
    // (the activation and weight arrays are free once every wave is here)
    float* sum = lds;
    for (int w = 0; w < kDbWaves; ++w) {
        __syncthreads();
        if (wave == w) {
            auto put = [&](int e, float v) {
                if (w == 0) sum[e] = v;
                else sum[e] += v;
            };
            tiles_out<4, 4>(dw2, [&](int m, int n, float v) { put(kGradW2 + m * 64 + n, v); });
            tiles_out<4, 1>(dw1, [&](int m, int n, float v) {
                if (n < 8) put(kGradW1 + m * 8 + n, v);
            });
            tiles_out<1, 4>(dw3, [&](int m, int n, float v) {
                if (m < 4) put(kGradW3 + m * 64 + n, v);
            });
            put(kGradB1 + lane, db1);
            put(kGradB2 + lane, db2);
            if (lane < 4) put(kGradB3 + lane, db3);
        }
    }
    __syncthreads();
    float* out = a.partial + (size_t)blockIdx.x * kGradFloats;
    for (int e = threadIdx.x; e < kGradFloats; e += 64 * kDbWaves) out[e] = sum[e];
}

struct MlpGradPtrs {
    float* p[6];             // dW1, db1, dW2, db2, dW3, db3 (accumulated)
};

// The per-wave slots are summed in two fixed-order steps, so that many
// threads share the reads: kReduceSplits partial sums per gradient element
// (slots split + k * kReduceSplits of each texture), then their sum added to
// the outputs. Texture i's slots start at slot off[i]; only its first
// min(groups[i], ceil(*count[i] / kDbWaves)) workgroups had blocks and wrote
// their slots.
constexpr int kReduceSplits = 64;

struct SlotRanges {
    int32_t ntex;
    int32_t off[STF_MAX_TEXTURES], groups[STF_MAX_TEXTURES];
    const int32_t* count[STF_MAX_TEXTURES];
};

__global__ __launch_bounds__(256) void decoder_grad_partial_kernel(const float* partial, SlotRanges r, float* level2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kGradFloats) return;
    float s = 0.0f;
    for (int i = 0; i < r.ntex; ++i) {
        const int n = min(r.groups[i], (*r.count[i] + kDbWaves - 1) / kDbWaves);
        for (int w = blockIdx.y; w < n; w += kReduceSplits) s += partial[(size_t)(r.off[i] + w) * kGradFloats + e];
    }
    level2[(size_t)blockIdx.y * kGradFloats + e] = s;
}

__global__ __launch_bounds__(256) void decoder_grad_reduce_kernel(const float* level2, MlpGradPtrs o) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kGradFloats) return;
    float s = 0.0f;
#pragma unroll 8
    for (int w = 0; w < kReduceSplits; ++w) s += level2[(size_t)w * kGradFloats + e];
    const int starts[6] = {kGradW1, kGradB1, kGradW2, kGradB2, kGradW3, kGradB3};
    int k = 5;
    while (e < starts[k]) --k;
    o.p[k][e - starts[k]] += s;
}

// Fills n floats from the 16-byte aligned p with zero (a kernel, not a
// memset node: safe under graph capture), one non-temporal 16-byte store per
// lane and step, then the last n % 4 floats.
__global__ __launch_bounds__(256) void zero_fill_kernel(float* p, int64_t n) {
    const int64_t n4 = n >> 2, stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    v4f* p4 = reinterpret_cast<v4f*>(p);
    for (int64_t i = first; i < n4; i += stride) __builtin_nontemporal_store(v4f{0.0f, 0.0f, 0.0f, 0.0f}, p4 + i);
    for (int64_t i = n4 * 4 + first; i < n; i += stride) p[i] = 0.0f;
}

}  // namespace stf
