// Adjoint kernels of the STF library: dL/dT of Eq. (14) for every footprint
// (device code), shared by the translation units of libstf.so that launch
// them. The forward building blocks (selection, tiles, bin windows) come
// from stf_kernels.h.
#pragma once

#include "stf_kernels.h"

namespace stf {

// LDS per wave: a small area (the whole tile's Nb float [kBins], the sums of
// 1/p; or 64 {s, r} records) and a wide area. For the whole tile the wide
// area first holds the exact u64 accumulators of Nb and, once they are
// converted, one row record per tile pixel for the matrix cores: its weights
// along the window's rows and columns, zero outside its support (kBinG
// each), and its four scaled gradients. For the other footprints it holds
// the members' coefficients and the pixels' scaled gradients of the gather,
// then the one-hot operands of the window sum. The workgroup's wide areas
// are contiguous; after the products they hold the workgroup's merge area.
constexpr int kBwdNbFloats = (kBins + 3) & ~3;
constexpr int kBwdRowFloats = 2 * kBinG + 4;
constexpr int kBwdWideFloats = kBins * 2 > 64 * kBwdRowFloats ? kBins * 2 : 64 * kBwdRowFloats;
static_assert(kBwdNbFloats % 4 == 0 && kBwdRowFloats % 4 == 0 && kBwdWideFloats % 4 == 0,
              "16-byte aligned LDS records");

// ============================================================================
// adjoint of Eq. (14)
// ============================================================================
//
// out_c = sum_i a_ci T[x_i] with a_ci = w_ci / B_c, w_ci = f_c(x_i) r_i and
// B_c = sum_i w_ci; the weights depend on UVs and random numbers only, so
// dL/dT[x] += sum_c sum_{i in S(c), x_i = x} a_ci dL/dout_c. The kernel
// recomputes every pick exactly as the forward pass does and recomputes B_c.
// For the whole tile the sum over i collapses per texel:
// dL/dT[x] = N_x sum_c f_c(x) q_c with N_x = sum_{i: x_i = x} r_i and
// q_c = dL/dout_c / B_c, a rank-64 product over the wave's texel window on
// the matrix cores. The other footprints first gather each pick's total,
// then add the 64 totals into the window with the same product (one-hot
// rows and columns). The four windows of a workgroup are merged in LDS and
// flushed with one global atomic per touched texel and channel.

// Workgroup of the launch grid this workgroup works on, renumbered so that
// each XCD runs one contiguous part of the grid in row-major order. The
// chip's eight XCDs take the workgroups of a launch round-robin by linear id
// and each has its own L2; neighbouring workgroups add into the same
// gradient texels, whose atomics then stay in one L2 (the forward kernels,
// which only read, measured slower with it). XCD x (linear ids x, x + 8, ...)
// gets ids x q + min(x, r) onward, with q, r the quotient and remainder of
// the grid size by 8: a bijection.
constexpr unsigned kXcds = 8;

__device__ __forceinline__ void xcd_block(int& bx, int& by) {
    const unsigned total = gridDim.x * gridDim.y, id = blockIdx.y * gridDim.x + blockIdx.x;
    const unsigned x = id % kXcds, q = total / kXcds, r = total % kXcds;
    const unsigned v = x * q + min(x, r) + id / kXcds;
    bx = (int)(v % gridDim.x);
    by = (int)(v / gridDim.x);
}

template <int C>
__device__ __forceinline__ void atomic_texel(float* g, int tw, uint32_t s, const float* v, float scale) {
    float* p = g + ((int64_t)(s >> 16) * tw + (s & 0xFFFFu)) * C;
#pragma unroll
    for (int c = 0; c < C; ++c) unsafeAtomicAdd(p + c, v[c] * scale);
}

// Workgroup merge of the adjoint windows: the four tiles of a workgroup sit
// side by side, so their bin windows overlap (fully at high magnification).
// Each wave adds its window's sums into one kMergeW x kMergeH texel area in
// LDS covering all four, and the workgroup flushes that area with one global
// atomic per touched texel and channel, instead of each wave flushing its
// own window: the global FP32 atomics drop by the overlap. A workgroup whose
// windows do not fit the area flushes per wave; waves whose supports leave
// their window send their gradients with global atomics and take no part.
constexpr int kMergeW = 32, kMergeH = 16;

struct MergeArea {
    float* v;                // [kMergeH * kMergeW][C] sums (over the workgroup's wide areas)
    int* info;               // per wave: contributes, base_x, base_y
    float* wide;             // this wave's wide area (kBwdWideFloats)
};

// The rank-64 window product on the matrix cores: for every cell (row i,
// column j) of the kBinG x kBinG window, the sum over the wave's 64 pixels k
// of a_k(i) b_k(j) q_k (per channel), from the pixels' row records
// {a_k at the kBinG rows, b_k at the kBinG columns, q_k}. K = the 64 pixels,
// four per v_mfma_f32_16x16x4_f32 (A[i][k] and B[k][j] of lane l: i = j =
// l % 16, k = l / 16); lanes of tile rows and columns 12-15 read the next
// entries, and those outputs are never used. Cell (4 (l / 16) + v, l % 16)
// lands in acc[c][v] of lane l.
template <int C>
__device__ __forceinline__ void window_product(const float* rows, int ij, int kp, v4f* acc) {
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 2
    for (int m = 0; m < 16; ++m) {
        const float* rp = rows + (4 * m + kp) * kBwdRowFloats;
        const float wa = rp[ij];
        const float wb = rp[kBinG + ij];
        const float4 q = *reinterpret_cast<const float4*>(rp + 2 * kBinG);
        const float qc[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa, wb * qc[c], acc[c], 0, 0, 0);
    }
}

// Sum of the wave's 64 pick totals per window cell: the rank-64 product of
// one-hot rows (the pick's window row) and one-hot columns carrying the
// totals, on v_mfma_f32_16x16x32_bf16. Each total is split exactly into
// three BF16 parts (hi + mid + lo = the FP32 value: every part takes the
// next 8 significant bits of the remainder), so the products are exact and
// only the FP32 accumulation rounds; K = 64 pixels x 3 parts = 6 products
// of 32 per channel, against 16 FP32 products of 4. LDS (the wave's wide
// area): the picks' window rows and columns [64] bytes each (0xFF for pixels
// off the screen, which match no cell), then the parts [C][3][64] BF16.
// Lane l holds k-values 8 (l / 16) .. + 7 of each product for window row
// (A) and column (B) l % 16, the same k in A and B, whatever order the
// hardware sums them in; cell (4 (l / 16) + v, l % 16) lands in acc[c][v].
template <int C>
__device__ __forceinline__ void onehot_window_sum(float* wide, const Pixel& P, uint32_t cx, uint32_t cy,
                                                  const float* tot, int ij, int kp, v4f* acc) {
    uint8_t* rowv = reinterpret_cast<uint8_t*>(wide);
    uint8_t* colv = rowv + 64;
    uint16_t* part = reinterpret_cast<uint16_t*>(rowv + 128);
    rowv[P.q] = P.valid ? (uint8_t)cy : (uint8_t)0xFF;
    colv[P.q] = P.valid ? (uint8_t)cx : (uint8_t)0xFF;
#pragma unroll
    for (int c = 0; c < C; c += 2) {
        // two channels per conversion (round to nearest even)
        f32x2 x = {tot[c], c + 1 < C ? tot[c + 1] : 0.0f};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t b = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2));
            part[(c * 3 + k) * 64 + P.q] = (uint16_t)(b & 0xFFFFu);
            if (c + 1 < C) part[((c + 1) * 3 + k) * 64 + P.q] = (uint16_t)(b >> 16);
            const f32x2 h = {__uint_as_float(b << 16), __uint_as_float(b & 0xFFFF0000u)};
            x = x - h;     // exact: at most 16, then 8 significant bits remain, so the third part is exact
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int k0 = 32 * t + 8 * kp;
        const uint2 r8 = *reinterpret_cast<const uint2*>(rowv + k0);
        const uint2 c8 = *reinterpret_cast<const uint2*>(colv + k0);
        u32x4 a, m;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint32_t rw = (h < 2 ? r8.x : r8.y) >> (16 * (h & 1));
            const uint32_t cw = (h < 2 ? c8.x : c8.y) >> (16 * (h & 1));
            a[h] = (((rw & 0xFFu) == (uint32_t)ij) ? 0x3F80u : 0u) |
                   ((((rw >> 8) & 0xFFu) == (uint32_t)ij) ? 0x3F800000u : 0u);      // BF16 1.0
            m[h] = (((cw & 0xFFu) == (uint32_t)ij) ? 0xFFFFu : 0u) |
                   ((((cw >> 8) & 0xFFu) == (uint32_t)ij) ? 0xFFFF0000u : 0u);
        }
        const bf16x8 av = __builtin_bit_cast(bf16x8, a);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const u32x4 v = *reinterpret_cast<const u32x4*>(part + (c * 3 + k) * 64 + k0) & m;
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf16x8, v), acc[c], 0, 0, 0);
            }
    }
    wave_lds_sync();                               // read before the merge reuses the area
}

// Pixels of the wave whose 2x2w window holds this lane's pixel (lx, ly),
// itself excluded: bit p for tile pixel p (row-major). A 2x2w window starts
// at most one pixel before its own pixel per axis (its origin is the pixel's
// coordinate or the one before, clamped to 0..6), so only the pixels within
// one of (lx, ly) per axis can hold it.
__device__ __forceinline__ uint64_t reverse_members(int fp, int lx, int ly) {
    uint64_t bits = 0ull;
    for (int py = max(ly - 1, 0); py <= min(ly + 1, 7); ++py)
        for (int px = max(lx - 1, 0); px <= min(lx + 1, 7); ++px) {
            int ox, oy, n;
            window_of(fp, px, py, ox, oy, n);
            if ((uint32_t)(lx - ox) < (uint32_t)n && (uint32_t)(ly - oy) < (uint32_t)n && (px != lx || py != ly))
                bits |= 1ull << (py * 8 + px);
        }
    return bits;
}

// Tables of at most kRevMaxK entries per pixel are gathered like the windows.
constexpr int kRevMaxK = kLutStageMax;

// Where each lane's pick receives contributions from, for the gather of the
// record footprints: square windows as a rectangle of pixels, the other
// windows as a mask of pixels, tables as a list
// of coefficient indices m * 64 + p (pixel p's entry m names this pixel) in
// LDS, ascending, so that the sums have a fixed order.
struct Reverse {
    uint64_t bits = 0ull;
    uint32_t rect = 0u;      // square windows: naming pixels x0 | x1 << 4 | y0 << 8 | y1 << 12 (inclusive)
    const uint16_t* list = nullptr;
    int at = 0, n = 0;
};

// Square windows are separable: the pixels whose window holds this one form
// a rectangle of tile pixels (origins clamp(p - 1, 0, 8 - n) per axis).
__device__ __forceinline__ uint32_t reverse_rect(int n, int lx, int ly) {
    int x0 = 8, x1 = -1, y0 = 8, y1 = -1;
    for (int p = 0; p < 8; ++p) {
        const int o = min(max(p - 1, 0), 8 - n);
        if (o <= lx && lx < o + n) { x0 = min(x0, p); x1 = max(x1, p); }
        if (o <= ly && ly < o + n) { y0 = min(y0, p); y1 = max(y1, p); }
    }
    return (uint32_t)x0 | ((uint32_t)x1 << 4) | ((uint32_t)y0 << 8) | ((uint32_t)y1 << 12);
}

// The lists of a table footprint (`lut`, [64][K] in LDS) for the wave (once
// per launch): count the entries naming each pixel (LDS integer atomics),
// prefix sums over the pixels, place the entries, then each pixel sorts its
// own list (insertion sort: quadratic in the entries naming the pixel, K on
// average; a table whose entries all name one pixel is slow but exact).
// `tmp` holds 128 ints of the wave's LDS.
__device__ __forceinline__ void build_reverse_table(int K, const uint8_t* lut, const Pixel& P, int* tmp,
                                                    uint16_t* list, Reverse& rev) {
    const uint8_t* row = lut + P.q * K;
    int* cnt = tmp;
    int* scan = tmp + 64;
    cnt[P.q] = 0;
    wave_lds_sync();
    for (int m = 0; m < K; ++m) {
        const int j = row[m] & 63;
        if (j != P.q) atomicAdd(&cnt[j], 1);
    }
    wave_lds_sync();
    const int n = cnt[P.q];
    int v = n;                                    // inclusive prefix over the pixel ids
    scan[P.q] = v;
    wave_lds_sync();
    for (int d = 1; d < 64; d <<= 1) {
        const int t = P.q >= d ? scan[P.q - d] : 0;
        wave_lds_sync();
        v += t;
        scan[P.q] = v;
        wave_lds_sync();
    }
    const int at = v - n;
    cnt[P.q] = at;                                // placement cursor
    wave_lds_sync();
    for (int m = 0; m < K; ++m) {
        const int j = row[m] & 63;
        if (j != P.q) list[atomicAdd(&cnt[j], 1)] = (uint16_t)(m * 64 + P.q);
    }
    wave_lds_sync();
    for (int i = 1; i < n; ++i) {                 // insertion sort of the own list
        const uint16_t x = list[at + i];
        int k = i - 1;
        while (k >= 0 && list[at + k] > x) {
            list[at + k + 1] = list[at + k];
            --k;
        }
        list[at + k + 1] = x;
    }
    wave_lds_sync();
    rev.list = list;
    rev.at = at;
    rev.n = n;
}

template <int FILT, int MODE, int C>
__device__ __forceinline__ void backward_slot(const Args& a, int slot, const Pixel& P, const SelCtx<FILT>& ctx,
                                              uint32_t hx, uint32_t hy, const float4& gin, float* lds,
                                              MergeArea merge, const Reverse& rev, const uint8_t* lut_lds) {
    constexpr int N = SelCtx<FILT>::N;
    const TexArg t = a.tex[slot];
    const int lane = lane_id();
    const int kx = ctx.x.pick(hx);
    const int ky = ctx.y.pick(hy);
    const uint32_t mx = (uint32_t)t.w - 1u, my = (uint32_t)t.h - 1u;
    const uint32_t sx = (uint32_t)(ctx.x.base + kx) & mx;
    const uint32_t sy = (uint32_t)(ctx.y.base + ky) & my;
    const uint32_t s = sx | (sy << 16);
    float* grad = a.out[slot];                              // dL/dT, [th][tw][C]
    const float gv[4] = {gin.x, gin.y, gin.z, gin.w};
    float g[C];
#pragma unroll
    for (int c = 0; c < C; ++c) g[c] = gv[c] * t.scale[c];
    const float r = (MODE == kModeStf || !P.valid) ? 0.0f : fast_rcp(ctx.x.wsel(kx) * ctx.y.wsel(ky));

    // The wave's kBinG x kBinG texel window holding every on-screen support;
    // lane l owns window cells (rows 4 (l / 16) + v, column l % 16) in vals.
    const int ij = lane & 15, kp = lane >> 4;
    int base_x = 0, base_y = 0;
    uint32_t rx = 0, ry = 0;
    const bool use_bins = bin_window<N>(P, ctx.x.base, ctx.y.base, mx, my, t.w, t.h, base_x, base_y, rx, ry);
    float vals[4][C];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int c = 0; c < C; ++c) vals[v][c] = 0.0f;

    if constexpr (MODE == kModeBins) {
        if (use_bins) {
            v4f acc[C];
            float* Nb = lds;
            // LDS: Nb float [kBins] (sum of 1/p per texel), N64 u64 [kBins]
            // (its exact integer accumulator, as in the forward pass)
            uint64_t* N64 = reinterpret_cast<uint64_t*>(merge.wide);
            for (int i = lane; i < kBins; i += 64) N64[i] = 0ull;
            for (int i = lane; i < kBins; i += 64) Nb[i] = 0.0f;
            const int my_bin = (int)(ry + ky) * kBinG + (int)(rx + kx);
            const bool fixed = !(a.flags & kFlagFloatBinSums) &&
                               __builtin_amdgcn_ballot_w64(P.valid && !fixed_range(r)) == 0;
            wave_lds_sync();
            if (fixed) {
                if (P.valid) atomicAdd(reinterpret_cast<unsigned long long*>(&N64[my_bin]),
                                       (unsigned long long)fixed_r(r));
                wave_lds_sync();
                for (int i = lane; i < kBins; i += 64) Nb[i] = float_r(N64[i]);
            } else {
                if (P.valid) atomicAdd(&Nb[my_bin], r);
            }
            wave_lds_sync();
            const int bin0 = (int)ry * kBinG + (int)rx;
            float B = 0.0f;
#pragma unroll
            for (int b = 0; b < N; ++b)
#pragma unroll
                for (int aa = 0; aa < N; ++aa) B += (ctx.x.w(aa) * ctx.y.w(b)) * Nb[bin0 + b * kBinG + aa];
            // Sum over the tile's pixels of f_c(x) q_c for every texel x of the
            // window (q_c = dL/dout_c / B_c): with f_c(x) = wy_c(row) wx_c(col)
            // it is the rank-64 product  Wy diag(q) Wx^T  (window_product).
            // Each pixel first publishes its row record (over the converted
            // 64-bit sums): its weight at every window row and column, zero
            // outside its support (off-screen pixels: all zero), then q.
            float* rows = merge.wide;                       // [64][kBwdRowFloats]
            {
                float* own = rows + P.q * kBwdRowFloats;
                const float inv = P.valid ? fast_rcp(B) : 0.0f;
                float4* o4 = reinterpret_cast<float4*>(own);
#pragma unroll
                for (int k = 0; k < 2 * kBinG / 4; ++k) o4[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (P.valid) {
#pragma unroll
                    for (int b = 0; b < N; ++b) own[ry + b] = ctx.y.w(b);
#pragma unroll
                    for (int b = 0; b < N; ++b) own[kBinG + rx + b] = ctx.x.w(b);
                }
                float qv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int c = 0; c < C; ++c) qv[c] = g[c] * inv;
                o4[2 * kBinG / 4] = make_float4(qv[0], qv[1], qv[2], qv[3]);
            }
            wave_lds_sync();
            window_product<C>(rows, ij, kp, acc);
            wave_lds_sync();                         // row records read before the merge reuses them
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 4 * kp + v;
                if (i < kBinG && ij < kBinG) {
                    const float nx = Nb[i * kBinG + ij];
#pragma unroll
                    for (int c = 0; c < C; ++c) vals[v][c] = acc[c][v] * nx;
                }
            }
        } else {
            // supports that leave the window: every pixel pairs with all 64 picks, global atomics
            uint2* meta = reinterpret_cast<uint2*>(lds);
            meta[P.q] = make_uint2(s, __float_as_uint(r));
            wave_lds_sync();
            float B = 1.0f;
            for (int j = 0; j < 64; ++j) {
                if (j == P.q) continue;
                const uint2 mj = meta[j];
                uint32_t dx, dy;
                if (support_offset<N>(mj.x, ctx.x.base, ctx.y.base, mx, my, dx, dy))
                    B += ctx.x.wsel(dx) * ctx.y.wsel(dy) * __uint_as_float(mj.y);
            }
            if (P.valid) {
                const float inv = fast_rcp(B);
                atomic_texel<C>(grad, t.w, s, g, inv);
                for (int j = 0; j < 64; ++j) {
                    if (j == P.q) continue;
                    const uint2 mj = meta[j];
                    const float rj = __uint_as_float(mj.y);
                    uint32_t dx, dy;
                    if (support_offset<N>(mj.x, ctx.x.base, ctx.y.base, mx, my, dx, dy) && rj != 0.0f)
                        atomic_texel<C>(grad, t.w, mj.x, g, ctx.x.wsel(dx) * ctx.y.wsel(dy) * rj * inv);
                }
            }
            wave_lds_sync();
        }
    } else {
        // Every contribution lands on some lane's pick: pixel p adds
        // f_p(s_j) r_j dL/dout_p / B_p to pick j of each other member j, and
        // dL/dout_p / B_p to its own. Each lane first gathers the total of its
        // pick (tot), then the wave deposits the 64 totals into its window
        // cells at once.
        float tot[C];
        if constexpr (MODE == kModeStf) {
#pragma unroll
            for (int c = 0; c < C; ++c) tot[c] = P.valid ? g[c] : 0.0f;
        } else if constexpr (MODE == kModeQuad) {
            uint32_t si[3];
            float ri[3];
            si[0] = quad_xor<1>(s); ri[0] = quad_xor<1>(r);
            si[1] = quad_xor<2>(s); ri[1] = quad_xor<2>(r);
            si[2] = quad_xor<3>(s); ri[2] = quad_xor<3>(r);
            float B = 1.0f, f[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                uint32_t dx, dy;
                const bool in = support_offset<N>(si[m], ctx.x.base, ctx.y.base, mx, my, dx, dy);
                f[m] = in ? ctx.x.wsel(dx) * ctx.y.wsel(dy) * ri[m] : 0.0f;
                B += f[m];
            }
            const float inv = P.valid ? fast_rcp(B) : 0.0f;
            // lane p's coefficient for partner p ^ (m + 1) reaches that partner
            // over the same xor exchange
#pragma unroll
            for (int c = 0; c < C; ++c) tot[c] = g[c] * inv;
            {
                const float k = f[0] * inv;
#pragma unroll
                for (int c = 0; c < C; ++c) tot[c] += quad_xor<1>(k * g[c]);
            }
            {
                const float k = f[1] * inv;
#pragma unroll
                for (int c = 0; c < C; ++c) tot[c] += quad_xor<2>(k * g[c]);
            }
            {
                const float k = f[2] * inv;
#pragma unroll
                for (int c = 0; c < C; ++c) tot[c] += quad_xor<3>(k * g[c]);
            }
        } else {
            // LDS: meta {s, r} [64] in the wave's small area; in the wide area
            // coef [K][64] (pixel p's f_p(s_j) r_j for its member m, zero when
            // s_j is off its support) and q [64][4] (dL/dout_p / B_p), or for a
            // table of more than kRevMaxK entries the per-lane sums [C][64]
            uint2* meta = reinterpret_cast<uint2*>(lds);
            float* coef = merge.wide;
            float* qrec = merge.wide + 16 * 64;
            float* lane_sum = merge.wide;
            const int fp = a.footprint;
            const bool scatter = fp == STF_FP_LUT && a.lut_k > kRevMaxK;     // long tables
            if (scatter) {
#pragma unroll
                for (int c = 0; c < C; ++c) lane_sum[c * 64 + P.q] = 0.0f;
            }
            meta[P.q] = make_uint2(s, __float_as_uint(r));
            wave_lds_sync();
            const int K = footprint_size(fp, a.lut_k);
            float B = 1.0f;
            // member m's coefficient f_p(s_j) r_j (zero for the pixel itself
            // and for picks off its support)
            auto member = [&](int m, int j) {
                float k = 0.0f;
                if (j != P.q) {
                    const uint2 mj = meta[j];
                    uint32_t dx, dy;
                    if (support_offset<N>(mj.x, ctx.x.base, ctx.y.base, mx, my, dx, dy))
                        k = ctx.x.wsel(dx) * ctx.y.wsel(dy) * __uint_as_float(mj.y);
                }
                B += k;
                if (!scatter) coef[m * 64 + P.q] = k;
            };
            if (fp == STF_FP_LUT && scatter) {
                for (int m = 0; m < K; ++m) member(m, a.lut[P.q * K + m] & 63);
            } else if (fp == STF_FP_LUT) {
                for (int m = 0; m < K; ++m) member(m, lut_lds[P.q * K + m] & 63);     // staged in LDS
            } else {
                // windows: origin and size once, then its rows and columns
                int ox, oy, n;
                window_of(fp, P.lx, P.ly, ox, oy, n);
                for (int wy = 0; wy < n; ++wy)
                    for (int wx = 0; wx < n; ++wx) member(wy * n + wx, (oy + wy) * 8 + ox + wx);
            }
            const float inv = P.valid ? fast_rcp(B) : 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) tot[c] = g[c] * inv;
            if (scatter) {
                // long tables: through per-lane sums
                if (P.valid) {
                    for (int m = 0; m < K; ++m) {
                        const int j = member_id(fp, P.lx, P.ly, m, a.lut, a.lut_k, P.q);
                        if (j == P.q) continue;
                        const uint2 mj = meta[j];
                        uint32_t dx, dy;
                        if (support_offset<N>(mj.x, ctx.x.base, ctx.y.base, mx, my, dx, dy) && mj.y != 0u) {
                            const float k = ctx.x.wsel(dx) * ctx.y.wsel(dy) * __uint_as_float(mj.y) * inv;
#pragma unroll
                            for (int c = 0; c < C; ++c) atomicAdd(lane_sum + c * 64 + j, k * g[c]);
                        }
                    }
                }
                wave_lds_sync();
#pragma unroll
                for (int c = 0; c < C; ++c) tot[c] += lane_sum[c * 64 + P.q];
            } else {
                // gather from the pixels that name this one: windows (the
                // member index follows from the naming pixel's window) or the
                // table's lists (entries may repeat)
                float4 q4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if constexpr (C >= 1) q4.x = tot[0];
                if constexpr (C >= 2) q4.y = tot[1];
                if constexpr (C >= 4) { q4.z = tot[2]; q4.w = tot[3]; }
                reinterpret_cast<float4*>(qrec)[P.q] = q4;
                wave_lds_sync();
                for (int e = 0; e < rev.n; ++e) {
                    const int idx = rev.list[rev.at + e];
                    const float k = coef[idx];
                    const float4 qp = reinterpret_cast<const float4*>(qrec)[idx & 63];
                    const float qc[4] = {qp.x, qp.y, qp.z, qp.w};
#pragma unroll
                    for (int c = 0; c < C; ++c) tot[c] = fmaf(k, qc[c], tot[c]);
                }
                if (fp == STF_FP_SQUARE3X3 || fp == STF_FP_SQUARE4X4) {
                    const int n = fp == STF_FP_SQUARE3X3 ? 3 : 4;
                    const int x0 = (int)(rev.rect & 15u), x1 = (int)((rev.rect >> 4) & 15u);
                    const int y0 = (int)((rev.rect >> 8) & 15u), y1 = (int)(rev.rect >> 12);
                    for (int py = y0; py <= y1; ++py) {
                        const int row = (P.ly - min(max(py - 1, 0), 8 - n)) * n + P.lx;
                        for (int px = x0; px <= x1; ++px) {
                            const int p = py * 8 + px;
                            if (p == P.q) continue;
                            const float k = coef[(row - min(max(px - 1, 0), 8 - n)) * 64 + p];
                            const float4 qp = reinterpret_cast<const float4*>(qrec)[p];
                            const float qc[4] = {qp.x, qp.y, qp.z, qp.w};
#pragma unroll
                            for (int c = 0; c < C; ++c) tot[c] = fmaf(k, qc[c], tot[c]);
                        }
                    }
                }
                uint64_t bits = rev.bits;
                while (bits) {
                    const int p = (int)__builtin_ctzll(bits);
                    bits &= bits - 1ull;
                    int ox, oy, n;
                    window_of(fp, p & 7, p >> 3, ox, oy, n);
                    const float k = coef[((P.ly - oy) * n + (P.lx - ox)) * 64 + p];
                    const float4 qp = reinterpret_cast<const float4*>(qrec)[p];
                    const float qc[4] = {qp.x, qp.y, qp.z, qp.w};
#pragma unroll
                    for (int c = 0; c < C; ++c) tot[c] = fmaf(k, qc[c], tot[c]);
                }
            }
            wave_lds_sync();                     // read before the window sum reuses the area
        }
        if (use_bins) {
            v4f acc[C];
            onehot_window_sum<C>(merge.wide, P, (sx - (uint32_t)base_x) & mx, (sy - (uint32_t)base_y) & my, tot,
                                 ij, kp, acc);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int c = 0; c < C; ++c) vals[v][c] = acc[c][v];
        } else if (P.valid) {
            atomic_texel<C>(grad, t.w, s, tot, 1.0f);
        }
    }

    // every wave of the workgroup reaches the barriers below, whichever
    // path it took; only waves with bins and an on-screen pixel add
    // lane holds window rows 4 (l / 16) + v, column l % 16
    const int wave = threadIdx.x >> 6;
    const bool contributes = use_bins && __builtin_amdgcn_ballot_w64(P.valid) != 0;
    if (lane == 0) {
        merge.info[wave * 4 + 0] = contributes ? 1 : 0;
        merge.info[wave * 4 + 1] = base_x;
        merge.info[wave * 4 + 2] = base_y;
    }
    __syncthreads();
    // the union of the contributing windows (offsets taken modulo the texture
    // size relative to the first one); the same result in every thread
    int ref = -1, lo_x = 0, hi_x = 0, lo_y = 0, hi_y = 0;
    for (int w = 0; w < kWavesPerGroup; ++w) {
        if (!merge.info[w * 4]) continue;
        if (ref < 0) ref = w;
        const int dx = wrapped_offset(merge.info[w * 4 + 1], merge.info[ref * 4 + 1], mx);
        const int dy = wrapped_offset(merge.info[w * 4 + 2], merge.info[ref * 4 + 2], my);
        lo_x = min(lo_x, dx); hi_x = max(hi_x, dx);
        lo_y = min(lo_y, dy); hi_y = max(hi_y, dy);
    }
    const bool merged = ref >= 0 && hi_x - lo_x + kBinG <= kMergeW && hi_y - lo_y + kBinG <= kMergeH;
    if (merged) {
        const int ux = merge.info[ref * 4 + 1] + lo_x, uy = merge.info[ref * 4 + 2] + lo_y;
        // every wave has passed the barrier above, so no row record is read any more
        for (int e = threadIdx.x; e < kMergeW * kMergeH * C; e += kThreads) merge.v[e] = 0.0f;
        __syncthreads();
        if (contributes) {
            // this window's corner in the area: its offset from the reference window,
            // as the union was formed (in [0, kMergeW - kBinG] x [0, kMergeH - kBinG])
            const int ox = wrapped_offset(base_x, merge.info[ref * 4 + 1], mx) - lo_x;
            const int oy = wrapped_offset(base_y, merge.info[ref * 4 + 2], my) - lo_y;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 4 * kp + v;
                if (i < kBinG && ij < kBinG) {
                    bool any = false;
#pragma unroll
                    for (int c = 0; c < C; ++c) any = any || vals[v][c] != 0.0f;
                    if (any) {
                        float* m = merge.v + ((oy + i) * kMergeW + ox + ij) * C;
#pragma unroll
                        for (int c = 0; c < C; ++c) atomicAdd(m + c, vals[v][c]);
                    }
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kMergeW * kMergeH; e += kThreads) {
            float q[C];
            bool any = false;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                q[c] = merge.v[e * C + c];
                any = any || q[c] != 0.0f;
            }
            if (any) {
                const uint32_t tx = (uint32_t)(ux + e % kMergeW) & mx;
                const uint32_t ty = (uint32_t)(uy + e / kMergeW) & my;
                atomic_texel<C>(grad, t.w, tx | (ty << 16), q, 1.0f);
            }
        }
    } else if (contributes) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 4 * kp + v;
            if (i < kBinG && ij < kBinG) {
                bool any = false;
#pragma unroll
                for (int c = 0; c < C; ++c) any = any || vals[v][c] != 0.0f;
                if (any) {
                    const uint32_t tx = (uint32_t)(base_x + ij) & mx;
                    const uint32_t ty = (uint32_t)(base_y + i) & my;
                    atomic_texel<C>(grad, t.w, tx | (ty << 16), vals[v], 1.0f);
                }
            }
        }
    }
    __syncthreads();             // merge area and window read before the next slot
}

// dL/dout of this lane's pixel for one slot (channels beyond the slot's
// count zero; off-screen pixels zero): one 4-, 8- or 16-byte load.
__device__ __forceinline__ float4 load_dout(const Args& a, int slot, const Pixel& P) {
    float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (!P.valid) return g;
    const int64_t pix = (int64_t)P.py * a.sw + P.px;
    const int ch = a.tex[slot].ch;
    if (ch == 4) {
        g = reinterpret_cast<const float4*>(a.dout[slot])[pix];
    } else if (ch == 2) {
        const float2 v = reinterpret_cast<const float2*>(a.dout[slot])[pix];
        g.x = v.x;
        g.y = v.y;
    } else {
        g.x = a.dout[slot][pix];
    }
    return g;
}

// The adjoint kernels are budgeted for kBwdWaves waves per SIMD (the record
// footprints' kernel for four: its gathers take more registers).
constexpr int kBwdWaves = 5;

template <int FILT, int MODE>
__global__ __launch_bounds__(kThreads, MODE == kModeRecords ? 4 : kBwdWaves) void backward_kernel(Args a) {
    // per wave: bin sums of 1/p or 64 {s, r} records, then the wide area
    // (u64 sums, row records, member coefficients, one-hot operands); the
    // wide areas of the workgroup together form the merge area
    constexpr int kPerWave = kBwdNbFloats;
    static_assert(kPerWave >= 128, "64 {s, r} records fit");
    static_assert(kMergeW * kMergeH * 4 <= kWavesPerGroup * kBwdWideFloats, "merge area fits");
    static_assert(16 * 64 + 64 * 4 <= kBwdWideFloats, "member coefficients and totals fit");
    __shared__ __align__(16) float lds_all[kWavesPerGroup * (kPerWave + kBwdWideFloats)];
    __shared__ int merge_info[kWavesPerGroup * 4];
    float* wide_all = lds_all + kWavesPerGroup * kPerWave;
    const MergeArea merge{wide_all, merge_info, wide_all + (threadIdx.x >> 6) * kBwdWideFloats};
    // the workgroup merges behind barriers: a wave whose tile column is off
    // screen stays (every lane off screen, nothing added)
    Pixel P;
    int bx, by;
    xcd_block(bx, by);
    place_pixel(a, bx * kWavesPerGroup + (threadIdx.x >> 6), by, P);
    const v2f uv = load_uv(a, P.px, P.py);
    P.u = uv.x;
    P.v = uv.y;
    float* lds = lds_all + (threadIdx.x >> 6) * kPerWave;
    // record footprints: where each pick's contributions come from, for the
    // gather; tables of at most kRevMaxK entries are staged in LDS (every
    // thread of the workgroup reaches the barrier)
    __shared__ uint16_t rev_lists[MODE == kModeRecords ? kWavesPerGroup * 64 * kRevMaxK : 1];
    __shared__ uint8_t lut_lds[MODE == kModeRecords ? 64 * kRevMaxK : 1];
    Reverse rev;
    if constexpr (MODE == kModeRecords) {
        if (a.footprint == STF_FP_LUT && a.lut_k <= kRevMaxK) {
            for (int i = threadIdx.x; i < 64 * a.lut_k; i += kThreads) lut_lds[i] = a.lut[i];
            __syncthreads();
        }
        if (a.footprint == STF_FP_SQUARE3X3 || a.footprint == STF_FP_SQUARE4X4)
            rev.rect = reverse_rect(a.footprint == STF_FP_SQUARE3X3 ? 3 : 4, P.lx, P.ly);
        else if (a.footprint != STF_FP_LUT)
            rev.bits = reverse_members(a.footprint, P.lx, P.ly);
        else if (a.lut_k <= kRevMaxK)
            build_reverse_table(a.lut_k, lut_lds, P, reinterpret_cast<int*>(lds),
                                rev_lists + (threadIdx.x >> 6) * 64 * kRevMaxK, rev);
    }
    SelCtx<FILT> ctx;
    // dL/dout of the pixel, one vector load per slot, the next slot's
    // requested before the current slot's work
    float4 gcur = load_dout(a, 0, P), gnext = gcur;
    for (int slot = 0; slot < a.ntex; ++slot) {
        if (slot + 1 < a.ntex) gnext = load_dout(a, slot + 1, P);
        uint32_t hx, hy;
        keyed_uniforms(a, P, slot, hx, hy);
        ctx.update(P, a.tex[slot].w, a.tex[slot].h);
        const int ch = a.tex[slot].ch;
        if (ch == 4) backward_slot<FILT, MODE, 4>(a, slot, P, ctx, hx, hy, gcur, lds, merge, rev, lut_lds);
        else if (ch == 2) backward_slot<FILT, MODE, 2>(a, slot, P, ctx, hx, hy, gcur, lds, merge, rev, lut_lds);
        else backward_slot<FILT, MODE, 1>(a, slot, P, ctx, hx, hy, gcur, lds, merge, rev, lut_lds);
        gcur = gnext;
    }
}

}  // namespace stf
