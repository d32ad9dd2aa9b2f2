// Host side of the C ABI declared in include/stf.h: argument validation,
// kernel selection and launches. The kernels live in stf_kernels.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "stf_decoder_backward.h"
#include "stf_backward.h"
#include "stf_status.h"

// The whole-tile kernels keep their 64-bit sums zero between textures of one
// size (the finalisation clears them); the latent decode's LDS scratch, used
// in between, must stay below them.
static_assert(stf::kDedupBytes <= stf::kAccFloatOffset * 4, "decode scratch overlaps the whole-tile sums");

namespace stf {

// Pack the decoder MLP for decode_latent. BF16: A operands in lane order
// with the K permutation of dec_unit, b1 folded into layer 1 as K index 8,
// b2 and b3 as FP32 accumulator start values. FP8: per-layer weight scale
// s_l = max|W_l| / 448, A operands W_l / s_l as FP8 E4M3 in the same lane
// order (8 one-byte K values per lane), every bias as b_l / s_l start
// values. One workgroup of 256 threads.
__global__ __launch_bounds__(256) void decoder_pack_kernel(stf_mlp m, uint8_t* out) {
    __shared__ float red[3][256];
    DecHeader* hd = reinterpret_cast<DecHeader*>(out);
    const bool fp8 = m.precision == STF_DECODER_FP8;
    float sc[3] = {1.0f, 1.0f, 1.0f};
    if (fp8) {
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
        for (int i = threadIdx.x; i < 64 * 8; i += 256) a0 = fmaxf(a0, fabsf(m.w1[i]));
        for (int i = threadIdx.x; i < 64 * 64; i += 256) a1 = fmaxf(a1, fabsf(m.w2[i]));
        for (int i = threadIdx.x; i < 4 * 64; i += 256) a2 = fmaxf(a2, fabsf(m.w3[i]));
        red[0][threadIdx.x] = a0;
        red[1][threadIdx.x] = a1;
        red[2][threadIdx.x] = a2;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                for (int l = 0; l < 3; ++l) red[l][threadIdx.x] = fmaxf(red[l][threadIdx.x], red[l][threadIdx.x + w]);
            __syncthreads();
        }
        for (int l = 0; l < 3; ++l) sc[l] = red[l][0] > 0.0f ? red[l][0] / 448.0f : 1.0f;
    }
    if (threadIdx.x == 0) {
        hd->precision = fp8 ? STF_DECODER_FP8 : STF_DECODER_BF16;
        for (int l = 0; l < 3; ++l) hd->scale[l] = sc[l];
    }
    for (int idx = threadIdx.x; idx < 14 * 64; idx += blockDim.x) {
        const int o = idx >> 6, lane = idx & 63, h = lane >> 5, row = lane & 31;
        float v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = 8 * h + t;
            if (o < 2) {                                      // layer 1, row tile o
                const int u = 32 * o + row;
                v[t] = h == 0 ? m.w1[u * 8 + t] / sc[0] : ((t == 0 && !fp8) ? m.b1[u] : 0.0f);
            } else if (o < 10) {                              // layer 2, row tile, K step
                const int mt = (o - 2) >> 2, st = (o - 2) & 3;
                v[t] = m.w2[(32 * mt + row) * 64 + dec_unit(st, k)] / sc[1];
            } else {                                          // layer 3, K step (rows >= 4 are padding)
                v[t] = row < 4 ? m.w3[row * 64 + dec_unit(o - 10, k)] / sc[2] : 0.0f;
            }
        }
        if (fp8) {
            uint32_t w[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                int x = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * i], v[4 * i + 1], 0, false);
                x = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * i + 2], v[4 * i + 3], x, true);
                w[i] = (uint32_t)x;
            }
            reinterpret_cast<uint2*>(out + kF8A1)[idx] = make_uint2(w[0], w[1]);
        } else {
            u32x4 q;
#pragma unroll
            for (int i = 0; i < 4; ++i) q[i] = pack_bf16(v[2 * i], v[2 * i + 1]);
            reinterpret_cast<u32x4*>(out + kDecA1)[idx] = q;
        }
    }
    float* C1 = reinterpret_cast<float*>(out + kF8C1);
    float* C2 = reinterpret_cast<float*>(out + (fp8 ? kF8C2 : kDecC2));
    float* C3 = reinterpret_cast<float*>(out + (fp8 ? kF8C3 : kDecC3));
    for (int idx = threadIdx.x; idx < 64; idx += blockDim.x) {
        const int mt = idx >> 5, h = (idx >> 4) & 1, j = idx & 15;
        if (fp8) C1[idx] = m.b1[32 * mt + acc_row(j, h)] / sc[0];
        C2[idx] = m.b2[32 * mt + acc_row(j, h)] / sc[1];
    }
    for (int idx = threadIdx.x; idx < 32; idx += blockDim.x) {
        const int h = idx >> 4, j = idx & 15, r = acc_row(j, h);
        C3[idx] = r < 4 ? m.b3[r] / sc[2] : 0.0f;
    }
}

}  // namespace stf

// ============================================================================
// host side of the C ABI
// ============================================================================

namespace stf_host {

namespace {
thread_local std::string g_last_error;
}

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

const char* last_error() { return g_last_error.c_str(); }

}  // namespace stf_host

namespace {

using stf_host::fail;

// Channels of the stored texel (8 for latent grids) and of the filtered,
// decoded texel (4 for latent grids).
int stored_channels(int fmt) {
    switch (fmt) {
    case STF_RGBA8_UNORM: case STF_RGBA16F: case STF_RGBA32F: case STF_RGBA_BF16: case STF_RGBA_FP8: return 4;
    case STF_RG16F: return 2;
    case STF_R8_UNORM: case STF_R32F: return 1;
    case STF_LATENT8_F16: case STF_LATENT8_BF16: case STF_LATENT8_FP8: return 8;
    default: return 0;
    }
}

bool is_latent(int fmt) { return fmt == STF_LATENT8_F16 || fmt == STF_LATENT8_BF16 || fmt == STF_LATENT8_FP8; }

int format_channels(int fmt) { return is_latent(fmt) ? 4 : stored_channels(fmt); }

int format_bytes(int fmt) {
    switch (fmt) {
    case STF_RGBA8_UNORM: case STF_RG16F: case STF_R32F: case STF_RGBA_FP8: return 4;
    case STF_RGBA16F: case STF_RGBA_BF16: case STF_LATENT8_FP8: return 8;
    case STF_RGBA32F: case STF_LATENT8_F16: case STF_LATENT8_BF16: return 16;
    case STF_R8_UNORM: return 1;
    default: return 0;
    }
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Validates everything the kernels assume and fills the kernel arguments.
// allow_latent: latent textures are accepted (with a decoder); all latent
// textures of one call share one packed decoder, stored in a.dec.
int prepare(const stf_texture* tex, int32_t ntex, const stf_screen* scr, const stf_params* p,
            bool need_data, stf::Args& a, bool allow_latent = false) {
    std::memset(&a, 0, sizeof a);
    if (tex == nullptr || scr == nullptr || p == nullptr)
        return fail(STF_EINVAL, "null descriptor pointer");
    if (ntex < 1 || ntex > STF_MAX_TEXTURES)
        return fail(STF_EINVAL, "ntex=%d outside 1..%d", ntex, STF_MAX_TEXTURES);
    if (scr->uv == nullptr) return fail(STF_EINVAL, "screen uv is null");
    if (scr->width < 1 || scr->height < 1 || scr->width > STF_MAX_SCREEN || scr->height > STF_MAX_SCREEN)
        return fail(STF_EINVAL, "screen %dx%d outside 1..%d", scr->width, scr->height, STF_MAX_SCREEN);
    if ((reinterpret_cast<uintptr_t>(scr->uv) & 7) != 0) return fail(STF_EINVAL, "uv not 8-byte aligned");
    if (p->filter != STF_BILINEAR && p->filter != STF_BICUBIC_BSPLINE)
        return fail(STF_EINVAL, "unknown filter %d", p->filter);
    if (p->address != STF_WRAP) return fail(STF_EUNSUPPORTED, "address mode %d not supported (WRAP only)", p->address);
    for (int i = 0; i < ntex; ++i) {
        const stf_texture& t = tex[i];
        const int ch = format_channels(t.format);
        const int bpp = format_bytes(t.format);
        if (ch == 0) return fail(STF_EINVAL, "texture %d: unknown format %d", i, t.format);
        if (t.reserved != 0) return fail(STF_EINVAL, "texture %d: reserved field must be 0", i);
        if (is_latent(t.format)) {
            if (!allow_latent)
                return fail(STF_EUNSUPPORTED, "texture %d: latent formats are not supported by this entry point", i);
            if (t.decoder == nullptr) return fail(STF_EINVAL, "texture %d: latent format without a decoder", i);
            if ((reinterpret_cast<uintptr_t>(t.decoder) % 16) != 0)
                return fail(STF_EINVAL, "texture %d: decoder not aligned to 16 bytes", i);
            if (a.dec != nullptr && a.dec != static_cast<const uint8_t*>(t.decoder))
                return fail(STF_EUNSUPPORTED, "texture %d: one call supports one decoder for all latent textures", i);
            a.dec = static_cast<const uint8_t*>(t.decoder);
        } else if (t.decoder != nullptr) {
            return fail(STF_EINVAL, "texture %d: decoder given for a format that is not latent", i);
        }
        if (need_data && t.data == nullptr) return fail(STF_EINVAL, "texture %d: data is null", i);
        if (!pow2(t.width) || !pow2(t.height) || t.width < 4 || t.height < 4 || t.width > 32768 || t.height > 32768)
            return fail(STF_EINVAL, "texture %d: %dx%d must be powers of two in 4..32768 for WRAP", i, t.width, t.height);
        if (need_data) {
            if (t.pitch_bytes < (int64_t)t.width * bpp || t.pitch_bytes % 16 != 0)
                return fail(STF_EINVAL, "texture %d: pitch %lld must be a multiple of 16 and >= width %d x %d bytes",
                            i, (long long)t.pitch_bytes, t.width, bpp);
            if ((reinterpret_cast<uintptr_t>(t.data) % 16) != 0)
                return fail(STF_EINVAL, "texture %d: data not aligned to 16 bytes", i);
        }
        a.tex[i].data = static_cast<const uint8_t*>(t.data);
        a.tex[i].pitch = t.pitch_bytes;
        a.tex[i].w = t.width;
        a.tex[i].h = t.height;
        a.tex[i].fmt = t.format;
        a.tex[i].ch = ch;
        a.tex[i].has_scale = t.scale != nullptr;
        for (int c = 0; c < 8; ++c) a.tex[i].scale[c] = 1.0f;
        if (t.scale != nullptr) {
            for (int c = 0; c < stored_channels(t.format); ++c) {
                if (!std::isfinite(t.scale[c])) return fail(STF_EINVAL, "texture %d: scale[%d] is not finite", i, c);
                a.tex[i].scale[c] = t.scale[c];
            }
        }
    }
    a.uv = scr->uv;
    a.ntex = ntex;
    a.sw = scr->width;
    a.sh = scr->height;
    a.seed = p->seed;
    a.frame = p->frame;
    if ((p->flags & ~(STF_SHARE_SELECTION | STF_FLOAT_BIN_SUMS)) != 0)
        return fail(STF_EINVAL, "unknown params flags 0x%x", p->flags);
    a.flags = (p->flags & STF_FLOAT_BIN_SUMS) ? stf::kFlagFloatBinSums : 0;
    if (p->reserved != 0) return fail(STF_EINVAL, "params reserved field must be 0");
    for (int i = 0; i < ntex; ++i) {
        a.leader[i] = i;
        if (p->flags & STF_SHARE_SELECTION)
            for (int j = 0; j < i; ++j)
                if (tex[j].width == tex[i].width && tex[j].height == tex[i].height) {
                    a.leader[i] = j;
                    break;
                }
    }
    return STF_OK;
}

int check_outputs(float* const* out, int32_t ntex) {
    if (out == nullptr) return fail(STF_EINVAL, "out array is null");
    for (int i = 0; i < ntex; ++i) {
        if (out[i] == nullptr) return fail(STF_EINVAL, "out[%d] is null", i);
        if ((reinterpret_cast<uintptr_t>(out[i]) & 15) != 0) return fail(STF_EINVAL, "out[%d] not 16-byte aligned", i);
    }
    return STF_OK;
}

int check_reuse(const stf_reuse* r) {
    if (r == nullptr) return fail(STF_EINVAL, "reuse descriptor is null");
    if (r->footprint < STF_FP_SELF || r->footprint > STF_FP_LUT)
        return fail(STF_EINVAL, "unknown footprint %d", r->footprint);
    if (r->footprint == STF_FP_LUT) {
        if (r->lut == nullptr) return fail(STF_EINVAL, "footprint LUT requires a lut pointer");
        if (r->lut_k < 1 || r->lut_k > 64) return fail(STF_EINVAL, "lut_k=%d outside 1..64", r->lut_k);
    }
    if ((r->flags & ~(STF_REUSE_EXACT_FILTERING | STF_REUSE_CLAMP)) != 0)
        return fail(STF_EINVAL, "unknown reuse flags 0x%x", r->flags);
    if (r->estimator < STF_EST_WIS || r->estimator > STF_EST_REGRESSION)
        return fail(STF_EINVAL, "unknown estimator %d", r->estimator);
    if ((r->flags & STF_REUSE_EXACT_FILTERING) && (r->estimator != STF_EST_WIS || (r->flags & STF_REUSE_CLAMP)))
        return fail(STF_EUNSUPPORTED, "exact filtering combines with the plain Eq. (14) estimator only");
    return STF_OK;
}


int finish_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(STF_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return STF_OK;
}

int forward(const stf_texture* tex, int32_t ntex, const stf_screen* scr, const stf_params* p,
            const stf_reuse* r, float* const* out, int32_t* sel, void* hip_stream) {
    stf_host::clear_error();
    stf::Args a;
    int rc = prepare(tex, ntex, scr, p, true, a, true);
    if (rc != STF_OK) return rc;
    if ((rc = check_outputs(out, ntex)) != STF_OK) return rc;
    if (sel != nullptr && (reinterpret_cast<uintptr_t>(sel) & 7) != 0) return fail(STF_EINVAL, "sel not 8-byte aligned");
    int mode = stf::kModeStf;
    if (r != nullptr) {
        if ((rc = check_reuse(r)) != STF_OK) return rc;
        a.footprint = r->footprint;
        a.lut = r->lut;
        a.lut_k = r->lut_k;
        a.flags |= r->flags;
        switch (r->footprint) {
        case STF_FP_SELF: mode = stf::kModeStf; break;
        case STF_FP_QUAD2X2: mode = stf::kModeQuad; break;
        case STF_FP_TILE8X8: mode = stf::kModeBins; break;
        default: mode = stf::kModeRecords; break;
        }
    }
    for (int i = 0; i < ntex; ++i) a.out[i] = out[i];
    a.sel = sel;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const bool cubic = p->filter == STF_BICUBIC_BSPLINE;
    if (r != nullptr && (r->estimator != STF_EST_WIS || (r->flags & STF_REUSE_CLAMP))) {
        if (a.dec != nullptr) return fail(STF_EUNSUPPORTED, "comparison estimators do not decode latent textures");
        a.estimator = r->estimator;
        if (cubic) hipLaunchKernelGGL((stf::estimator_kernel<1>), stf::grid_of(a), dim3(stf::kThreads), 0, s, a);
        else hipLaunchKernelGGL((stf::estimator_kernel<0>), stf::grid_of(a), dim3(stf::kThreads), 0, s, a);
        return finish_launch("estimator");
    }
    switch (mode) {
    case stf::kModeStf: cubic ? stf::launch_forward<1, stf::kModeStf>(a, s) : stf::launch_forward<0, stf::kModeStf>(a, s); break;
    case stf::kModeQuad: cubic ? stf::launch_forward<1, stf::kModeQuad>(a, s) : stf::launch_forward<0, stf::kModeQuad>(a, s); break;
    case stf::kModeRecords: cubic ? stf::launch_forward<1, stf::kModeRecords>(a, s) : stf::launch_forward<0, stf::kModeRecords>(a, s); break;
    default: cubic ? stf::launch_forward<1, stf::kModeBins>(a, s) : stf::launch_forward<0, stf::kModeBins>(a, s); break;
    }
    return finish_launch("forward");
}

}  // namespace

extern "C" {

int stf_filter(const stf_texture* tex, int32_t ntex, const stf_screen* scr, const stf_params* p,
               float* const* out, int32_t* sel, void* hip_stream) {
    return forward(tex, ntex, scr, p, nullptr, out, sel, hip_stream);
}

int stf_filter_reuse(const stf_texture* tex, int32_t ntex, const stf_screen* scr, const stf_params* p,
                     const stf_reuse* r, float* const* out, int32_t* sel, void* hip_stream) {
    if (r == nullptr) {
        stf_host::clear_error();
        return fail(STF_EINVAL, "reuse descriptor is null");
    }
    return forward(tex, ntex, scr, p, r, out, sel, hip_stream);
}

int stf_filter_reference(const stf_texture* tex, int32_t ntex, const stf_screen* scr, const stf_params* p,
                         float* const* out, void* hip_stream) {
    stf_host::clear_error();
    stf::Args a;
    int rc = prepare(tex, ntex, scr, p, true, a, true);
    if (rc != STF_OK) return rc;
    if ((rc = check_outputs(out, ntex)) != STF_OK) return rc;
    for (int i = 0; i < ntex; ++i) a.out[i] = out[i];
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const dim3 g = stf::grid_of(a), b(stf::kThreads);
    const bool cubic = p->filter == STF_BICUBIC_BSPLINE;
    if (a.dec != nullptr) {
        if (cubic) hipLaunchKernelGGL((stf::reference_kernel<1, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((stf::reference_kernel<0, true>), g, b, 0, s, a);
    } else {
        if (cubic) hipLaunchKernelGGL((stf::reference_kernel<1, false>), g, b, 0, s, a);
        else hipLaunchKernelGGL((stf::reference_kernel<0, false>), g, b, 0, s, a);
    }
    return finish_launch("reference");
}

int stf_decoder_pack(const stf_mlp* mlp, void* packed, void* hip_stream) {
    stf_host::clear_error();
    if (mlp == nullptr || packed == nullptr) return fail(STF_EINVAL, "null mlp descriptor or packed buffer");
    const float* ws[6] = {mlp->w1, mlp->b1, mlp->w2, mlp->b2, mlp->w3, mlp->b3};
    for (int i = 0; i < 6; ++i) {
        if (ws[i] == nullptr) return fail(STF_EINVAL, "mlp array %d is null", i);
        if ((reinterpret_cast<uintptr_t>(ws[i]) & 3) != 0) return fail(STF_EINVAL, "mlp array %d not 4-byte aligned", i);
    }
    if ((reinterpret_cast<uintptr_t>(packed) & 15) != 0) return fail(STF_EINVAL, "packed buffer not aligned to 16 bytes");
    if (mlp->precision != STF_DECODER_BF16 && mlp->precision != STF_DECODER_FP8)
        return fail(STF_EINVAL, "unknown decoder precision %d", mlp->precision);
    if (mlp->reserved != 0) return fail(STF_EINVAL, "mlp reserved field must be 0");
    static_assert(stf::kDecBytes == STF_DECODER_BYTES, "packed decoder size");
    hipLaunchKernelGGL(stf::decoder_pack_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(hip_stream), *mlp,
                       static_cast<uint8_t*>(packed));
    return finish_launch("decoder pack");
}

int stf_backward(const stf_texture* tex, int32_t ntex, const stf_screen* scr, const stf_params* p,
                 const stf_reuse* r, const float* const* dout, float* const* dtex, void* hip_stream) {
    stf_host::clear_error();
    stf::Args a;
    int rc = prepare(tex, ntex, scr, p, false, a);
    if (rc != STF_OK) return rc;
    if ((rc = check_reuse(r)) != STF_OK) return rc;
    if (r->flags & (STF_REUSE_EXACT_FILTERING | STF_REUSE_CLAMP) || r->estimator != STF_EST_WIS)
        return fail(STF_EUNSUPPORTED, "the adjoint covers the plain Eq. (14) estimator only");
    if (dout == nullptr || dtex == nullptr) return fail(STF_EINVAL, "dout/dtex arrays are null");
    for (int i = 0; i < ntex; ++i) {
        if (dout[i] == nullptr || dtex[i] == nullptr) return fail(STF_EINVAL, "dout[%d]/dtex[%d] is null", i, i);
        const uintptr_t va = (uintptr_t)(4 * a.tex[i].ch) - 1;     // dout is read one pixel vector at a time
        if ((reinterpret_cast<uintptr_t>(dout[i]) & va) || (reinterpret_cast<uintptr_t>(dtex[i]) & 3))
            return fail(STF_EINVAL, "dout[%d] not %d-byte or dtex[%d] not 4-byte aligned", i, 4 * a.tex[i].ch, i);
        a.out[i] = dtex[i];
        a.dout[i] = dout[i];
    }
    a.footprint = r->footprint;
    a.lut = r->lut;
    a.lut_k = r->lut_k;
    int mode;
    switch (r->footprint) {
    case STF_FP_SELF: mode = stf::kModeStf; break;
    case STF_FP_QUAD2X2: mode = stf::kModeQuad; break;
    case STF_FP_TILE8X8: mode = stf::kModeBins; break;
    default: mode = stf::kModeRecords; break;
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const bool cubic = p->filter == STF_BICUBIC_BSPLINE;
    const dim3 g = stf::grid_of(a), b(stf::kThreads);
#define STF_BW(F, M) hipLaunchKernelGGL((stf::backward_kernel<F, M>), g, b, 0, s, a)
    switch (mode) {
    case stf::kModeStf: if (cubic) STF_BW(1, stf::kModeStf); else STF_BW(0, stf::kModeStf); break;
    case stf::kModeQuad: if (cubic) STF_BW(1, stf::kModeQuad); else STF_BW(0, stf::kModeQuad); break;
    case stf::kModeRecords: if (cubic) STF_BW(1, stf::kModeRecords); else STF_BW(0, stf::kModeRecords); break;
    default: if (cubic) STF_BW(1, stf::kModeBins); else STF_BW(0, stf::kModeBins); break;
    }
#undef STF_BW
    return finish_launch("backward");
}

}  // extern "C"

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace layout of stf_backward_decoder: per texture the dense FP32
// gradient of its decoded texels [th * tw][4], then one slot of weight
// gradients per decoder-backward wavefront of every texture, then the
// partial sums of the reduction's first step.
struct DecBwdLayout {
    size_t g[STF_MAX_TEXTURES];
    size_t list[STF_MAX_TEXTURES], count[STF_MAX_TEXTURES];   // the block mask follows g directly
    int groups[STF_MAX_TEXTURES];     // workgroups of the decoder kernel, one weight-gradient slot each
    int total_groups = 0;
    size_t partial = 0, level2 = 0, total = 0;
};

DecBwdLayout dec_bwd_layout(const stf_texture* tex, int32_t ntex) {
    DecBwdLayout l;
    size_t off = 0;
    for (int i = 0; i < ntex; ++i) {
        const int64_t n = (int64_t)tex[i].width * tex[i].height;
        const int64_t blocks = (n + stf::kDbN - 1) / stf::kDbN;
        l.g[i] = off;                                   // n * 16 is a multiple of 256 (n >= 16, a power of two)
        off += align256((size_t)n * 16 + (size_t)(blocks + 31) / 32 * 4);
        l.list[i] = off;
        off += align256((size_t)blocks * 4);
        l.count[i] = off;
        off += 256;
        const int64_t waves = std::min<int64_t>(blocks, stf::kDecBwdMaxWaves);
        l.groups[i] = (int)((waves + stf::kDbWaves - 1) / stf::kDbWaves);
        l.total_groups += l.groups[i];
    }
    l.partial = off;
    l.level2 = off + align256((size_t)l.total_groups * stf::kGradFloats * 4);
    l.total = l.level2 + align256((size_t)stf::kReduceSplits * stf::kGradFloats * 4);
    return l;
}

// The latent textures of a decoder adjoint call: latent formats, one decoder.
int check_decoder_textures(const stf_texture* tex, int32_t ntex) {
    if (tex == nullptr) return fail(STF_EINVAL, "null texture descriptors");
    if (ntex < 1 || ntex > STF_MAX_TEXTURES) return fail(STF_EINVAL, "ntex=%d outside 1..%d", ntex, STF_MAX_TEXTURES);
    for (int i = 0; i < ntex; ++i) {
        if (!is_latent(tex[i].format))
            return fail(STF_EINVAL, "texture %d: the decoder adjoint takes latent textures only", i);
        if (!pow2(tex[i].width) || !pow2(tex[i].height) || tex[i].width < 4 || tex[i].height < 4 ||
            tex[i].width > 32768 || tex[i].height > 32768)
            return fail(STF_EINVAL, "texture %d: %dx%d must be powers of two in 4..32768", i, tex[i].width,
                        tex[i].height);
    }
    return STF_OK;
}

}  // namespace

extern "C" {

int64_t stf_backward_decoder_workspace_bytes(const stf_texture* tex, int32_t ntex) {
    stf_host::clear_error();
    if (check_decoder_textures(tex, ntex) != STF_OK) return -1;
    return (int64_t)dec_bwd_layout(tex, ntex).total;
}

int stf_backward_decoder(const stf_texture* tex, int32_t ntex, const stf_screen* scr, const stf_params* p,
                         const stf_reuse* r, const float* const* dout, const stf_mlp* mlp, float* const* dlatent,
                         const stf_mlp_grad* dmlp, void* workspace, int64_t workspace_bytes, void* hip_stream) {
    stf_host::clear_error();
    int rc = check_decoder_textures(tex, ntex);
    if (rc != STF_OK) return rc;
    stf::Args a;
    if ((rc = prepare(tex, ntex, scr, p, true, a, true)) != STF_OK) return rc;
    if ((rc = check_reuse(r)) != STF_OK) return rc;
    if (r->flags & (STF_REUSE_EXACT_FILTERING | STF_REUSE_CLAMP) || r->estimator != STF_EST_WIS)
        return fail(STF_EUNSUPPORTED, "the adjoint covers the plain Eq. (14) estimator only");
    if (mlp == nullptr || dmlp == nullptr) return fail(STF_EINVAL, "mlp or its gradient descriptor is null");
    const float* ws[6] = {mlp->w1, mlp->b1, mlp->w2, mlp->b2, mlp->w3, mlp->b3};
    float* const gs[6] = {dmlp->w1, dmlp->b1, dmlp->w2, dmlp->b2, dmlp->w3, dmlp->b3};
    for (int i = 0; i < 6; ++i) {
        if (ws[i] == nullptr || gs[i] == nullptr) return fail(STF_EINVAL, "mlp array %d or its gradient is null", i);
        if ((reinterpret_cast<uintptr_t>(ws[i]) & 3) || (reinterpret_cast<uintptr_t>(gs[i]) & 3))
            return fail(STF_EINVAL, "mlp array %d or its gradient not 4-byte aligned", i);
    }
    if (mlp->precision != STF_DECODER_BF16 && mlp->precision != STF_DECODER_FP8)
        return fail(STF_EINVAL, "unknown decoder precision %d", mlp->precision);
    if (mlp->reserved != 0) return fail(STF_EINVAL, "mlp reserved field must be 0");
    if (dout == nullptr || dlatent == nullptr) return fail(STF_EINVAL, "dout/dlatent arrays are null");
    for (int i = 0; i < ntex; ++i) {
        if (dout[i] == nullptr || dlatent[i] == nullptr) return fail(STF_EINVAL, "dout[%d]/dlatent[%d] is null", i, i);
        if ((reinterpret_cast<uintptr_t>(dout[i]) & 15) || (reinterpret_cast<uintptr_t>(dlatent[i]) & 3))
            return fail(STF_EINVAL, "dout[%d] not 16-byte or dlatent[%d] not 4-byte aligned", i, i);
    }
    const DecBwdLayout l = dec_bwd_layout(tex, ntex);
    if (workspace == nullptr) return fail(STF_EINVAL, "workspace is null");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(STF_EINVAL, "workspace not aligned to 256 bytes");
    if (workspace_bytes < (int64_t)l.total)
        return fail(STF_EINVAL, "workspace of %lld bytes, %lld needed", (long long)workspace_bytes, (long long)l.total);
    uint8_t* wsp = static_cast<uint8_t*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);

    // 1. the texel adjoint of every slot into its dense FP32 buffer (cleared
    //    first); the latent scale precedes the decoder, so none applies here
    for (int i = 0; i < ntex; ++i) {
        float* g = reinterpret_cast<float*>(wsp + l.g[i]);
        const int64_t texels = (int64_t)tex[i].width * tex[i].height;
        const int64_t n = texels * 4 + ((texels + stf::kDbN - 1) / stf::kDbN + 31) / 32;   // g, then the block mask
        hipLaunchKernelGGL(stf::zero_fill_kernel, dim3((unsigned)std::min<int64_t>((n / 4 + 255) / 256 + 1, 1024)),
                           dim3(256), 0, s, g, n);     // g is 256-byte aligned
        a.out[i] = g;
        a.dout[i] = dout[i];
        a.tex[i].has_scale = 0;
        for (int c = 0; c < 8; ++c) a.tex[i].scale[c] = 1.0f;
    }
    a.footprint = r->footprint;
    a.lut = r->lut;
    a.lut_k = r->lut_k;
    const bool cubic = p->filter == STF_BICUBIC_BSPLINE;
    const dim3 grid = stf::grid_of(a), block(stf::kThreads);
#define STF_BW(F, M) hipLaunchKernelGGL((stf::backward_kernel<F, M>), grid, block, 0, s, a)
    switch (r->footprint) {
    case STF_FP_SELF: if (cubic) STF_BW(1, stf::kModeStf); else STF_BW(0, stf::kModeStf); break;
    case STF_FP_QUAD2X2: if (cubic) STF_BW(1, stf::kModeQuad); else STF_BW(0, stf::kModeQuad); break;
    case STF_FP_TILE8X8: if (cubic) STF_BW(1, stf::kModeBins); else STF_BW(0, stf::kModeBins); break;
    default: if (cubic) STF_BW(1, stf::kModeRecords); else STF_BW(0, stf::kModeRecords); break;
    }
#undef STF_BW
    // 2. per texture: the blocks some gradient reaches, listed in order, then
    //    through the decoder; 3. the weight gradients summed
    float* partial = reinterpret_cast<float*>(wsp + l.partial);
    stf::SlotRanges ranges;
    ranges.ntex = ntex;
    int slot0 = 0;
    for (int i = 0; i < ntex; ++i) {
        stf::DecBwdArgs d;
        d.data = static_cast<const uint8_t*>(tex[i].data);
        d.pitch = tex[i].pitch_bytes;
        d.tw = tex[i].width;
        d.th = tex[i].height;
        d.fmt = tex[i].format;
        d.nblocks = (int)(((int64_t)d.tw * d.th + stf::kDbN - 1) / stf::kDbN);
        for (int c = 0; c < 8; ++c) d.scale[c] = tex[i].scale != nullptr ? tex[i].scale[c] : 1.0f;
        d.g = reinterpret_cast<const float*>(wsp + l.g[i]);
        uint32_t* mask = reinterpret_cast<uint32_t*>(wsp + l.g[i] + (size_t)d.tw * d.th * 16);
        int32_t* list = reinterpret_cast<int32_t*>(wsp + l.list[i]);
        int32_t* count = reinterpret_cast<int32_t*>(wsp + l.count[i]);
        hipLaunchKernelGGL(stf::decoder_block_mask_kernel, dim3((unsigned)((d.nblocks + 15) / 16)), dim3(256), 0, s, d.g,
                           (int64_t)d.tw * d.th, d.nblocks, mask);
        hipLaunchKernelGGL(stf::decoder_block_list_kernel, dim3(1), dim3(stf::kListThreads), 0, s,
                           static_cast<const uint32_t*>(mask), d.nblocks, list, count);
        d.list = list;
        d.count = count;
        ranges.off[i] = slot0;
        ranges.groups[i] = l.groups[i];
        ranges.count[i] = count;
        d.w1 = mlp->w1;
        d.b1 = mlp->b1;
        d.w2 = mlp->w2;
        d.b2 = mlp->b2;
        d.w3 = mlp->w3;
        d.dlat = dlatent[i];
        d.partial = partial + (size_t)slot0 * stf::kGradFloats;
        hipLaunchKernelGGL(stf::decoder_backward_kernel, dim3((unsigned)l.groups[i]), dim3(64 * stf::kDbWaves), 0, s, d);
        slot0 += l.groups[i];
    }
    stf::MlpGradPtrs o;
    for (int i = 0; i < 6; ++i) o.p[i] = gs[i];
    float* level2 = reinterpret_cast<float*>(wsp + l.level2);
    hipLaunchKernelGGL(stf::decoder_grad_partial_kernel, dim3((stf::kGradFloats + 255) / 256, stf::kReduceSplits),
                       dim3(256), 0, s, static_cast<const float*>(partial), ranges, level2);
    hipLaunchKernelGGL(stf::decoder_grad_reduce_kernel, dim3((stf::kGradFloats + 255) / 256), dim3(256), 0, s,
                       static_cast<const float*>(level2), o);
    return finish_launch("decoder backward");
}

const char* stf_last_error(void) { return stf_host::last_error(); }

int stf_version(void) { return STF_VERSION; }

}  // extern "C"
