/*
 * stf.h - C ABI of the MI355X (gfx950) stochastic texture filtering library.
 *
 * Implements stochastic texture filtering (STF) with sample reuse under
 * magnification from Wronski, Pharr and Akenine-Moeller, "Improved
 * Stochastic Texture Filtering Through Sample Reuse" (2025):
 *   - one-tap STF: each pixel picks one texel with probability equal to its
 *     filter weight and returns it unweighted (Sec. 2.2, Sec. S1);
 *   - sample reuse: pixels of one 8x8 screen tile (one 64-lane wavefront)
 *     exchange their picked texels and combine them with the weighted
 *     importance sampling estimator of Eq. (14) (Sec. 4.2, Sec. 4.5);
 *   - the deterministic filter of Eq. (3) as ground truth;
 *   - the adjoint of Eq. (14) with respect to the texels.
 *
 * Conventions shared by every entry point:
 *   - Pointers named "device" are HIP device pointers owned by the caller;
 *     the library never frees or retains them. Descriptor structs and the
 *     arrays of output pointers are host memory read during the call only.
 *   - Every call validates its arguments on the host before anything is
 *     enqueued; on error nothing is launched, the return value is negative
 *     and stf_last_error() describes the problem.
 *   - Work is enqueued asynchronously on `hip_stream` (a hipStream_t; NULL
 *     means the default stream). No call synchronises or allocates.
 *   - The forward outputs are a pure function of the inputs, seed, frame and
 *     texture slot index.
 *   - Screen layout: UV is FP32 [height][width][2] row-major (u then v);
 *     outputs are FP32 [height][width][C] row-major, C = channels of the
 *     texture format (4 for latent formats, which are decoded); pixel
 *     (px, py) has its centre at (px+1/2, py+1/2).
 *   - Texture layout: row y starts at data + y * pitch_bytes; texels are
 *     tightly packed within a row. Texel (0,0) is the first texel. The base
 *     address and pitch_bytes are multiples of 16 and the allocation holds
 *     height * pitch_bytes bytes (kernels read aligned 16-byte blocks inside
 *     a row).
 *   - Texel-space coordinate of a texture coordinate u on a texture of
 *     size W: x = u * W - 0.5 in FP32 (Sec. 4.5 listing); the sub-texel
 *     fraction is quantised to 16 bits.
 *   - Addressing: STF_WRAP on power-of-two textures of 4..32768 texels per
 *     axis; texel identity is the index modulo the texture size.
 */
#ifndef STF_H
#define STF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STF_VERSION 2
#define STF_MAX_TEXTURES 4
#define STF_MAX_SCREEN 32768

typedef enum stf_status {
    STF_OK = 0,
    STF_EINVAL = -1,        /* bad pointer, size, enum value or layout */
    STF_EUNSUPPORTED = -2,  /* valid request the library does not implement */
    STF_EHIP = -3           /* the HIP runtime reported an error at launch */
} stf_status;

typedef enum stf_filter_kind {
    STF_BILINEAR = 0,        /* tent filter, 2x2 support (Sec. S6) */
    STF_BICUBIC_BSPLINE = 1  /* uniform cubic B-spline, 4x4 support (Sec. 5.4) */
} stf_filter_kind;

typedef enum stf_format {      /* channels, bytes per texel, decode (times the optional per-channel scale) */
    STF_RGBA8_UNORM = 0,       /* 4, 4,  byte / 255 (linear, no sRGB) */
    STF_RGBA16F = 1,           /* 4, 8,  IEEE half, exact */
    STF_RG16F = 2,             /* 2, 4,  IEEE half, exact */
    STF_R8_UNORM = 3,          /* 1, 1,  byte / 255 */
    STF_RGBA32F = 4,           /* 4, 16, exact */
    STF_R32F = 5,              /* 1, 4,  exact */
    STF_RGBA_BF16 = 6,         /* 4, 8,  bfloat16, exact */
    STF_RGBA_FP8 = 7,          /* 4, 4,  OCP FP8 E4M3 (bias 7, no infinities), exact */
    STF_LATENT8_F16 = 8,       /* 8 latent channels, 16, half; decoded to RGBA by the texture's decoder */
    STF_LATENT8_BF16 = 9,      /* 8 latent channels, 16, bfloat16; decoded likewise */
    STF_LATENT8_FP8 = 10       /* 8 latent channels, 8, FP8 E4M3; decoded likewise */
} stf_format;

typedef enum stf_address {
    STF_WRAP = 0
} stf_address;

/* Sharing footprints S(c) on the tile pixel coordinates (lx, ly) in [0,8)^2
 * of the 8x8 screen tile that one wavefront processes (Sec. 4.3). Every
 * footprint contains the pixel itself. Windows keep their size at tile edges
 * by shifting inward. Pixels outside the screen take part in no footprint. */
typedef enum stf_footprint {
    STF_FP_SELF = 0,        /* {c}: reduces exactly to one-tap STF */
    STF_FP_QUAD2X2 = 1,     /* 2x2 quad with even origin (Sec. 2.3, "2x2q") */
    STF_FP_WAVE2X2 = 2,     /* 2x2 window, origin l - ((l' + (l >> 1)) & 1) per axis ("2x2w") */
    STF_FP_SQUARE3X3 = 3,   /* origin clamp(l - 1, 0, 5) per axis */
    STF_FP_SQUARE4X4 = 4,   /* origin clamp(l - 1, 0, 4) per axis */
    STF_FP_TILE8X8 = 5,     /* all 64 pixels of the tile (the whole wavefront) */
    STF_FP_LUT = 6          /* caller table, see stf_reuse */
} stf_footprint;

typedef struct stf_texture {
    const void* data;       /* device, texel payload */
    int32_t width;          /* texels */
    int32_t height;         /* texels */
    int64_t pitch_bytes;    /* >= width * bytes per texel, multiple of 16 */
    int32_t format;         /* stf_format */
    int32_t reserved;       /* must be 0 */
    const float* scale;     /* host, nullable: per-channel dequantization scale (one per stored
                               channel: 8 for latent formats, applied before the decoder),
                               finite; NULL means 1. Read during the call only. */
    const void* decoder;    /* device, STF_DECODER_BYTES written by stf_decoder_pack: required
                               for latent formats (all latent textures of one call share one
                               decoder), NULL otherwise; 16-byte aligned */
} stf_texture;

typedef struct stf_screen {
    const float* uv;        /* device, FP32 [height][width][2] */
    int32_t width;          /* pixels, 1..STF_MAX_SCREEN */
    int32_t height;         /* pixels, 1..STF_MAX_SCREEN */
} stf_screen;

/* Shared selection (Sec. 4.5: textures with the same UV and resolution can
 * share one selection loop): every slot uses the random numbers, hence the
 * texel positions, of the first slot of the same texture size. Each slot's
 * output is still a reuse estimate of that texture; their errors become
 * correlated. */
#define STF_SHARE_SELECTION 1

/* Testing aid for the whole-tile (STF_FP_TILE8X8) forward and adjoint
 * kernels: the per-texel sums of reciprocal PMFs use FP32 LDS atomics, the
 * path those kernels otherwise take only for a wave that holds a pick of
 * probability below 2^-34 (exact 64-bit integer sums cover all others).
 * Results stay within FP32 rounding of the default path but may depend on
 * the order of the atomic adds. */
#define STF_FLOAT_BIN_SUMS 2

typedef struct stf_params {
    int32_t filter;         /* stf_filter_kind */
    int32_t address;        /* stf_address */
    uint32_t seed;          /* random stream: pcg4d(px, py, frame, seed + (k>>1)*0x9E3779B9), k the slot
                               (or with STF_SHARE_SELECTION the first slot of the same size) */
    uint32_t frame;
    int32_t flags;          /* 0, STF_SHARE_SELECTION | STF_FLOAT_BIN_SUMS */
    int32_t reserved;       /* must be 0 */
} stf_params;

/* Exact filtering (Sec. 4.2): a pixel whose footprint's picks include every
 * texel of positive weight under its own filter returns the Eq. (3) value
 * over those texels instead of the estimate. Biased, lower error; practical
 * for bilinear (4 texels), rare for bicubic (16). */
#define STF_REUSE_EXACT_FILTERING 1
/* Clamp the estimate per channel to the range of the shared texels inside
 * the pixel's own filter support (Sec. 4.1; biased, bounds the error of the
 * comparison estimators; Eq. (14) already lies in that range). */
#define STF_REUSE_CLAMP 2

/* Estimator over the shared picks: the paper's Eq. (14), or one of the
 * estimators Sec. 4.1 compares it with (comparison only: one generic
 * kernel, not the optimised path). With w_i = f_c(x_i) / p_i(x_i) and n
 * shared picks:
 *   STF_EST_IS             (1/n) sum w_i T_i, Eq. (6)
 *   STF_EST_MIS            sum f_c(x_i) T_i / sum_j p_j(x_i) (balance heuristic)
 *   STF_EST_PAIRWISE_MIS   pairwise MIS with the pixel's own technique as the
 *                          canonical one: m_i = p_i / ((n-1) p_i + p_c),
 *                          m_c = 1/(n-1) sum_i p_c / (p_c + (n-1) p_i)
 *   STF_EST_REGRESSION     (1/n) sum [w_i T_i - beta (w_i - 1)], Eq. (7),
 *                          beta = sum (w_i - wbar) w_i T_i / sum (w_i - wbar)^2 */
typedef enum stf_estimator {
    STF_EST_WIS = 0,
    STF_EST_IS = 1,
    STF_EST_MIS = 2,
    STF_EST_PAIRWISE_MIS = 3,
    STF_EST_REGRESSION = 4
} stf_estimator;

typedef struct stf_reuse {
    int32_t footprint;      /* stf_footprint */
    int32_t lut_k;          /* STF_FP_LUT only: entries per pixel, 1..64 */
    const uint8_t* lut;     /* STF_FP_LUT only: device [64][lut_k] row-major tile
                               pixel ids (ly*8+lx, low 6 bits used); an entry
                               equal to the pixel itself is ignored, the pixel
                               is always a member; repeated entries count
                               repeatedly. NULL for other footprints. */
    int32_t flags;          /* STF_REUSE_EXACT_FILTERING (with STF_EST_WIS only) | STF_REUSE_CLAMP */
    int32_t estimator;      /* stf_estimator; 0 = Eq. (14) */
} stf_reuse;

/*
 * One-tap STF (Sec. 2.2; Sec. S1 shows the importance-sampling estimator
 * reduces to returning the picked texel). For each texture slot t each pixel
 * picks one texel of its filter support with probability equal to the filter
 * weight, using two uniforms from the hash of (px, py, frame, seed, t), and
 * writes the decoded texel.
 *   tex    host array of ntex descriptors (1 <= ntex <= STF_MAX_TEXTURES)
 *   out    host array of ntex device pointers, out[t] FP32 [H][W][C_t]
 *   sel    optional device int32 [ntex][H][W][2]: picked texel (x, y),
 *          wrapped into [0, size); NULL to skip
 * Returns STF_OK or a negative stf_status.
 */
int stf_filter(const stf_texture* tex, int32_t ntex, const stf_screen* scr,
               const stf_params* p, float* const* out, int32_t* sel, void* hip_stream);

/*
 * STF with sample reuse (Sec. 4). Each pixel c picks its texel exactly as
 * stf_filter does (same `sel`), then combines the picks of the members i of
 * its footprint with Eq. (14):
 *     out_c = sum_i w_i T_i / sum_i w_i,   w_i = f_c(x_i) / p_i(x_i),
 * where f_c is c's filter weight at texel x_i and p_i the probability with
 * which i picked it; w_i = 0 for texels outside c's support (skipped, never
 * multiplied) and w_c = 1, so with no useful neighbour out_c equals the
 * one-tap STF value (Sec. 4.5). The result always lies within the range of
 * the texels under c's own filter (Eq. (5)).
 *   r      host descriptor of the footprint (and device LUT for STF_FP_LUT)
 * Other arguments as stf_filter.
 */
int stf_filter_reuse(const stf_texture* tex, int32_t ntex, const stf_screen* scr,
                     const stf_params* p, const stf_reuse* r, float* const* out,
                     int32_t* sel, void* hip_stream);

/*
 * Deterministic filtered value, Eq. (3): sum over the filter support of
 * weight * texel, with the same coordinates and 16-bit fractions as the
 * stochastic paths (ground truth for PSNR; the full-filter cost).
 * p->seed and p->frame are ignored.
 */
int stf_filter_reference(const stf_texture* tex, int32_t ntex, const stf_screen* scr,
                         const stf_params* p, float* const* out, void* hip_stream);

/*
 * Adjoint of stf_filter_reuse with respect to the texels. The weights of
 * Eq. (14) depend only on UVs and random numbers, so the output is linear in
 * the texels: out_c = sum_i a_ci T[x_i], a_ci = w_i / sum_j w_j, and
 *     dL/dT[x] += sum_c sum_{i in S(c), x_i = x} a_ci dL/dout_c.
 *   tex    descriptors of the forward textures (data may be NULL: only size
 *          and format are used)
 *   dout   host array of ntex device pointers, FP32 [H][W][C_t], each aligned to
 *          4 * C_t bytes (one pixel's channels are read as one vector)
 *   dtex   host array of ntex device pointers, FP32 [tex height][tex width][C_t],
 *          dense (pitch = width * C_t * 4); ACCUMULATED into (+=), so clear
 *          it first for a plain gradient. Summation order is not fixed
 *          (floating-point atomics): results agree to rounding, not bits.
 *          dL/dout must be finite: the per-window sums multiply exact zeros
 *          by it, so an infinity or NaN can reach other texels of a window.
 * Same p and r as the forward call being differentiated. Latent formats
 * are rejected (STF_EUNSUPPORTED). A per-channel scale multiplies dL/dout,
 * so dtex is the gradient with respect to the texel before its scale.
 */
int stf_backward(const stf_texture* tex, int32_t ntex, const stf_screen* scr,
                 const stf_params* p, const stf_reuse* r, const float* const* dout,
                 float* const* dtex, void* hip_stream);

/*
 * Latent decoder MLP of the neural-texture setting (Sec. 1, Sec. 5.6):
 *     RGBA = W3 ReLU(W2 ReLU(W1 x + b1) + b2) + b3,   x = 8 latent channels.
 * Arrays are device FP32, row-major [out][in]. Latent textures are decoded
 * per picked texel on the matrix cores with FP32 accumulation, in BF16 or
 * FP8 operands (precision below).
 */
/* Decoder arithmetic (stf_mlp.precision):
 *   STF_DECODER_BF16  v_mfma_f32_32x32x16_bf16: w1, b1, w2, w3 rounded to BF16,
 *                     b2, b3 FP32; latents (times their scale) and hidden
 *                     activations rounded to BF16 (RN).
 *   STF_DECODER_FP8   v_mfma_f32_32x32x16_fp8_fp8: each W_l stored as FP8 E4M3
 *                     of W_l / s_l with s_l = max|W_l| / 448, biases FP32;
 *                     latents (times their scale) and hidden activations
 *                     rounded to FP8 E4M3 (RN). Twice the matrix-core rate,
 *                     about 2^-4 relative rounding per value. */
#define STF_DECODER_BF16 0
#define STF_DECODER_FP8 1

typedef struct stf_mlp {
    const float* w1;        /* [64][8] */
    const float* b1;        /* [64] */
    const float* w2;        /* [64][64] */
    const float* b2;        /* [64] */
    const float* w3;        /* [4][64] */
    const float* b3;        /* [4] */
    int32_t precision;      /* STF_DECODER_BF16 or STF_DECODER_FP8 */
    int32_t reserved;       /* must be 0 */
} stf_mlp;

#define STF_DECODER_BYTES 14736

/*
 * Pack `mlp` into the device buffer `packed` (STF_DECODER_BYTES, 16-byte
 * aligned, owned by the caller), enqueued on `hip_stream`. The buffer is then
 * named by stf_texture.decoder of latent textures, in calls on the same
 * stream or after synchronisation. The weights are read on the device and
 * are not validated (non-finite values propagate to the outputs).
 */
int stf_decoder_pack(const stf_mlp* mlp, void* packed, void* hip_stream);

/* Gradients of the decoder's weights and biases (device FP32 arrays of the
 * shapes in stf_mlp, accumulated). */
typedef struct stf_mlp_grad {
    float* w1;              /* [64][8] */
    float* b1;              /* [64] */
    float* w2;              /* [64][64] */
    float* b2;              /* [64] */
    float* w3;              /* [4][64] */
    float* b3;              /* [4] */
} stf_mlp_grad;

/* Device workspace stf_backward_decoder needs for these textures (latent
 * formats, power-of-two sizes), or -1 if they are invalid: per texture a
 * dense FP32 texel gradient (16 bytes per texel) followed by one bit per
 * block of 16 texels, and the list of the blocks a gradient reaches (4 bytes
 * per block); then one weight-gradient slot (about 20 KB) per workgroup of
 * the decoder kernel (at most 512 per texture) and the partial sums of their
 * reduction. */
int64_t stf_backward_decoder_workspace_bytes(const stf_texture* tex, int32_t ntex);

/*
 * Adjoint of stf_filter_reuse over latent textures with respect to the
 * latents and the decoder MLP (the neural-texture setting of Sec. 1 and
 * Sec. 5.6, differentiated through Eq. (14)). The weights of Eq. (14) do not
 * depend on texel values, so with g_x the texel adjoint of stf_backward (the
 * gradient with respect to the decoded RGBA of texel x),
 *     dL/dlatent_x += J_x^T g_x,   dL/dW_l, dL/db_l += sums over the texels,
 * where J_x is the Jacobian of the decoder at latent x (ReLU derivative 1
 * where its input is > 0, else 0).
 *   tex       latent textures (data read: the activations are recomputed),
 *             all with the same packed decoder as in the forward call
 *   p, r      as the forward call being differentiated (plain Eq. (14):
 *             no exact filtering, clamping or comparison estimator)
 *   dout      host array of ntex device pointers, FP32 [H][W][4], 16-byte aligned
 *   mlp       the FP32 weights the decoder was packed from: the adjoint is
 *             that of the FP32 decoder, the forward pass's BF16/FP8 rounding
 *             of weights and activations taken as the identity
 *   dlatent   host array of ntex device pointers, FP32 [tex height][tex width][8]
 *             dense, ACCUMULATED (+=): the gradient with respect to the
 *             stored latent value before its per-channel scale
 *   dmlp      device gradient arrays, ACCUMULATED (+=)
 *   workspace device, >= stf_backward_decoder_workspace_bytes(tex, ntex),
 *             256-byte aligned, owned by the caller, no initialisation needed
 * FP32 arithmetic on the matrix cores; the texel adjoint sums with FP32
 * atomics (order not fixed), everything after it in a fixed order.
 */
int stf_backward_decoder(const stf_texture* tex, int32_t ntex, const stf_screen* scr, const stf_params* p,
                         const stf_reuse* r, const float* const* dout, const stf_mlp* mlp, float* const* dlatent,
                         const stf_mlp_grad* dmlp, void* workspace, int64_t workspace_bytes, void* hip_stream);

/*
 * Pseudorandom sparse sharing footprints (Sec. 4.3, "Pseudorandom Sparse
 * Footprints"; generator of Sec. S5). Writes a footprint LUT for
 * STF_FP_LUT: for each of the 64 tile pixels (row-major ids) k-1 distinct
 * other pixels, drawn around it from a discrete normal distribution of
 * deviation sigma (widened where draws keep failing, near the tile
 * borders), chosen among n_cand candidate sets per pixel so that every pixel
 * is shared about equally often: the best of `trials` random choices, then
 * coordinate descent, the best of `restarts` runs. The score is the sum of
 * squared usage counts (ideal 64 (k-1)^2), which orders configurations as
 * the standard deviation of the counts does. Deterministic in all
 * parameters; random numbers come from pcg4d(q + 64 j, attempt, restart,
 * seed ^ 0x5EED0001) for the draws and pcg4d(q, trial, restart,
 * seed ^ 0x5EED0002) for the trials.
 */
typedef struct stf_footprint_params {
    int32_t k;              /* footprint size including the pixel itself, 2..64 */
    int32_t n_cand;         /* candidate sets per pixel, 1..64 (the paper: 16-32) */
    float sigma;            /* deviation of the draws in tile pixels, > 0 (the paper: 1.4) */
    int32_t trials;         /* random choices per restart, 1..2^24 (the paper: 10 000) */
    int32_t restarts;       /* 1..4096 (the paper: 30) */
    uint32_t seed;
    int32_t reserved;       /* must be 0 */
} stf_footprint_params;

/* Device workspace stf_footprint_generate needs for `p`, or -1 if p is
 * invalid (see stf_last_error). */
int64_t stf_footprint_workspace_bytes(const stf_footprint_params* p);

/*
 *   workspace  device, >= stf_footprint_workspace_bytes(p) bytes, 256-byte
 *              aligned, owned by the caller; contents need no initialisation
 *   lut        device uint8 [64][k-1], written
 *   score      device int64, nullable: the LUT's score
 * Enqueued on `hip_stream`; nothing is allocated.
 */
int stf_footprint_generate(const stf_footprint_params* p, void* workspace, int64_t workspace_bytes, uint8_t* lut,
                           int64_t* score, void* hip_stream);

/*
 * stf_footprint_generate without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The workspace is a static device array
 * of STF_FOOTPRINT_STATIC_BYTES per GPU, part of the library's image and held
 * until the process ends; the call itself allocates nothing. Parameters
 * whose workspace (stf_footprint_workspace_bytes) exceeds that size are
 * rejected with STF_EINVAL (the paper's settings, k = 9, 32 candidates,
 * 30 restarts, need about 0.5 MB). Same results as stf_footprint_generate.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (different streams, or several host threads) race and must be
 * serialised by the caller; calls on different GPUs do not interact. The
 * first call on a device resolves the array's address with that device
 * current (STF_EHIP if that fails).
 */
#define STF_FOOTPRINT_STATIC_BYTES (4 << 20)
int stf_footprint_generate_static(const stf_footprint_params* p, uint8_t* lut, int64_t* score, void* hip_stream);

/* Message for the last non-OK status returned on this thread ("" if none).
 * The pointer stays valid until the next call on this thread. */
const char* stf_last_error(void);

/* STF_VERSION of the built library. */
int stf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STF_H */
