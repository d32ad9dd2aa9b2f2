// Host-only check of the C ABI's argument validation, built by
// tests/test_abi_host.py without device code at -O0 with AddressSanitizer and
// UndefinedBehaviorSanitizer. Every call here is rejected on the host before
// any launch, so no GPU is touched. Exit status 0 when every check holds.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "stf.h"

static int failures = 0;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

static const void* fake(uintptr_t a) { return reinterpret_cast<const void*>(a); }

static void good(stf_texture& t, stf_screen& s, stf_params& p) {
    std::memset(&t, 0, sizeof t);
    t.data = fake(256);
    t.width = 64;
    t.height = 64;
    t.pitch_bytes = 64 * 4;
    t.format = STF_RGBA8_UNORM;
    s.uv = static_cast<const float*>(fake(4096));
    s.width = 16;
    s.height = 16;
    std::memset(&p, 0, sizeof p);
    p.filter = STF_BICUBIC_BSPLINE;
}

static bool has(const char* needle) { return std::strstr(stf_last_error(), needle) != nullptr; }

int main() {
    stf_texture t;
    stf_screen s;
    stf_params p;
    float* out[4] = {(float*)fake(4096), (float*)fake(8192), (float*)fake(12288), (float*)fake(16384)};

    // a failing call records a message; the next successful call clears it
    good(t, s, p);
    s.uv = nullptr;
    CHECK(stf_filter(&t, 1, &s, &p, out, nullptr, nullptr) == STF_EINVAL);
    CHECK(has("uv"));
    stf_footprint_params fp = {9, 32, 1.4f, 10000, 30, 0u, 0};
    CHECK(stf_footprint_workspace_bytes(&fp) > 0);
    CHECK(stf_last_error()[0] == '\0');

    // every other entry point clears it too
    CHECK(stf_filter(nullptr, 1, &s, &p, out, nullptr, nullptr) == STF_EINVAL);
    CHECK(has("null"));
    good(t, s, p);
    t.width = 48;
    CHECK(stf_filter_reference(&t, 1, &s, &p, out, nullptr) == STF_EINVAL);
    CHECK(has("powers of two"));
    stf_footprint_params bad = fp;
    bad.k = 1;
    CHECK(stf_footprint_workspace_bytes(&bad) == -1);
    CHECK(stf_version() == STF_VERSION);
    CHECK(stf_footprint_workspace_bytes(&fp) > 0);
    CHECK(stf_last_error()[0] == '\0');

    // the descriptor checks of test_abi.py
    struct Case { void (*mutate)(stf_texture&, stf_screen&, stf_params&); int code; const char* needle; };
    static const float nan_scale[4] = {1.0f, NAN, 1.0f, 1.0f};
    const Case cases[] = {
        {[](stf_texture&, stf_screen& s, stf_params&) { s.uv = nullptr; }, STF_EINVAL, "uv"},
        {[](stf_texture&, stf_screen& s, stf_params&) { s.width = 0; }, STF_EINVAL, "screen"},
        {[](stf_texture&, stf_screen& s, stf_params&) { s.height = STF_MAX_SCREEN + 1; }, STF_EINVAL, "screen"},
        {[](stf_texture&, stf_screen& s, stf_params&) { s.uv = (const float*)fake(4100); }, STF_EINVAL, "aligned"},
        {[](stf_texture&, stf_screen&, stf_params& p) { p.filter = 7; }, STF_EINVAL, "filter"},
        {[](stf_texture&, stf_screen&, stf_params& p) { p.address = 1; }, STF_EUNSUPPORTED, "address"},
        {[](stf_texture&, stf_screen&, stf_params& p) { p.flags = 4; }, STF_EINVAL, "flags"},
        {[](stf_texture&, stf_screen&, stf_params& p) { p.reserved = 3; }, STF_EINVAL, "reserved"},
        {[](stf_texture& t, stf_screen&, stf_params&) { t.format = 99; }, STF_EINVAL, "format"},
        {[](stf_texture& t, stf_screen&, stf_params&) { t.height = 2; }, STF_EINVAL, "powers of two"},
        {[](stf_texture& t, stf_screen&, stf_params&) { t.pitch_bytes = 100; }, STF_EINVAL, "pitch"},
        {[](stf_texture& t, stf_screen&, stf_params&) { t.data = nullptr; }, STF_EINVAL, "data"},
        {[](stf_texture& t, stf_screen&, stf_params&) { t.data = fake(264); }, STF_EINVAL, "aligned"},
        {[](stf_texture& t, stf_screen&, stf_params&) { t.reserved = 1; }, STF_EINVAL, "reserved"},
        {[](stf_texture& t, stf_screen&, stf_params&) { t.format = STF_LATENT8_FP8; }, STF_EINVAL, "decoder"},
        {[](stf_texture& t, stf_screen&, stf_params&) { t.decoder = fake(4096); }, STF_EINVAL, "not latent"},
        {[](stf_texture& t, stf_screen&, stf_params&) { t.scale = nan_scale; }, STF_EINVAL, "scale"},
    };
    for (const Case& c : cases) {
        good(t, s, p);
        c.mutate(t, s, p);
        CHECK(stf_filter(&t, 1, &s, &p, out, nullptr, nullptr) == c.code);
        CHECK(has(c.needle));
        stf_reuse r = {STF_FP_TILE8X8, 0, nullptr, 0, 0};
        CHECK(stf_filter_reuse(&t, 1, &s, &p, &r, out, nullptr, nullptr) == c.code);
        CHECK(has(c.needle));
    }

    // counts, outputs and reuse descriptors
    good(t, s, p);
    CHECK(stf_filter(&t, 0, &s, &p, out, nullptr, nullptr) == STF_EINVAL);
    CHECK(stf_filter(&t, STF_MAX_TEXTURES + 1, &s, &p, out, nullptr, nullptr) == STF_EINVAL);
    CHECK(stf_filter(&t, 1, &s, &p, nullptr, nullptr, nullptr) == STF_EINVAL);
    float* null_out[1] = {nullptr};
    CHECK(stf_filter(&t, 1, &s, &p, null_out, nullptr, nullptr) == STF_EINVAL);
    float* odd_out[1] = {(float*)fake(4100)};
    CHECK(stf_filter(&t, 1, &s, &p, odd_out, nullptr, nullptr) == STF_EINVAL);
    CHECK(stf_filter(&t, 1, &s, &p, out, (int32_t*)fake(4100), nullptr) == STF_EINVAL);
    CHECK(stf_filter_reuse(&t, 1, &s, &p, nullptr, out, nullptr, nullptr) == STF_EINVAL);
    stf_reuse r = {42, 0, nullptr, 0, 0};
    CHECK(stf_filter_reuse(&t, 1, &s, &p, &r, out, nullptr, nullptr) == STF_EINVAL);
    r = {STF_FP_LUT, 4, nullptr, 0, 0};
    CHECK(stf_filter_reuse(&t, 1, &s, &p, &r, out, nullptr, nullptr) == STF_EINVAL);
    CHECK(has("lut"));
    r = {STF_FP_LUT, 65, (const uint8_t*)fake(4096), 0, 0};
    CHECK(stf_filter_reuse(&t, 1, &s, &p, &r, out, nullptr, nullptr) == STF_EINVAL);
    r = {STF_FP_TILE8X8, 0, nullptr, 4, 0};
    CHECK(stf_filter_reuse(&t, 1, &s, &p, &r, out, nullptr, nullptr) == STF_EINVAL);
    r = {STF_FP_TILE8X8, 0, nullptr, 0, 7};
    CHECK(stf_filter_reuse(&t, 1, &s, &p, &r, out, nullptr, nullptr) == STF_EINVAL);
    r = {STF_FP_TILE8X8, 0, nullptr, STF_REUSE_EXACT_FILTERING, STF_EST_IS};
    CHECK(stf_filter_reuse(&t, 1, &s, &p, &r, out, nullptr, nullptr) == STF_EUNSUPPORTED);

    // the adjoint
    const float* dout[1] = {(const float*)fake(4096)};
    float* dtex[1] = {(float*)fake(8192)};
    r = {STF_FP_TILE8X8, 0, nullptr, STF_REUSE_CLAMP, 0};
    CHECK(stf_backward(&t, 1, &s, &p, &r, dout, dtex, nullptr) == STF_EUNSUPPORTED);
    r = {STF_FP_TILE8X8, 0, nullptr, 0, 0};
    CHECK(stf_backward(&t, 1, &s, &p, &r, nullptr, dtex, nullptr) == STF_EINVAL);
    const float* null_dout[1] = {nullptr};
    CHECK(stf_backward(&t, 1, &s, &p, &r, null_dout, dtex, nullptr) == STF_EINVAL);
    CHECK(stf_backward(&t, 1, &s, &p, nullptr, dout, dtex, nullptr) == STF_EINVAL);

    // the decoder packer
    stf_mlp m = {(const float*)fake(4096), (const float*)fake(4096), (const float*)fake(4096), nullptr,
                 (const float*)fake(4096), (const float*)fake(4096), STF_DECODER_BF16, 0};
    CHECK(stf_decoder_pack(&m, (void*)fake(4096), nullptr) == STF_EINVAL);
    m.b2 = (const float*)fake(4096);
    m.precision = 2;
    CHECK(stf_decoder_pack(&m, (void*)fake(4096), nullptr) == STF_EINVAL);
    m.precision = STF_DECODER_BF16;
    CHECK(stf_decoder_pack(&m, (void*)fake(4104), nullptr) == STF_EINVAL);
    CHECK(stf_decoder_pack(nullptr, (void*)fake(4096), nullptr) == STF_EINVAL);

    // the footprint generator
    const int64_t n = stf_footprint_workspace_bytes(&fp);
    CHECK(n >= 30 * 64 * 32 * 8 && n % 256 == 0);
    CHECK(stf_footprint_generate(&fp, nullptr, n, (uint8_t*)fake(4096), nullptr, nullptr) == STF_EINVAL);
    CHECK(stf_footprint_generate(&fp, (void*)fake(4096), n - 1, (uint8_t*)fake(4096), nullptr, nullptr) == STF_EINVAL);
    CHECK(has("workspace"));
    CHECK(stf_footprint_generate(&fp, (void*)fake(4096 + 64), n, (uint8_t*)fake(4096), nullptr, nullptr) ==
          STF_EINVAL);
    CHECK(stf_footprint_generate(nullptr, (void*)fake(4096), n, (uint8_t*)fake(4096), nullptr, nullptr) ==
          STF_EINVAL);

    // and the message is gone after a successful call
    CHECK(stf_footprint_workspace_bytes(&fp) == n);
    CHECK(stf_last_error()[0] == '\0');

    if (failures == 0) std::printf("abi host checks passed\n");
    return failures == 0 ? 0 : 1;
}
