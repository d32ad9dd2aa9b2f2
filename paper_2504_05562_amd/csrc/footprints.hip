// Pseudorandom sparse sharing footprints (Sec. 4.3, "Pseudorandom Sparse
// Footprints"; generator of Sec. S5) on the GPU.
//
// For each of the 64 pixels of the 8x8 wave tile the generator picks K-1
// other tile pixels to share with, balancing locality (draws around the
// pixel from a discrete normal distribution) against even use of every
// pixel (the score). Three stages per restart, restarts in parallel:
//   stage 1  n_cand candidate sets per pixel, one thread per set;
//   stage 2  `trials` random choices of one set per pixel, one wavefront per
//            trial: usage counts in LDS, score = sum of squared counts
//            (orders configurations exactly as the standard deviation of
//            the counts does, the total being fixed), packed with the trial
//            index into one 64-bit atomic minimum per restart;
//   stage 3  coordinate descent, one wavefront per restart: for each pixel
//            in turn every lane scores one candidate set, the wave takes the
//            best, until a sweep over all pixels changes nothing;
//   then the restart with the lowest score gives the LUT.
// Random numbers: pcg4d keyed as
//   stage 1: pcg4d(q + 64 j, attempt, restart, seed ^ 0x5EED0001) -> (x, y, z, -):
//            offset (x mod 15 - 7, y mod 15 - 7), accepted iff z < T_L[dx^2 + dy^2]
//   stage 2: pcg4d(q, trial, restart, seed ^ 0x5EED0002).x mod n_cand
// with T_L[r2] = floor(2^32 exp(-r2 / (2 (sigma 1.25^L)^2))), L = min(attempt / 64, 7),
// T_7 = 2^32 (any valid draw). A draw outside the tile, equal to the pixel
// or already in the set is rejected; after 64 * 8 + 4096 attempts the set is
// completed with the lowest-numbered unused pixels (this only bounds the loop).
// Ties go to the lowest trial, candidate and restart index.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "stf.h"
#include "stf_device.h"
#include "stf_status.h"

namespace stf {
namespace fp {

constexpr uint32_t kKey1 = 0x5EED0001u;
constexpr uint32_t kKey2 = 0x5EED0002u;
constexpr int kPerLevel = 64;
constexpr int kLevels = 8;
constexpr int kAttemptCap = kPerLevel * kLevels + 4096;
constexpr int kR2 = 2 * 7 * 7 + 1;

struct Params {
    int k, n_cand, trials, restarts;
    float sigma;
    uint32_t seed;
    uint8_t* cand;        // [restarts][64][n_cand][k-1]
    uint64_t* best2;      // [restarts] (score << 32) | trial
    uint64_t* final_;     // [restarts] (score << 32) | restart
    uint8_t* choice;      // [restarts][64]
};

__device__ __forceinline__ uint8_t* set_of(const Params& p, int r, int q, int j) {
    return p.cand + (((size_t)r * 64 + q) * p.n_cand + j) * (p.k - 1);
}

__global__ __launch_bounds__(256) void init_kernel(Params p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.restarts) {
        p.best2[i] = ~0ull;
        p.final_[i] = ~0ull;
    }
}

// Stage 1: one thread per candidate set (q, j) of restart blockIdx.y.
__global__ __launch_bounds__(256) void stage1_kernel(Params p) {
    __shared__ uint64_t T[kLevels][kR2];
    for (int i = threadIdx.x; i < kLevels * kR2; i += blockDim.x) {
        const int L = i / kR2, r2 = i % kR2;
        if (L == kLevels - 1) {
            T[L][r2] = 1ull << 32;
        } else {
            double s = (double)p.sigma;
            for (int l = 0; l < L; ++l) s *= 1.25;
            T[L][r2] = (uint64_t)floor(4294967296.0 * exp(-(double)r2 / (2.0 * s * s)));
        }
    }
    __syncthreads();
    const int sid = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (sid >= 64 * p.n_cand) return;
    const int q = sid % 64, j = sid / 64;
    const int qx = q % 8, qy = q / 8;
    const int m = p.k - 1;
    uint8_t* out = set_of(p, r, q, j);
    uint64_t used = 1ull << q;
    int filled = 0;
    for (int a = 0; a < kAttemptCap && filled < m; ++a) {
        const uint4 h = pcg4d(make_uint4((uint32_t)(q + 64 * j), (uint32_t)a, (uint32_t)r, p.seed ^ kKey1));
        const int dx = (int)(h.x % 15u) - 7, dy = (int)(h.y % 15u) - 7;
        const int L = min(a / kPerLevel, kLevels - 1);
        const int tx = qx + dx, ty = qy + dy;
        if ((uint64_t)h.z >= T[L][dx * dx + dy * dy]) continue;
        if (tx < 0 || tx >= 8 || ty < 0 || ty >= 8) continue;
        const int t = ty * 8 + tx;
        if (used & (1ull << t)) continue;
        used |= 1ull << t;
        out[filled++] = (uint8_t)t;
    }
    for (int t = 0; t < 64 && filled < m; ++t) {
        if (!(used & (1ull << t))) {
            used |= 1ull << t;
            out[filled++] = (uint8_t)t;
        }
    }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    return v;
}

__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t w = ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o, 64) << 32) |
                           (uint32_t)__shfl_xor((int)(uint32_t)v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

// Stage 2: wave w of block b scores trials b * 4 + w, + 4 * gridDim.x, ...
// of restart blockIdx.y.
__global__ __launch_bounds__(256) void stage2_kernel(Params p) {
    __shared__ uint32_t counts[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = blockIdx.y;
    const int m = p.k - 1;
    uint64_t best = ~0ull;
    for (int t = blockIdx.x * 4 + wave; t < p.trials; t += 4 * gridDim.x) {
        counts[wave][lane] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t j = pcg4d(make_uint4((uint32_t)lane, (uint32_t)t, (uint32_t)r, p.seed ^ kKey2)).x %
                           (uint32_t)p.n_cand;
        const uint8_t* set = set_of(p, r, lane, (int)j);
        for (int e = 0; e < m; ++e) atomicAdd(&counts[wave][set[e]], 1u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t c = counts[wave][lane];
        const uint32_t score = wave_sum(c * c);
        const uint64_t key = ((uint64_t)score << 32) | (uint32_t)t;
        best = key < best ? key : best;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (lane == 0 && best != ~0ull) atomicMin(reinterpret_cast<unsigned long long*>(&p.best2[r]), best);
}

// Stage 3: one wavefront per restart.
__global__ __launch_bounds__(64) void stage3_kernel(Params p) {
    __shared__ uint32_t counts[64];
    __shared__ uint8_t choice[64];
    const int lane = threadIdx.x, r = blockIdx.x;
    const int m = p.k - 1;
    const uint32_t t = (uint32_t)(p.best2[r] & 0xFFFFFFFFull);
    choice[lane] = (uint8_t)(pcg4d(make_uint4((uint32_t)lane, t, (uint32_t)r, p.seed ^ kKey2)).x % (uint32_t)p.n_cand);
    counts[lane] = 0u;
    __syncthreads();
    {
        const uint8_t* set = set_of(p, r, lane, choice[lane]);
        for (int e = 0; e < m; ++e) atomicAdd(&counts[set[e]], 1u);
    }
    __syncthreads();
    uint32_t score = wave_sum(counts[lane] * counts[lane]);
    bool changed = true;
    // every accepted change lowers the integer score, so sweeps end; the cap
    // only guards the loop
    for (int sweep = 0; changed && sweep < 100000; ++sweep) {
        changed = false;
        for (int q = 0; q < 64; ++q) {
            const uint8_t* cur = set_of(p, r, q, choice[q]);
            // removing the current set: sum of (2c - 1) over its members
            uint32_t remove = 0;
            for (int e = 0; e < m; ++e) remove += 2u * counts[cur[e]] - 1u;
            uint64_t key = ~0ull;
            if (lane < p.n_cand) {
                const uint8_t* alt = set_of(p, r, q, lane);
                uint32_t add = 0;
                for (int e = 0; e < m; ++e) {
                    const uint8_t x = alt[e];
                    uint32_t in_cur = 0;
                    for (int f = 0; f < m; ++f) in_cur |= (cur[f] == x) ? 1u : 0u;
                    add += 2u * (counts[x] - in_cur) + 1u;
                }
                key = ((uint64_t)(score - remove + add) << 32) | (uint32_t)lane;
            }
            key = wave_min64(key);
            const uint32_t best_score = (uint32_t)(key >> 32);
            const int best_j = (int)(key & 0xFFFFFFFFu);
            if (best_score < score) {
                __syncthreads();
                if (lane < m) {
                    atomicSub(&counts[cur[lane]], 1u);
                }
                __syncthreads();
                if (lane < m) atomicAdd(&counts[set_of(p, r, q, best_j)[lane]], 1u);
                if (lane == 0) choice[q] = (uint8_t)best_j;
                __syncthreads();
                score = best_score;
                changed = true;
            }
        }
    }
    p.choice[(size_t)r * 64 + lane] = choice[lane];
    if (lane == 0) p.final_[r] = ((uint64_t)score << 32) | (uint32_t)r;
}

// Best restart -> LUT [64][k-1] and its score.
__global__ __launch_bounds__(64) void finish_kernel(Params p, uint8_t* lut, int64_t* score_out) {
    const int lane = threadIdx.x;
    uint64_t best = ~0ull;
    for (int r = lane; r < p.restarts; r += 64) best = p.final_[r] < best ? p.final_[r] : best;
    best = wave_min64(best);
    const int r = (int)(best & 0xFFFFFFFFu);
    const int m = p.k - 1;
    const uint8_t* set = set_of(p, r, lane, p.choice[(size_t)r * 64 + lane]);
    for (int e = 0; e < m; ++e) lut[lane * m + e] = set[e];
    if (lane == 0 && score_out != nullptr) *score_out = (int64_t)(best >> 32);
}

struct Layout {
    size_t cand, best2, final_, choice, total;
};

Layout layout_of(const stf_footprint_params& p) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    Layout l;
    l.cand = 0;
    l.best2 = up((size_t)p.restarts * 64 * p.n_cand * (p.k - 1));
    l.final_ = l.best2 + up((size_t)p.restarts * 8);
    l.choice = l.final_ + up((size_t)p.restarts * 8);
    l.total = l.choice + up((size_t)p.restarts * 64);
    return l;
}

int validate(const stf_footprint_params* p) {
    if (p == nullptr) return stf_host::fail(STF_EINVAL, "footprint parameters are null");
    if (p->k < 2 || p->k > 64) return stf_host::fail(STF_EINVAL, "k=%d outside 2..64", p->k);
    if (p->n_cand < 1 || p->n_cand > 64) return stf_host::fail(STF_EINVAL, "n_cand=%d outside 1..64", p->n_cand);
    if (p->trials < 1 || p->trials > (1 << 24)) return stf_host::fail(STF_EINVAL, "trials=%d outside 1..2^24", p->trials);
    if (p->restarts < 1 || p->restarts > 4096)
        return stf_host::fail(STF_EINVAL, "restarts=%d outside 1..4096", p->restarts);
    if (!(p->sigma > 0.0f) || !std::isfinite(p->sigma)) return stf_host::fail(STF_EINVAL, "sigma must be finite and > 0");
    if (p->reserved != 0) return stf_host::fail(STF_EINVAL, "reserved field must be 0");
    return STF_OK;
}

// Workspace of stf_footprint_generate_static: a file-scope device array, one
// copy per GPU, held until the process ends. Host code never passes its name
// to a kernel (on the host it is only a stand-in for the symbol): the device
// address of each GPU's copy comes from hipGetSymbolAddress, resolved once per
// device with that device current.
__device__ __align__(256) uint8_t scratch[STF_FOOTPRINT_STATIC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, or nullptr with the
// error recorded.
void* static_scratch() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        stf_host::fail(STF_EHIP, "hipGetDevice failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        stf_host::fail(STF_EUNSUPPORTED, "device %d beyond the %d devices the static workspace supports", dev,
                       kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            stf_host::fail(STF_EHIP, "hipGetSymbolAddress of the static workspace failed: %s", hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace fp
}  // namespace stf

extern "C" {

int64_t stf_footprint_workspace_bytes(const stf_footprint_params* p) {
    stf_host::clear_error();
    if (stf::fp::validate(p) != STF_OK) return -1;
    return (int64_t)stf::fp::layout_of(*p).total;
}

int stf_footprint_generate(const stf_footprint_params* prm, void* workspace, int64_t workspace_bytes, uint8_t* lut,
                           int64_t* score, void* hip_stream) {
    using namespace stf::fp;
    stf_host::clear_error();
    int rc = validate(prm);
    if (rc != STF_OK) return rc;
    const Layout l = layout_of(*prm);
    if (workspace == nullptr || lut == nullptr) return stf_host::fail(STF_EINVAL, "workspace or lut is null");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return stf_host::fail(STF_EINVAL, "workspace not aligned to 256 bytes");
    if (workspace_bytes < (int64_t)l.total)
        return stf_host::fail(STF_EINVAL, "workspace of %lld bytes, %lld needed", (long long)workspace_bytes,
                              (long long)l.total);
    if (score != nullptr && (reinterpret_cast<uintptr_t>(score) & 7) != 0)
        return stf_host::fail(STF_EINVAL, "score not 8-byte aligned");
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    Params p;
    p.k = prm->k;
    p.n_cand = prm->n_cand;
    p.trials = prm->trials;
    p.restarts = prm->restarts;
    p.sigma = prm->sigma;
    p.seed = prm->seed;
    p.cand = ws + l.cand;
    p.best2 = reinterpret_cast<uint64_t*>(ws + l.best2);
    p.final_ = reinterpret_cast<uint64_t*>(ws + l.final_);
    p.choice = ws + l.choice;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(init_kernel, dim3((p.restarts + 255) / 256), dim3(256), 0, s, p);
    hipLaunchKernelGGL(stage1_kernel, dim3((64 * p.n_cand + 255) / 256, p.restarts), dim3(256), 0, s, p);
    const int blocks2 = std::min((p.trials + 3) / 4, 256);
    hipLaunchKernelGGL(stage2_kernel, dim3(blocks2, p.restarts), dim3(256), 0, s, p);
    hipLaunchKernelGGL(stage3_kernel, dim3(p.restarts), dim3(64), 0, s, p);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, p, lut, score);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return stf_host::fail(STF_EHIP, "footprint generator launch failed: %s", hipGetErrorString(e));
    return STF_OK;
}

int stf_footprint_generate_static(const stf_footprint_params* prm, uint8_t* lut, int64_t* score, void* hip_stream) {
    stf_host::clear_error();
    const int rc = stf::fp::validate(prm);
    if (rc != STF_OK) return rc;
    const int64_t need = (int64_t)stf::fp::layout_of(*prm).total;
    if (need > (int64_t)STF_FOOTPRINT_STATIC_BYTES)
        return stf_host::fail(STF_EINVAL,
                              "parameters need a %lld-byte workspace, above the static limit of %lld bytes "
                              "(restarts * 64 * n_cand * (k-1) must stay below it); use stf_footprint_generate",
                              (long long)need, (long long)STF_FOOTPRINT_STATIC_BYTES);
    void* ws = stf::fp::static_scratch();
    if (ws == nullptr) return STF_EHIP;
    // the kernels initialise every word of the workspace they read
    return stf_footprint_generate(prm, ws, (int64_t)STF_FOOTPRINT_STATIC_BYTES, lut, score, hip_stream);
}

}  // extern "C"
