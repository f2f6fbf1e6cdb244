// The stochastic hard concrete gate's noise and per-frame densification (clone, split, prune).
//
// Random numbers come from Philox4x32-10 (Salmon et al., SC 2011), a counter-based generator: every draw is a
// pure function of (counter, key), so a draw does not depend on launch shape or order, and a graph replay that
// advances the step counter on the device draws afresh.  Uniforms are the top 23 bits of a word plus one half,
// scaled by 2^-23 (exact in float32, never 0 or 1).
//
// Densification keeps each Gaussian's children in place, in parent order: the plan gives every Gaussian an
// action and the exclusive scan of its child counts (0 pruned, 1 kept, 2 cloned or split), and every
// per-Gaussian array is then expanded through that map; clone and split children get their changes last.
#include <cmath>

#include "qg_internal.h"

namespace qg {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kGateTag = 0x67617465u;   // "gate"
constexpr uint32_t kSplitTag = 0x73706C74u;  // "splt"

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint32_t hi0 = __umulhi(kPhiloxM0, c.x), lo0 = kPhiloxM0 * c.x;
        const uint32_t hi1 = __umulhi(kPhiloxM1, c.z), lo1 = kPhiloxM1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__device__ __forceinline__ float unit_open(uint32_t x) { return ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f); }

// Logistic sample log u - log(1 - u) of the gate of Gaussian i at optimiser step `step`.
__global__ void k_gate_noise(int64_t n, uint32_t k0, uint32_t k1, int32_t step, const int32_t* __restrict__ step_dev,
                             float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t s = step_dev ? (uint32_t)step_dev[0] : (uint32_t)step;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)i, s, kGateTag, 0u), k0, k1);
    const float u = unit_open(w.x);
    out[i] = logf(u) - logf(1.f - u);
}

// One iteration's densification statistic: |(sx dL/dx', sy dL/dy')| of a visible Gaussian, and its visit count.
__global__ void k_densify_accumulate(int64_t n, const float* __restrict__ gxy, const int32_t* __restrict__ ntiles,
                                     float sx, float sy, float* __restrict__ accum, float* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || ntiles[i] <= 0) return;
    accum[i] += hypotf(sx * gxy[i], sy * gxy[n + i]);
    count[i] += 1.f;
}

constexpr int kPlanBlock = 256, kPlanIPT = 4, kPlanTile = kPlanBlock * kPlanIPT;

__device__ __forceinline__ uint8_t plan_action(int64_t i, const float* __restrict__ accum,
                                               const float* __restrict__ count, const float* __restrict__ attrs,
                                               int64_t ld, double threshold, double max_scale, double min_opacity) {
    const double logit = (double)attrs[10 * ld + i];
    if (1.0 / (1.0 + exp(-logit)) < min_opacity) return 3;  // prune
    const double c = (double)count[i];
    const double score = c > 0.0 ? (double)accum[i] / c : 0.0;
    if (!(score >= threshold)) return 0;  // keep
    const double ls = fmax(fmax((double)attrs[7 * ld + i], (double)attrs[8 * ld + i]), (double)attrs[9 * ld + i]);
    return exp(ls) > max_scale ? 2 : 1;  // split or clone
}

__device__ __forceinline__ int64_t n_children(uint8_t a) { return a == 3 ? 0 : (a == 0 ? 1 : 2); }

template <typename T>
__device__ __forceinline__ T block_sum(T x, T* s_w) {
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    if (__lane_id() == 0) s_w[threadIdx.x / 64] = x;
    __syncthreads();
    T t = 0;
    for (int k = 0; k < (int)blockDim.x / 64; ++k) t += s_w[k];
    __syncthreads();
    return t;
}

// Pass 1: actions and each tile's child count.
__global__ __launch_bounds__(kPlanBlock) void k_plan(int64_t n, const float* __restrict__ accum,
                                                     const float* __restrict__ count, const float* __restrict__ attrs,
                                                     int64_t ld, double threshold, double max_scale,
                                                     double min_opacity, uint8_t* __restrict__ action,
                                                     int64_t* __restrict__ tile_sum) {
    __shared__ int64_t s_w[kPlanBlock / 64];
    int64_t c = 0;
#pragma unroll
    for (int r = 0; r < kPlanIPT; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kPlanTile + r * kPlanBlock + threadIdx.x;
        if (i < n) {
            const uint8_t a = plan_action(i, accum, count, attrs, ld, threshold, max_scale, min_opacity);
            action[i] = a;
            c += n_children(a);
        }
    }
    const int64_t t = block_sum<int64_t>(c, s_w);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = t;
}

// Pass 2: exclusive scan of the tile sums in place (one block of 1024 threads, sequential chunks).
__global__ __launch_bounds__(1024) void k_plan_scan(int64_t ntiles, int64_t* __restrict__ tile_sum,
                                                    int64_t* __restrict__ total) {
    __shared__ int64_t s[1024];
    int64_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < ntiles ? tile_sum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t add = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < ntiles) tile_sum[i] = carry + s[threadIdx.x] - v;
        carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Pass 3: per-Gaussian exclusive offsets from the scanned tile sums (block-local scan in the same item order).
__global__ __launch_bounds__(kPlanBlock) void k_plan_offsets(int64_t n, const uint8_t* __restrict__ action,
                                                             const int64_t* __restrict__ tile_off,
                                                             int64_t* __restrict__ offsets) {
    __shared__ int64_t s_w[kPlanBlock / 64];
    __shared__ int64_t s_run;
    if (threadIdx.x == 0) s_run = tile_off[blockIdx.x];
    __syncthreads();
    for (int r = 0; r < kPlanIPT; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kPlanTile + r * kPlanBlock + threadIdx.x;
        const int64_t c = i < n ? n_children(action[i]) : 0;
        // inclusive wave scan, then the waves in order
        int64_t x = c;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (__lane_id() >= o) x += y;
        }
        if (__lane_id() == 63) s_w[threadIdx.x / 64] = x;
        __syncthreads();
        int64_t wbase = 0, tot = 0;
        for (int k = 0; k < kPlanBlock / 64; ++k) {
            if (k < (int)threadIdx.x / 64) wbase += s_w[k];
            tot += s_w[k];
        }
        const int64_t run = s_run;
        if (i < n) offsets[i] = run + wbase + x - c;
        __syncthreads();
        if (threadIdx.x == 0) s_run = run + tot;
        __syncthreads();
    }
}

// Copies each plane of every parent to its children; mode 1 (optimiser moments) keeps the value only on the
// first child of a kept or cloned Gaussian and starts every new Gaussian at zero.
__global__ void k_expand(int64_t n, const uint8_t* __restrict__ action, const int64_t* __restrict__ offsets,
                         int32_t nplanes, const float* __restrict__ src, int64_t ld_src, float* __restrict__ dst,
                         int64_t ld_dst, int32_t mode) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint8_t a = action[i];
    const int64_t k = n_children(a), o = offsets[i];
    if (k == 0) return;
    const bool keep_first = a == 0 || a == 1;
    for (int p = 0; p < nplanes; ++p) {
        const float v = src[(int64_t)p * ld_src + i];
        for (int64_t c = 0; c < k; ++c)
            dst[(int64_t)p * ld_dst + o + c] = (mode == 1 && !(c == 0 && keep_first)) ? 0.f : v;
    }
}

// Children after the expansion.  Clone (action 1): both copies' stored opacity logit moves by
// logit(o') - logit(o), o' = 1 - sqrt(1 - o), o the parent's decoded opacity, so that the coincident pair
// composites like the parent where its Gaussian factor is 1 (double precision).  Split (action 2): mean +
// R(q) (s * z) with the parent's decoded rotation and scale, log-scale - ln 1.6.
__global__ void k_children(int64_t n, const uint8_t* __restrict__ action, const int64_t* __restrict__ offsets,
                           const float* __restrict__ dec, int64_t ld, uint32_t k0, uint32_t k1, uint32_t rnd,
                           float* __restrict__ dst, int64_t ld_dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint8_t act = action[i];
    if (act == 1) {
        const double x = (double)dec[10 * ld + i];
        const double sq = sqrt(1.0 / (1.0 + exp(x)));  // sqrt(1 - o)
        const float shift = (float)((log1p(-sq) - log(sq)) - x);
        for (int c = 0; c < 2; ++c) dst[10 * ld_dst + offsets[i] + c] += shift;
        return;
    }
    if (act != 2) return;
    float z[8];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)i, rnd, kSplitTag, (uint32_t)b), k0, k1);
        const float u0 = unit_open(w.x), u1 = unit_open(w.y), u2 = unit_open(w.z), u3 = unit_open(w.w);
        const float r0 = sqrtf(-2.f * logf(u0)), r1 = sqrtf(-2.f * logf(u2));
        const float t0 = 6.28318530717958647692f * u1, t1 = 6.28318530717958647692f * u3;
        z[4 * b + 0] = r0 * cosf(t0);
        z[4 * b + 1] = r0 * sinf(t0);
        z[4 * b + 2] = r1 * cosf(t1);
        z[4 * b + 3] = r1 * sinf(t1);
    }
    float qw = dec[3 * ld + i], qx = dec[4 * ld + i], qy = dec[5 * ld + i], qz = dec[6 * ld + i];
    const float inv = 1.f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= inv;
    qx *= inv;
    qy *= inv;
    qz *= inv;
    const float R[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                        2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                        2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
    const float s[3] = {expf(dec[7 * ld + i]), expf(dec[8 * ld + i]), expf(dec[9 * ld + i])};
    const float lshift = 0.47000362924573558f;  // ln 1.6
    for (int c = 0; c < 2; ++c) {
        const int64_t j = offsets[i] + c;
        const float v[3] = {s[0] * z[3 * c + 0], s[1] * z[3 * c + 1], s[2] * z[3 * c + 2]};
#pragma unroll
        for (int r = 0; r < 3; ++r) dst[r * ld_dst + j] += R[3 * r] * v[0] + R[3 * r + 1] * v[1] + R[3 * r + 2] * v[2];
#pragma unroll
        for (int r = 0; r < 3; ++r) dst[(7 + r) * ld_dst + j] -= lshift;
    }
}

int64_t plan_tiles(int64_t n) { return std::max<int64_t>(1, ceil_div(n, kPlanTile)); }

}  // namespace
}  // namespace qg

using namespace qg;

extern "C" qg_status qg_gate_noise(int64_t n, uint64_t seed, int32_t step, const int32_t* step_state, float* noise,
                                   qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && n < (1ll << 32), "n=%lld outside [0, 2^32)", (long long)n);
    QG_REQUIRE(n == 0 || noise, "noise is NULL");
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("gate_noise", s);
        k_gate_noise<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, (uint32_t)seed, (uint32_t)(seed >> 32), step,
                                                                step_state, noise);
    }
    QG_LAUNCH_CHECK("qg_gate_noise");
    return QG_OK;
}

extern "C" qg_status qg_densify_accumulate(int64_t n, const float* grad_xy, const int32_t* ntiles, float sx, float sy,
                                           float* accum, float* count, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0, "n < 0");
    QG_REQUIRE(sx > 0.f && sy > 0.f, "sx and sy must be > 0");
    QG_REQUIRE(n == 0 || (grad_xy && ntiles && accum && count), "a required pointer is NULL");
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    k_densify_accumulate<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, grad_xy, ntiles, sx, sy, accum, count);
    QG_LAUNCH_CHECK("qg_densify_accumulate");
    return QG_OK;
}

extern "C" size_t qg_densify_plan_workspace_size(int64_t n) {
    if (n < 0) return 0;
    return align_up((size_t)plan_tiles(n) * sizeof(int64_t));
}

extern "C" qg_status qg_densify_plan(int64_t n, const float* accum, const float* count, const float* attrs, int64_t ld,
                                     double threshold, double max_scale, double min_opacity, uint8_t* action,
                                     int64_t* offsets, void* ws, size_t ws_bytes, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n, "n=%lld ld=%lld invalid", (long long)n, (long long)ld);
    QG_REQUIRE(threshold >= 0.0 && max_scale > 0.0 && min_opacity >= 0.0 && min_opacity < 1.0,
               "need threshold >= 0, max_scale > 0, 0 <= min_opacity < 1");
    QG_REQUIRE(offsets && (n == 0 || (accum && count && attrs && action)), "a required pointer is NULL");
    const size_t need = qg_densify_plan_workspace_size(n);
    QG_REQUIRE(ws && ws_bytes >= need, "workspace too small: %zu < %zu", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return qg_zero(offsets, 8, stream);
    const int64_t nt = plan_tiles(n);
    int64_t* tiles = (int64_t*)ws;
    {
        QG_TIMED("densify_plan", s);
        k_plan<<<(unsigned)nt, kPlanBlock, 0, s>>>(n, accum, count, attrs, ld, threshold, max_scale, min_opacity,
                                                   action, tiles);
        k_plan_scan<<<1, 1024, 0, s>>>(nt, tiles, offsets + n);
        k_plan_offsets<<<(unsigned)nt, kPlanBlock, 0, s>>>(n, action, tiles, offsets);
    }
    QG_LAUNCH_CHECK("qg_densify_plan");
    return QG_OK;
}

extern "C" qg_status qg_densify_expand(int64_t n, const uint8_t* action, const int64_t* offsets, int32_t nplanes,
                                       const float* src, int64_t ld_src, float* dst, int64_t ld_dst, int32_t mode,
                                       qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld_src >= n && nplanes >= 1 && ld_dst >= 0, "bad sizes");
    QG_REQUIRE(mode == 0 || mode == 1, "mode must be 0 (copy) or 1 (moments)");
    QG_REQUIRE(n == 0 || (action && offsets && src && dst), "a required pointer is NULL");
    QG_REQUIRE(src != dst, "dst may not alias src");
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("densify_expand", s);
        k_expand<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, action, offsets, nplanes, src, ld_src, dst, ld_dst,
                                                            mode);
    }
    QG_LAUNCH_CHECK("qg_densify_expand");
    return QG_OK;
}

extern "C" qg_status qg_densify_children(int64_t n, const uint8_t* action, const int64_t* offsets,
                                         const float* decoded, int64_t ld, uint64_t seed, int32_t round,
                                         float* prev_out, int64_t ld_out, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n && ld_out >= 0, "bad sizes");
    QG_REQUIRE(n == 0 || (action && offsets && decoded && prev_out), "a required pointer is NULL");
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("densify_children", s);
        k_children<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, action, offsets, decoded, ld, (uint32_t)seed,
                                                           (uint32_t)(seed >> 32), (uint32_t)round, prev_out, ld_out);
    }
    QG_LAUNCH_CHECK("qg_densify_children");
    return QG_OK;
}
