// Residual decode and position gate (Eq. 4-8) and their backward.
//
// Forward, one thread per Gaussian: round the latent (Eq. 5), run the shared decoder
// r = W2 SiLU(W1 l) (weights are wave-uniform and stay in scalar registers / the scalar cache), add the
// residual to the previous attributes (Eq. 4), gate the position residual with the hard-concrete gate
// (Eq. 6-7) and sum Eq. 8's probabilities per block.  Attribute planes are read and written as
// coalesced SoA rows.
//
// Backward: per-Gaussian gradients (straight-through latents, pre-gate position residual, gate logit)
// in one pass; the decoder weight gradients are sums over all Gaussians, formed per block from LDS-staged
// activations and reduced over blocks in a fixed order (deterministic).
#include <cmath>

#include "qg_internal.h"

namespace qg {
namespace {

constexpr int kL = 8;    // latent width
constexpr int kH = 32;   // hidden width
constexpr int kM = 56;   // outputs: rotation 4, log-scale 3, opacity logit 1, SH 48
constexpr int kDecBlock = 256;

__device__ __forceinline__ float sigmoidf_(float x) { return 1.f / (1.f + expf(-x)); }

__global__ __launch_bounds__(kDecBlock) void k_decode_fwd(int64_t n, int64_t ld, const float* __restrict__ prev,
                                                          const float* __restrict__ lat, const float* __restrict__ W1,
                                                          const float* __restrict__ W2,
                                                          const float* __restrict__ lp, const float* __restrict__ ga,
                                                          float g0, float g1, float tau, float reg_shift,
                                                          float* __restrict__ out, float* __restrict__ gate_out,
                                                          float* __restrict__ lreg_part) {
    __shared__ float s_red[kDecBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kDecBlock + threadIdx.x;
    const bool valid = i < n;
    float preg = 0.f;
    if (valid) {
        float l[kL];
#pragma unroll
        for (int k = 0; k < kL; ++k) l[k] = rintf(lat[k * ld + i]);
        float h[kH];
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < kL; ++k) acc = __builtin_fmaf(W1[j * kL + k], l[k], acc);
            h[j] = acc * sigmoidf_(acc);
        }
#pragma unroll 4
        for (int m = 0; m < kM; ++m) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < kH; ++j) acc = __builtin_fmaf(W2[m * kH + j], h[j], acc);
            out[(3 + m) * ld + i] = prev[(3 + m) * ld + i] + acc;
        }
        const float a = ga[i];
        const float gt = sigmoidf_(a / tau) * (g1 - g0) + g0;
        const float g = fminf(1.f, fmaxf(0.f, gt));
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c * ld + i] = prev[c * ld + i] + g * lp[c * ld + i];
        if (gate_out) gate_out[i] = g;
        preg = sigmoidf_(a - reg_shift);
    }
    if (lreg_part) {
        // block sum of Eq. 8's probabilities
        for (int o = 32; o >= 1; o >>= 1) preg += __shfl_xor(preg, o);
        if (__lane_id() == 0) s_red[threadIdx.x / kWave] = preg;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.f;
            for (int w = 0; w < kDecBlock / kWave; ++w) t += s_red[w];
            lreg_part[blockIdx.x] = t;
        }
    }
}

// Backward.  Block = 128 threads; each block covers kChunks chunks of 128 Gaussians and keeps its share of
// the weight-gradient sums in registers: thread t owns dW2[m][j] for m in 7*(t/16) .. +7, j in 2*(t%16) .. +2,
// and dW1[j][k] for j = t % 32, k = t/32 + 4 r (r = 0, 1).
constexpr int kBB = 128;
constexpr int kChunks = 4;

__global__ __launch_bounds__(kBB) void k_decode_bwd(int64_t n, int64_t ld, const float* __restrict__ lat,
                                                    const float* __restrict__ W1, const float* __restrict__ W2,
                                                    const float* __restrict__ lp, const float* __restrict__ ga,
                                                    float g0, float g1, float tau, float reg_shift, float reg_scale,
                                                    const float* __restrict__ GA, float* __restrict__ g_lat,
                                                    float* __restrict__ g_lp, float* __restrict__ g_ga,
                                                    float* __restrict__ wpart) {
    __shared__ float s_dr[kBB][kM + 1];
    __shared__ float s_h[kBB][kH + 1];
    __shared__ float s_dp[kBB][kH + 1];
    __shared__ float s_l[kBB][kL + 1];
    const int t = threadIdx.x;
    const int mg = t / 16, jg = t % 16;
    float accW2[7][2];
#pragma unroll
    for (int a = 0; a < 7; ++a) accW2[a][0] = accW2[a][1] = 0.f;
    float accW1[2] = {0.f, 0.f};
    const int j1 = t % 32, k1 = t / 32;
    for (int c = 0; c < kChunks; ++c) {
        const int64_t i = ((int64_t)blockIdx.x * kChunks + c) * kBB + t;
        const bool valid = i < n;
        float l[kL], dr[kM];
        if (valid) {
#pragma unroll
            for (int k = 0; k < kL; ++k) l[k] = rintf(lat[k * ld + i]);
#pragma unroll
            for (int m = 0; m < kM; ++m) dr[m] = GA[(3 + m) * ld + i];
        } else {
#pragma unroll
            for (int k = 0; k < kL; ++k) l[k] = 0.f;
#pragma unroll
            for (int m = 0; m < kM; ++m) dr[m] = 0.f;
        }
        float pre[kH], h[kH];
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < kL; ++k) acc = __builtin_fmaf(W1[j * kL + k], l[k], acc);
            pre[j] = acc;
            h[j] = acc * sigmoidf_(acc);
        }
        // dh = W2^T dr ; dpre = dh * SiLU'(pre)
        float dp[kH];
#pragma unroll
        for (int j = 0; j < kH; ++j) dp[j] = 0.f;
#pragma unroll 4
        for (int m = 0; m < kM; ++m) {
#pragma unroll
            for (int j = 0; j < kH; ++j) dp[j] = __builtin_fmaf(W2[m * kH + j], dr[m], dp[j]);
        }
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            const float sg = sigmoidf_(pre[j]);
            dp[j] *= sg * (1.f + pre[j] * (1.f - sg));
        }
        if (valid) {
            // straight-through: d/d latent = d/d rounded latent = W1^T dpre
#pragma unroll
            for (int k = 0; k < kL; ++k) {
                float acc = 0.f;
#pragma unroll
                for (int j = 0; j < kH; ++j) acc = __builtin_fmaf(W1[j * kL + k], dp[j], acc);
                g_lat[k * ld + i] += acc;
            }
            // gate and position residual
            const float a = ga[i];
            const float gh = sigmoidf_(a / tau);
            const float gt = gh * (g1 - g0) + g0;
            const float g = fminf(1.f, fmaxf(0.f, gt));
            float dot = 0.f;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const float dpos = GA[cc * ld + i];
                dot = __builtin_fmaf(dpos, lp[cc * ld + i], dot);
                g_lp[cc * ld + i] += g * dpos;
            }
            float da = (gt > 0.f && gt < 1.f) ? dot * (g1 - g0) * gh * (1.f - gh) / tau : 0.f;
            const float pr = sigmoidf_(a - reg_shift);
            da = __builtin_fmaf(reg_scale, pr * (1.f - pr), da);
            g_ga[i] += da;
        }
        // stage for the weight-gradient sums
#pragma unroll
        for (int m = 0; m < kM; ++m) s_dr[t][m] = dr[m];
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            s_h[t][j] = valid ? h[j] : 0.f;
            s_dp[t][j] = valid ? dp[j] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < kL; ++k) s_l[t][k] = l[k];
        __syncthreads();
        for (int q = 0; q < kBB; ++q) {
            const float h0 = s_h[q][2 * jg], h1 = s_h[q][2 * jg + 1];
#pragma unroll
            for (int a = 0; a < 7; ++a) {
                const float d = s_dr[q][7 * mg + a];
                accW2[a][0] = __builtin_fmaf(d, h0, accW2[a][0]);
                accW2[a][1] = __builtin_fmaf(d, h1, accW2[a][1]);
            }
            const float dpj = s_dp[q][j1];
            accW1[0] = __builtin_fmaf(dpj, s_l[q][k1], accW1[0]);
            accW1[1] = __builtin_fmaf(dpj, s_l[q][k1 + 4], accW1[1]);
        }
        __syncthreads();
    }
    float* wp = wpart + (size_t)blockIdx.x * (kH * kL + kM * kH);
    wp[j1 * kL + k1] = accW1[0];
    wp[j1 * kL + k1 + 4] = accW1[1];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
        wp[kH * kL + (7 * mg + a) * kH + 2 * jg] = accW2[a][0];
        wp[kH * kL + (7 * mg + a) * kH + 2 * jg + 1] = accW2[a][1];
    }
}

// out[o] += sum over blocks b (in order) of part[b][o]
__global__ void k_reduce_parts(const float* __restrict__ part, int64_t nblocks, int width, float* __restrict__ gW1,
                               float* __restrict__ gW2) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= width) return;
    float acc = 0.f;
    for (int64_t b = 0; b < nblocks; ++b) acc += part[(size_t)b * width + o];
    if (o < kH * kL)
        gW1[o] += acc;
    else
        gW2[o - kH * kL] += acc;
}

int64_t bwd_blocks(int64_t n) { return std::max<int64_t>(1, ceil_div(n, (int64_t)kBB * kChunks)); }

}  // namespace
}  // namespace qg

using namespace qg;

static qg_status check_decoder(int32_t L, int32_t Hd, int32_t M) {
    QG_REQUIRE(L >= 1 && L <= 16, "L=%d outside [1, 16]", L);
    QG_REQUIRE(Hd == 0 || Hd == 32, "Hd=%d must be 0 or 32", Hd);
    QG_REQUIRE(M == 56, "M=%d must be 56", M);
    if (!(L == kL && Hd == kH)) {
        set_error("decoder shape L=%d Hd=%d not built (supported: L=8, Hd=32)", L, Hd);
        return QG_ERR_UNSUPPORTED;
    }
    return QG_OK;
}

static qg_status check_gate(float g0, float g1, float tau) {
    QG_REQUIRE(g0 < 0.f && g1 > 1.f && tau > 0.f, "need gamma0 < 0, gamma1 > 1, tau > 0");
    return QG_OK;
}

extern "C" int64_t qg_decode_lreg_blocks(int64_t n) { return std::max<int64_t>(1, ceil_div(n, kDecBlock)); }

extern "C" qg_status qg_decode_residuals(int64_t n, int64_t ld, const float* prev_attrs, const float* latents,
                                         int32_t L, const float* W1, const float* W2, int32_t Hd, int32_t M,
                                         const float* pos_pre, const float* gate_logit, float gamma0, float gamma1,
                                         float tau, float* attrs_out, float* gate_out, float* lreg_partial,
                                         qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n, "n=%lld ld=%lld: need 0 <= n <= ld", (long long)n, (long long)ld);
    qg_status st = check_decoder(L, Hd, M);
    if (st != QG_OK) return st;
    st = check_gate(gamma0, gamma1, tau);
    if (st != QG_OK) return st;
    QG_REQUIRE(n == 0 || (prev_attrs && latents && W1 && W2 && pos_pre && gate_logit && attrs_out),
               "a required pointer is NULL");
    QG_REQUIRE(attrs_out != prev_attrs, "attrs_out may not alias prev_attrs");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = qg_decode_lreg_blocks(n);
    if (n == 0) {
        if (lreg_partial) return qg_zero(lreg_partial, 4 * nb, stream);
        return QG_OK;
    }
    const float shift = tau * logf(-gamma0 / gamma1);
    {
        QG_TIMED("decode_fwd", s);
        k_decode_fwd<<<(unsigned)nb, kDecBlock, 0, s>>>(n, ld, prev_attrs, latents, W1, W2, pos_pre, gate_logit, gamma0,
                                                        gamma1, tau, shift, attrs_out, gate_out, lreg_partial);
    }
    QG_LAUNCH_CHECK("qg_decode_residuals");
    return QG_OK;
}

extern "C" size_t qg_decode_bwd_workspace_size(int64_t n, int32_t L, int32_t Hd, int32_t M) {
    (void)L;
    (void)Hd;
    (void)M;
    if (n < 0) return 0;
    return align_up((size_t)bwd_blocks(n) * (kH * kL + kM * kH) * sizeof(float));
}

extern "C" qg_status qg_decode_residuals_bwd(int64_t n, int64_t ld, const float* latents, int32_t L,
                                             const float* W1, const float* W2, int32_t Hd, int32_t M,
                                             const float* pos_pre, const float* gate_logit, float gamma0,
                                             float gamma1, float tau, const float* grad_attrs, float lambda_reg,
                                             float* grad_latents, float* grad_W1, float* grad_W2,
                                             float* grad_pos_pre, float* grad_gate_logit, void* ws, size_t ws_bytes,
                                             qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n, "n=%lld ld=%lld: need 0 <= n <= ld", (long long)n, (long long)ld);
    qg_status st = check_decoder(L, Hd, M);
    if (st != QG_OK) return st;
    st = check_gate(gamma0, gamma1, tau);
    if (st != QG_OK) return st;
    QG_REQUIRE(n == 0 || (latents && W1 && W2 && pos_pre && gate_logit && grad_attrs && grad_latents && grad_W1 &&
                          grad_W2 && grad_pos_pre && grad_gate_logit),
               "a required pointer is NULL");
    const size_t need = qg_decode_bwd_workspace_size(n, L, Hd, M);
    QG_REQUIRE(ws && ws_bytes >= need, "workspace too small: %zu < %zu", ws_bytes, need);
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = bwd_blocks(n);
    const float shift = tau * logf(-gamma0 / gamma1);
    const float reg_scale = lambda_reg / (float)n;
    {
        QG_TIMED("decode_bwd", s);
        k_decode_bwd<<<(unsigned)nb, kBB, 0, s>>>(n, ld, latents, W1, W2, pos_pre, gate_logit, gamma0, gamma1, tau, shift,
                                                  reg_scale, grad_attrs, grad_latents, grad_pos_pre, grad_gate_logit,
                                                  (float*)ws);
    }
    const int width = kH * kL + kM * kH;
    {
        QG_TIMED("decode_wreduce", s);
        k_reduce_parts<<<(unsigned)ceil_div(width, 256), 256, 0, s>>>((const float*)ws, nb, width, grad_W1, grad_W2);
    }
    QG_LAUNCH_CHECK("qg_decode_residuals_bwd");
    return QG_OK;
}
