// Residual decode and position gate (Eq. 4-8) and their backward.
//
// Both directions run the decoder's dense products on the matrix cores (FP32 MFMA, one wave per group
// of 16 Gaussians): round the latent (Eq. 5), r = W2 SiLU(W1 l), add the residual to the previous
// attributes (Eq. 4), gate the position residual with the hard-concrete gate (Eq. 6-7) and sum Eq. 8's
// probabilities.  The backward forms the straight-through latent gradient, the gate and pre-gate
// position gradients, and the decoder weight gradients (sums over all Gaussians, kept in MFMA
// accumulators per wave, then summed per block and over blocks in a fixed order: deterministic).
#include <cmath>

#include "qg_internal.h"

namespace qg {
namespace {

constexpr int kL = 8;    // latent width
constexpr int kH = 32;   // hidden width
constexpr int kM = 56;   // outputs: rotation 4, log-scale 3, opacity logit 1, SH 48
constexpr int kDecBlock = 256;

__device__ __forceinline__ float sigmoidf_(float x) { return 1.f / (1.f + expf(-x)); }

// ------------------------------------------------------------------------------------------------
// MFMA formulation (v_mfma_f32_16x16x4f32, wave64).  For a 16x16x4 step, lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and accumulates D[4*(l/16)+i][l%16], i = 0..3.  A group of 16 Gaussians is handled
// by one wave; "layout T" means a register holds (feature 16b + 4*(l/16) + i, Gaussian l%16) and
// "layout N" means (Gaussian 4*(l/16) + i, feature 16b + l%16).  Each GEMM is oriented so that the
// output registers of one product are directly the B operand of the next, with the contraction
// step r taking the features (or Gaussians) {r, 4+r, 8+r, 12+r} of a 16-block: the constant
// operand is loaded in the matching permuted order.
// ------------------------------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float silu(float x) { return x * sigmoidf_(x); }
__device__ __forceinline__ float silu_grad(float x) {
    const float s = sigmoidf_(x);
    return s * (1.f + x * (1.f - s));
}

constexpr int kGroup = 16;
constexpr int kMB = 4;  // 56 outputs padded to 64 = 4 blocks of 16

// Forward: pre^T = W1 L^T (layout T), H^T = SiLU(pre^T), R^T = W2 H^T (layout T), out = prev + [g l_p ; R].
__global__ __launch_bounds__(256) void k_decode_fwd_mfma(int64_t n, int64_t ld, const float* __restrict__ prev,
                                                         const float* __restrict__ lat, const float* __restrict__ W1,
                                                         const float* __restrict__ W2, const float* __restrict__ lp,
                                                         const float* __restrict__ ga, float g0, float g1, float tau,
                                                         float reg_shift, float* __restrict__ out,
                                                         float* __restrict__ gate_out, float* __restrict__ lreg_part) {
    __shared__ float s_red[4];
    const int lane = __lane_id(), q = lane / 16, c16 = lane % 16;
    // constant operands
    float aW1[2][2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) aW1[jb][ks] = W1[(16 * jb + c16) * kL + 4 * ks + q];
    float aW2[kMB][2][4];
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = 16 * mb + c16;
                aW2[mb][jb][r] = m < kM ? W2[m * kH + 16 * jb + 4 * q + r] : 0.f;
            }
    const int64_t ngroups = (n + kGroup - 1) / kGroup;
    const int64_t wave = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    float preg = 0.f;
    for (int64_t grp = wave; grp < ngroups; grp += nwaves) {
        const int64_t gb = grp * kGroup;
        const int64_t g = gb + c16;
        const bool gv = g < n;
        f4 pre[2];
        {
            const float b0 = gv ? rintf(lat[(int64_t)q * ld + g]) : 0.f;
            const float b1 = gv ? rintf(lat[(int64_t)(4 + q) * ld + g]) : 0.f;
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                f4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = mfma(aW1[jb][0], b0, acc);
                acc = mfma(aW1[jb][1], b1, acc);
                pre[jb] = acc;
            }
        }
        f4 R[kMB];
#pragma unroll
        for (int mb = 0; mb < kMB; ++mb) R[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float h = silu(pre[jb][r]);
#pragma unroll
                for (int mb = 0; mb < kMB; ++mb) R[mb] = mfma(aW2[mb][jb][r], h, R[mb]);
            }
        if (gv) {
#pragma unroll
            for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = 16 * mb + 4 * q + i;
                    if (m < kM) out[(int64_t)(3 + m) * ld + g] = prev[(int64_t)(3 + m) * ld + g] + R[mb][i];
                }
            // position residual and gate: lane quarter q < 3 handles coordinate q of Gaussian g
            const float a = ga[g];
            const float gt = sigmoidf_(a / tau) * (g1 - g0) + g0;
            const float gg = fminf(1.f, fmaxf(0.f, gt));
            if (q < 3) out[(int64_t)q * ld + g] = prev[(int64_t)q * ld + g] + gg * lp[(int64_t)q * ld + g];
            if (q == 3) {
                if (gate_out) gate_out[g] = gg;
                preg += sigmoidf_(a - reg_shift);
            }
        }
    }
    if (lreg_part) {
        for (int o = 32; o >= 1; o >>= 1) preg += __shfl_xor(preg, o);
        if (lane == 0) s_red[threadIdx.x / 64] = preg;
        __syncthreads();
        if (threadIdx.x == 0) lreg_part[blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    }
}

// Backward.  Per group of 16 Gaussians:
//   pre   = L W1^T            (layout N)       dH = dR W2        (layout N)       dpre = dH * SiLU'(pre)
//   dW2  += dR^T H            (rows m, cols j)  dW1^T += L^T dpre (rows k, cols j)
//   dL^T  = W1^T dpre^T       (dpre transposed to layout T through 2 KB of LDS)
// plus the elementwise gate / position-residual gradients.  Weight-gradient sums stay in registers over
// all groups of the wave, are combined across the block's 4 waves in LDS, and written as one partial
// per block; a second kernel adds the partials in block order.
constexpr int kBwdWidth = kH * kL + kM * kH;  // 2048

__global__ __launch_bounds__(256) void k_decode_bwd_mfma(int64_t n, int64_t ld, const float* __restrict__ lat,
                                                         const float* __restrict__ W1, const float* __restrict__ W2,
                                                         const float* __restrict__ lp, const float* __restrict__ ga,
                                                         float g0, float g1, float tau, float reg_shift,
                                                         float reg_scale, const float* __restrict__ GA,
                                                         float* __restrict__ g_lat, float* __restrict__ g_lp,
                                                         float* __restrict__ g_ga, float* __restrict__ wpart) {
    __shared__ float s_t[4][kGroup][kH + 1];  // per-wave transpose buffer for dpre
    __shared__ float s_w[kBwdWidth];          // block sum of the weight gradients
    const int lane = __lane_id(), q = lane / 16, c16 = lane % 16, w = threadIdx.x / 64;
    for (int i = threadIdx.x; i < kBwdWidth; i += 256) s_w[i] = 0.f;
    // constant operands
    float bW1[2][2];  // B of pre = L W1^T: (k = 4ks + q, j = 16jb + c16)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) bW1[jb][ks] = W1[(16 * jb + c16) * kL + 4 * ks + q];
    float bW2[14][2];  // B of dH = dR W2: (m = 4ks + q, j = 16jb + c16)
#pragma unroll
    for (int ks = 0; ks < 14; ++ks)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) bW2[ks][jb] = W2[(4 * ks + q) * kH + 16 * jb + c16];
    float aW1T[8];  // A of dL^T = W1^T dpre^T: (k = c16, j = 4ks + q)
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) aW1T[ks] = c16 < kL ? W1[(4 * ks + q) * kL + c16] : 0.f;
    f4 accW2[kMB][2];
    f4 accW1[2];
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb) accW2[mb][0] = accW2[mb][1] = f4{0.f, 0.f, 0.f, 0.f};
    accW1[0] = accW1[1] = f4{0.f, 0.f, 0.f, 0.f};
    const int64_t ngroups = (n + kGroup - 1) / kGroup;
    const int64_t wave = (int64_t)blockIdx.x * 4 + w;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t grp = wave; grp < ngroups; grp += nwaves) {
        const int64_t gb = grp * kGroup;
        const int64_t gA = gb + c16;  // Gaussian of this lane in A-row layouts
        const bool vA = gA < n;
        // pre (layout N)
        f4 pre[2];
        {
            const float a0 = vA ? rintf(lat[(int64_t)q * ld + gA]) : 0.f;
            const float a1 = vA ? rintf(lat[(int64_t)(4 + q) * ld + gA]) : 0.f;
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                f4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = mfma(a0, bW1[jb][0], acc);
                acc = mfma(a1, bW1[jb][1], acc);
                pre[jb] = acc;
            }
        }
        // dH = dR W2 (layout N)
        f4 dH[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int ks = 0; ks < 14; ++ks) {
            const float a = vA ? GA[(int64_t)(3 + 4 * ks + q) * ld + gA] : 0.f;
            dH[0] = mfma(a, bW2[ks][0], dH[0]);
            dH[1] = mfma(a, bW2[ks][1], dH[1]);
        }
        // dpre, H (layout N: Gaussian 4q + i, feature 16jb + c16)
        f4 dP[2], H[2];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dP[jb][i] = dH[jb][i] * silu_grad(pre[jb][i]);
                H[jb][i] = silu(pre[jb][i]);
            }
        // weight gradients; contraction step i takes Gaussians {i, 4+i, 8+i, 12+i}
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t gN = gb + 4 * q + i;
            const bool vN = gN < n;
#pragma unroll
            for (int mb = 0; mb < kMB; ++mb) {
                const int m = 16 * mb + c16;
                const float a = (vN && m < kM) ? GA[(int64_t)(3 + m) * ld + gN] : 0.f;
                accW2[mb][0] = mfma(a, H[0][i], accW2[mb][0]);
                accW2[mb][1] = mfma(a, H[1][i], accW2[mb][1]);
            }
            const float al = (vN && c16 < kL) ? rintf(lat[(int64_t)c16 * ld + gN]) : 0.f;
            accW1[0] = mfma(al, dP[0][i], accW1[0]);
            accW1[1] = mfma(al, dP[1][i], accW1[1]);
        }
        // dL^T = W1^T dpre^T: transpose dpre to (feature 4ks + q, Gaussian c16) through LDS
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) s_t[w][4 * q + i][16 * jb + c16] = dP[jb][i];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        f4 dL = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) dL = mfma(aW1T[ks], s_t[w][c16][4 * ks + q], dL);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (vA && q < 2) {
#pragma unroll
            for (int i = 0; i < 4; ++i) g_lat[(int64_t)(4 * q + i) * ld + gA] += dL[i];
        }
        // gate and pre-gate position residual: lane quarter q < 3 holds coordinate q of Gaussian gA
        float dpos = 0.f, lpv = 0.f;
        if (vA && q < 3) {
            dpos = GA[(int64_t)q * ld + gA];
            lpv = lp[(int64_t)q * ld + gA];
        }
        float dot = dpos * lpv;
        dot += __shfl_down(dot, 16);
        dot += __shfl_down(dot, 32);  // lanes 0..15: sum over the three coordinates
        if (vA) {
            const float a = ga[gA];
            const float gh = sigmoidf_(a / tau);
            const float gt = gh * (g1 - g0) + g0;
            const float gg = fminf(1.f, fmaxf(0.f, gt));
            if (q < 3) g_lp[(int64_t)q * ld + gA] += gg * dpos;
            if (q == 0) {
                float da = (gt > 0.f && gt < 1.f) ? dot * (g1 - g0) * gh * (1.f - gh) / tau : 0.f;
                const float pr = sigmoidf_(a - reg_shift);
                da = __builtin_fmaf(reg_scale, pr * (1.f - pr), da);
                g_ga[gA] += da;
            }
        }
    }
    // combine the 4 waves of the block in LDS (fixed order: wave 0, 1, 2, 3)
    for (int k = 0; k < 4; ++k) {
        __syncthreads();
        if (w == k) {
#pragma unroll
            for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
                for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int m = 16 * mb + 4 * q + i;
                        if (m < kM) s_w[kH * kL + m * kH + 16 * jb + c16] += accW2[mb][jb][i];
                    }
            if (q < 2) {
#pragma unroll
                for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) s_w[(16 * jb + c16) * kL + 4 * q + i] += accW1[jb][i];
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBwdWidth; i += 256) wpart[(size_t)blockIdx.x * kBwdWidth + i] = s_w[i];
}

// out[o] += sum over blocks b, in order, of part[b][o]; 64 outputs per block, 4 interleaved partial chains
// combined in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_parts(const float* __restrict__ part, int64_t nblocks,
                                                      float* __restrict__ gW1, float* __restrict__ gW2) {
    __shared__ float s[4][64];
    const int o = blockIdx.x * 64 + threadIdx.x % 64;
    const int c = threadIdx.x / 64;
    float acc = 0.f;
    for (int64_t b = c; b < nblocks; b += 4) acc += part[(size_t)b * kBwdWidth + o];
    s[c][threadIdx.x % 64] = acc;
    __syncthreads();
    if (c == 0) {
        const float t = ((s[0][threadIdx.x] + s[1][threadIdx.x]) + s[2][threadIdx.x]) + s[3][threadIdx.x];
        if (o < kH * kL)
            gW1[o] += t;
        else
            gW2[o - kH * kL] += t;
    }
}

int64_t fwd_blocks(int64_t n) {
    const int64_t groups = std::max<int64_t>(1, ceil_div(n, kGroup));
    return std::min<int64_t>(ceil_div(groups, 4), 1024);
}

int64_t bwd_blocks(int64_t n) {
    const int64_t groups = std::max<int64_t>(1, ceil_div(n, kGroup));
    return std::min<int64_t>(ceil_div(groups, 4), 512);
}

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

extern "C" int64_t qg_decode_lreg_blocks(int64_t n) { return fwd_blocks(n); }

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
    const int64_t nb = fwd_blocks(n);
    if (n == 0) {
        if (lreg_partial) return qg_zero(lreg_partial, 4 * nb, stream);
        return QG_OK;
    }
    const float shift = tau * logf(-gamma0 / gamma1);
    {
        QG_TIMED("decode_fwd", s);
        k_decode_fwd_mfma<<<(unsigned)nb, 256, 0, s>>>(n, ld, prev_attrs, latents, W1, W2, pos_pre, gate_logit,
                                                       gamma0, gamma1, tau, shift, attrs_out, gate_out, lreg_partial);
    }
    QG_LAUNCH_CHECK("qg_decode_residuals");
    return QG_OK;
}

extern "C" size_t qg_decode_bwd_workspace_size(int64_t n, int32_t L, int32_t Hd, int32_t M) {
    (void)L;
    (void)Hd;
    (void)M;
    if (n < 0) return 0;
    return align_up((size_t)bwd_blocks(n) * kBwdWidth * sizeof(float));
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
        k_decode_bwd_mfma<<<(unsigned)nb, 256, 0, s>>>(n, ld, latents, W1, W2, pos_pre, gate_logit, gamma0, gamma1,
                                                       tau, shift, reg_scale, grad_attrs, grad_latents, grad_pos_pre,
                                                       grad_gate_logit, (float*)ws);
    }
    {
        QG_TIMED("decode_wreduce", s);
        k_reduce_parts<<<(unsigned)(kBwdWidth / 64), 256, 0, s>>>((const float*)ws, nb, grad_W1, grad_W2);
    }
    QG_LAUNCH_CHECK("qg_decode_residuals_bwd");
    return QG_OK;
}
