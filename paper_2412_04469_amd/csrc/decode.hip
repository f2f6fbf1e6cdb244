// Residual decode and position gate (Eq. 4-8) and their backward.
//
// The decoder's dense products run on FP32 matrix cores (decoder_mfma.h).  One wave owns 64 consecutive
// Gaussians at a time: the MFMA results go through LDS so that every access to an attribute plane is a
// contiguous 256-byte row (lane = Gaussian).  Forward: round the latent (Eq. 5), r = W2 SiLU(W1 l), add
// the residual to the previous attributes (Eq. 4), gate the position residual with the hard-concrete
// gate (Eq. 6-7) and sum Eq. 8's probabilities.  Backward: the straight-through latent gradient, the gate
// and pre-gate position gradients, and the decoder weight gradients (kept in MFMA accumulators per wave,
// summed per block in a fixed wave order, then over blocks in a fixed order: deterministic).
#include <cmath>

#include "decoder_mfma.h"

namespace qg {
namespace {

using namespace dec;

constexpr int kChunk = 64;  // Gaussians per wave iteration

int64_t fwd_blocks(int64_t n) {
    const int64_t chunks = std::max<int64_t>(1, ceil_div(n, kChunk));
    return std::min<int64_t>(ceil_div(chunks, 4), 1024);
}

int64_t bwd_blocks(int64_t n) {
    const int64_t chunks = std::max<int64_t>(1, ceil_div(n, kChunk));
    return std::min<int64_t>(ceil_div(chunks, 4), 512);
}

__global__ __launch_bounds__(256) void k_decode_fwd(int64_t n, int64_t ld, const float* __restrict__ prev,
                                                    const float* __restrict__ lat, const float* __restrict__ W1,
                                                    const float* __restrict__ W2, const float* __restrict__ lp,
                                                    const float* __restrict__ ga, const float* __restrict__ gnoise,
                                                    float g0, float g1, float tau, float reg_shift,
                                                    float* __restrict__ out, float* __restrict__ gate_out,
                                                    float* __restrict__ lreg_part) {
    __shared__ float s_res[4][kChunk][kM + 1];
    __shared__ float s_red[4];
    const int lane = __lane_id(), w = threadIdx.x / 64, c = lane % 16;
    FwdOps ops;
    load_fwd_ops(W1, W2, ops);
    const int64_t nchunks = ceil_div(n, kChunk);
    float preg = 0.f;
    for (int64_t ch = (int64_t)blockIdx.x * 4 + w; ch < nchunks; ch += (int64_t)gridDim.x * 4) {
        const int64_t base = ch * kChunk;
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
            const int64_t g = base + 16 * sg + c;
            const bool gv = g < n;
            auto latf = [&](int k) { return gv ? rintf(lat[(int64_t)k * ld + g]) : 0.f; };
            auto outf = [&](int m, float v) { s_res[w][16 * sg + c][m] = v; };
            decode_group_fwd(ops, latf, outf);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t g = base + lane;
        if (g < n) {
#pragma unroll 8
            for (int m = 0; m < kM; ++m) out[(int64_t)(3 + m) * ld + g] = prev[(int64_t)(3 + m) * ld + g] + s_res[w][lane][m];
            const float a = ga[g];
            // the stochastic gate adds its logistic sample to log(alpha) inside the sigmoid (Eq. 6)
            const float gg = gate_of(gnoise ? a + gnoise[g] : a, g0, g1, tau, nullptr, nullptr);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                out[(int64_t)k * ld + g] = __builtin_fmaf(gg, lp[(int64_t)k * ld + g], prev[(int64_t)k * ld + g]);
            if (gate_out) gate_out[g] = gg;
            preg += sigm(a - reg_shift);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (lreg_part) {
        for (int o = 32; o >= 1; o >>= 1) preg += __shfl_xor(preg, o);
        if (lane == 0) s_red[w] = preg;
        __syncthreads();
        if (threadIdx.x == 0) lreg_part[blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    }
}

__global__ __launch_bounds__(256) void k_decode_bwd(int64_t n, int64_t ld, const float* __restrict__ lat,
                                                    const float* __restrict__ W1, const float* __restrict__ W2,
                                                    const float* __restrict__ lp, const float* __restrict__ ga,
                                                    const float* __restrict__ gnoise, float g0, float g1, float tau,
                                                    float reg_shift, float reg_scale,
                                                    const float* __restrict__ GA, float* __restrict__ g_lat,
                                                    float* __restrict__ g_lp, float* __restrict__ g_ga,
                                                    float* __restrict__ wpart) {
    __shared__ float s_dr[4][kChunk][kM + 1];
    __shared__ float s_t[4][16][33];
    __shared__ float s_w[kWidth];
    const int lane = __lane_id(), w = threadIdx.x / 64, q = lane / 16, c = lane % 16;
    for (int i = threadIdx.x; i < kWidth; i += 256) s_w[i] = 0.f;
    BwdOps ops;
    load_bwd_ops(W1, W2, ops);
    BwdAcc acc;
    zero_acc(acc);
    const int64_t nchunks = ceil_div(n, kChunk);
    for (int64_t ch = (int64_t)blockIdx.x * 4 + w; ch < nchunks; ch += (int64_t)gridDim.x * 4) {
        const int64_t base = ch * kChunk;
        const int64_t g = base + lane;
        const bool gv = g < n;
        // stage dL/dr (planes 3..58) with lane = Gaussian; gate and position gradients elementwise
#pragma unroll 8
        for (int m = 0; m < kM; ++m) s_dr[w][lane][m] = gv ? GA[(int64_t)(3 + m) * ld + g] : 0.f;
        if (gv) {
            const float a = ga[g];
            float gh, gt;
            const float gg = gate_of(gnoise ? a + gnoise[g] : a, g0, g1, tau, &gh, &gt);
            float dot = 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float dpos = GA[(int64_t)k * ld + g];
                dot = __builtin_fmaf(dpos, lp[(int64_t)k * ld + g], dot);
                g_lp[(int64_t)k * ld + g] += gg * dpos;
            }
            float da = (gt > 0.f && gt < 1.f) ? dot * (g1 - g0) * gh * (1.f - gh) / tau : 0.f;
            const float pr = sigm(a - reg_shift);
            g_ga[g] += __builtin_fmaf(reg_scale, pr * (1.f - pr), da);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
            const int64_t gA = base + 16 * sg + c;
            const bool vA = gA < n;
            auto latA = [&](int k) { return vA ? rintf(lat[(int64_t)k * ld + gA]) : 0.f; };
            auto latN = [&](int k, int i) {
                const int64_t gN = base + 16 * sg + 4 * q + i;
                return gN < n ? rintf(lat[(int64_t)k * ld + gN]) : 0.f;
            };
            auto drA = [&](int m) { return s_dr[w][16 * sg + c][m]; };
            auto drN = [&](int m, int i) { return m < kM ? s_dr[w][16 * sg + 4 * q + i][m] : 0.f; };
            auto dlat = [&](int k, float v) {
                if (vA) g_lat[(int64_t)k * ld + gA] += v;
            };
            decode_group_bwd(ops, acc, latA, latN, drA, drN, dlat, TransposeBuf{s_t[w]});
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int k = 0; k < 4; ++k) {
        __syncthreads();
        if (w == k) add_acc(acc, s_w);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kWidth; i += 256) wpart[(size_t)blockIdx.x * kWidth + i] = s_w[i];
}

// out[o] += sum over blocks b of part[b][o], in a fixed order: 32 outputs per block, 8 interleaved chains
// (b = c, c + 8, ...) per output, combined in chain order.
// Sum of the per-block partials, deterministic: a block owns 16 columns; its 64 row groups each sum every
// 64th partial, then one thread per column adds the 64 group sums in order.
__global__ __launch_bounds__(1024) void k_reduce_parts(const float* __restrict__ part, int64_t nblocks,
                                                       float* __restrict__ gW1, float* __restrict__ gW2) {
    __shared__ float s[64][17];
    const int col = threadIdx.x % 16, rg = threadIdx.x / 16;
    const int o = blockIdx.x * 16 + col;
    float acc = 0.f;
#pragma unroll 16
    for (int64_t b = rg; b < nblocks; b += 64) acc += part[(size_t)b * kWidth + o];
    s[rg][col] = acc;
    __syncthreads();
    if (threadIdx.x < 16) {
        float t = 0.f;
        for (int k = 0; k < 64; ++k) t += s[k][col];
        if (o < kH * kL)
            gW1[o] += t;
        else
            gW2[o - kH * kL] += t;
    }
}

// Eq. 8 as a mean: out[0] = (sum of the nb block sums) / n, in a fixed order (strided per-thread sums in double,
// then a tree over the 256 threads).
__global__ __launch_bounds__(256) void k_lreg_mean(const float* __restrict__ part, int64_t nb, int64_t n,
                                                   float* __restrict__ out) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) acc += (double)part[b];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = n > 0 ? (float)(s[0] / (double)n) : 0.f;
}

// Adjoint of the mean with respect to the gate logits, the weight dLoss/dL_reg read from the device.
__global__ void k_lreg_bwd(int64_t n, const float* __restrict__ a, float reg_shift, const float* __restrict__ weight,
                           float inv_n, float* __restrict__ ga) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float pr = sigm(a[i] - reg_shift);
    ga[i] += (weight[0] * inv_n) * (pr * (1.f - pr));
}

}  // namespace

qg_status decode_reduce_launch(const float* part, int64_t nblocks, float* gW1, float* gW2, hipStream_t s) {
    QG_TIMED("decode_wreduce", s);
    k_reduce_parts<<<(unsigned)(kWidth / 16), 1024, 0, s>>>(part, nblocks, gW1, gW2);
    QG_LAUNCH_CHECK("decode weight reduce");
    return QG_OK;
}

}  // namespace qg

using namespace qg;

using namespace qg::dec;

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
                                         const float* pos_pre, const float* gate_logit, const float* gate_noise,
                                         float gamma0, float gamma1, float tau, float* attrs_out, float* gate_out,
                                         float* lreg_partial, qg_stream stream) {
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
        k_decode_fwd<<<(unsigned)nb, 256, 0, s>>>(n, ld, prev_attrs, latents, W1, W2, pos_pre, gate_logit, gate_noise,
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
    return align_up((size_t)bwd_blocks(n) * kWidth * sizeof(float));
}

extern "C" qg_status qg_decode_residuals_bwd(int64_t n, int64_t ld, const float* latents, int32_t L,
                                             const float* W1, const float* W2, int32_t Hd, int32_t M,
                                             const float* pos_pre, const float* gate_logit, const float* gate_noise,
                                             float gamma0, float gamma1, float tau, const float* grad_attrs,
                                             float lambda_reg,
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
        k_decode_bwd<<<(unsigned)nb, 256, 0, s>>>(n, ld, latents, W1, W2, pos_pre, gate_logit, gate_noise, gamma0,
                                                  gamma1, tau, shift, reg_scale, grad_attrs, grad_latents, grad_pos_pre,
                                                  grad_gate_logit, (float*)ws);
    }
    QG_LAUNCH_CHECK("qg_decode_residuals_bwd");
    return decode_reduce_launch((const float*)ws, nb, grad_W1, grad_W2, s);
}

extern "C" qg_status qg_decode_lreg_mean(int64_t n, const float* lreg_partial, int64_t nblocks, float* out,
                                         qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && nblocks >= 0, "n=%lld nblocks=%lld must be >= 0", (long long)n, (long long)nblocks);
    QG_REQUIRE(out && (nblocks == 0 || lreg_partial), "a required pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("decode_lreg_mean", s);
        k_lreg_mean<<<1, 256, 0, s>>>(lreg_partial, nblocks, n, out);
    }
    QG_LAUNCH_CHECK("qg_decode_lreg_mean");
    return QG_OK;
}

extern "C" qg_status qg_decode_lreg_bwd(int64_t n, const float* gate_logit, float gamma0, float gamma1, float tau,
                                        const float* weight, float* grad_gate_logit, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0, "n=%lld < 0", (long long)n);
    qg_status st = check_gate(gamma0, gamma1, tau);
    if (st != QG_OK) return st;
    QG_REQUIRE(n == 0 || (gate_logit && weight && grad_gate_logit), "a required pointer is NULL");
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    const float shift = tau * logf(-gamma0 / gamma1);
    {
        QG_TIMED("decode_lreg_bwd", s);
        k_lreg_bwd<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, gate_logit, shift, weight, 1.f / (float)n,
                                                               grad_gate_logit);
    }
    QG_LAUNCH_CHECK("qg_decode_lreg_bwd");
    return QG_OK;
}

// ---------------------------------------------------------------------------------------------------------
// Paper-mode decoder (Eq. 5 as written): one linear decoder per attribute category, r_c = D_c rint(l_c).
// Rotation (4 planes from 3), scaling (3 from 7), opacity (1 from 10), colour base (3 from 11) and colour
// frequencies (45 from 14); latent dimensions L_c from the host.  D is packed category by category, each D_c
// row-major [M_c][L_c].  It is a block-diagonal map of about 500 flop per Gaussian against ~600 bytes moved,
// so it runs on the vector units, one lane per Gaussian; the decoder's weight gradient sum over Gaussians is
// reduced per wave by shuffles, per block in wave order and over blocks in block order (deterministic).
// ---------------------------------------------------------------------------------------------------------
namespace qg {
namespace {

constexpr int kCats = 5;
constexpr int kCatPlane[kCats] = {3, 7, 10, 11, 14};
constexpr int kCatOut[kCats] = {4, 3, 1, 3, 45};
constexpr int kLinMaxL = 16;                      // per category
constexpr int kLinMaxP = 56 * kLinMaxL;           // packed decoder floats

struct LinDims {
    int L[kCats];     // latent dims
    int loff[kCats];  // first latent plane of the category
    int doff[kCats];  // first packed decoder float of the category
    int total_L, total_P;
};

__device__ __forceinline__ int cat_plane(int c) {
    return c == 0 ? 3 : (c == 1 ? 7 : (c == 2 ? 10 : (c == 3 ? 11 : 14)));
}
__device__ __forceinline__ int cat_out(int c) { return c == 0 ? 4 : (c == 1 ? 3 : (c == 2 ? 1 : (c == 3 ? 3 : 45))); }

constexpr int kLinBlock = 256;

__global__ __launch_bounds__(kLinBlock) void k_decode_linear(int64_t n, int64_t ld, const float* __restrict__ prev,
                                                             const float* __restrict__ lat, LinDims dm,
                                                             const float* __restrict__ D, const float* __restrict__ lp,
                                                             const float* __restrict__ ga,
                                                             const float* __restrict__ gnoise, float g0, float g1,
                                                             float tau, float reg_shift, float* __restrict__ out,
                                                             float* __restrict__ gate_out,
                                                             float* __restrict__ lreg_part) {
    __shared__ float s_D[kLinMaxP];
    __shared__ float s_red[kLinBlock / 64];
    for (int i = threadIdx.x; i < dm.total_P; i += kLinBlock) s_D[i] = D[i];
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * kLinBlock + threadIdx.x;
    float preg = 0.f;
    if (g < n) {
#pragma unroll 1
        for (int c = 0; c < kCats; ++c) {
            float l[kLinMaxL];
#pragma unroll
            for (int k = 0; k < kLinMaxL; ++k) l[k] = k < dm.L[c] ? rintf(lat[(int64_t)(dm.loff[c] + k) * ld + g]) : 0.f;
            const float* Dc = s_D + dm.doff[c];
            const int M = cat_out(c), L = dm.L[c], p0 = cat_plane(c);
            for (int m = 0; m < M; ++m) {
                float r = 0.f;
#pragma unroll
                for (int k = 0; k < kLinMaxL; ++k)
                    if (k < L) r = __builtin_fmaf(Dc[m * L + k], l[k], r);
                out[(int64_t)(p0 + m) * ld + g] = prev[(int64_t)(p0 + m) * ld + g] + r;
            }
        }
        const float a = ga[g];
        const float gg = gate_of(gnoise ? a + gnoise[g] : a, g0, g1, tau, nullptr, nullptr);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            out[(int64_t)k * ld + g] = __builtin_fmaf(gg, lp[(int64_t)k * ld + g], prev[(int64_t)k * ld + g]);
        if (gate_out) gate_out[g] = gg;
        preg = sigm(a - reg_shift);
    }
    if (lreg_part) {
        for (int o = 32; o >= 1; o >>= 1) preg += __shfl_xor(preg, o);
        if (__lane_id() == 0) s_red[threadIdx.x / 64] = preg;
        __syncthreads();
        if (threadIdx.x == 0) lreg_part[blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    }
}

// Backward: dL/dl_c = D_c^T dL/dr_c (straight-through), the gate and pre-gate position gradients as in the MLP
// form, and per block the sum over its Gaussians of dL/dr_c rint(l_c)^T (wave sums by shuffles, then the waves in
// order) into wpart[block][P].
__global__ __launch_bounds__(kLinBlock) void k_decode_linear_bwd(
    int64_t n, int64_t ld, const float* __restrict__ lat, LinDims dm, const float* __restrict__ D,
    const float* __restrict__ lp, const float* __restrict__ ga, const float* __restrict__ gnoise, float g0, float g1,
    float tau, float reg_shift, float reg_scale, const float* __restrict__ GA, float* __restrict__ g_lat,
    float* __restrict__ g_lp, float* __restrict__ g_ga, float* __restrict__ wpart) {
    __shared__ float s_D[kLinMaxP];
    __shared__ float s_w[kLinBlock / 64][kLinMaxP];
    for (int i = threadIdx.x; i < dm.total_P; i += kLinBlock) s_D[i] = D[i];
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * kLinBlock + threadIdx.x;
    const bool gv = g < n;
    const int w = threadIdx.x / 64, lane = __lane_id();
#pragma unroll 1
    for (int c = 0; c < kCats; ++c) {
        const int M = cat_out(c), L = dm.L[c], p0 = cat_plane(c);
        float l[kLinMaxL], gl[kLinMaxL];
#pragma unroll
        for (int k = 0; k < kLinMaxL; ++k) {
            l[k] = (gv && k < L) ? rintf(lat[(int64_t)(dm.loff[c] + k) * ld + g]) : 0.f;
            gl[k] = 0.f;
        }
        const float* Dc = s_D + dm.doff[c];
        for (int m = 0; m < M; ++m) {
            const float dr = gv ? GA[(int64_t)(p0 + m) * ld + g] : 0.f;
#pragma unroll
            for (int k = 0; k < kLinMaxL; ++k) {
                if (k >= L) continue;
                gl[k] = __builtin_fmaf(Dc[m * L + k], dr, gl[k]);
                float v = dr * l[k];  // this Gaussian's term of dL/dD_c[m][k]; summed over the wave
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
                if (lane == 0) s_w[w][dm.doff[c] + m * L + k] = v;
            }
        }
        if (gv) {
#pragma unroll
            for (int k = 0; k < kLinMaxL; ++k)
                if (k < L) g_lat[(int64_t)(dm.loff[c] + k) * ld + g] += gl[k];
        }
    }
    if (gv) {
        const float a = ga[g];
        float gh, gt;
        const float gg = gate_of(gnoise ? a + gnoise[g] : a, g0, g1, tau, &gh, &gt);
        float dot = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float dpos = GA[(int64_t)k * ld + g];
            dot = __builtin_fmaf(dpos, lp[(int64_t)k * ld + g], dot);
            g_lp[(int64_t)k * ld + g] += gg * dpos;
        }
        const float da = (gt > 0.f && gt < 1.f) ? dot * (g1 - g0) * gh * (1.f - gh) / tau : 0.f;
        const float pr = sigm(a - reg_shift);
        g_ga[g] += __builtin_fmaf(reg_scale, pr * (1.f - pr), da);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < dm.total_P; i += kLinBlock)
        wpart[(size_t)blockIdx.x * dm.total_P + i] = (s_w[0][i] + s_w[1][i]) + (s_w[2][i] + s_w[3][i]);
}

// grad_D[i] += sum over blocks of wpart[b][i]: one wave per decoder float, lane l summing blocks l, l + 64, ...
// in order, then a fixed butterfly over the lanes (deterministic).
__global__ __launch_bounds__(256) void k_linear_reduce(const float* __restrict__ wpart, int64_t nb, int P,
                                                       float* __restrict__ gD) {
    const int i = blockIdx.x * 4 + threadIdx.x / 64, lane = __lane_id();
    if (i >= P) return;
    float s = 0.f;
    for (int64_t b = lane; b < nb; b += 64) s += wpart[(size_t)b * P + i];
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) gD[i] += s;
}

bool lin_dims(const int32_t* dims, LinDims* d) {
    if (!dims) {
        set_error("dims is NULL");
        return false;
    }
    int lo = 0, po = 0;
    for (int c = 0; c < kCats; ++c) {
        if (dims[c] < 1 || dims[c] > kLinMaxL) {
            set_error("latent dimension %d of category %d outside [1, %d]", dims[c], c, kLinMaxL);
            return false;
        }
        d->L[c] = dims[c];
        d->loff[c] = lo;
        d->doff[c] = po;
        lo += dims[c];
        po += dims[c] * kCatOut[c];
    }
    d->total_L = lo;
    d->total_P = po;
    return true;
}

}  // namespace
}  // namespace qg

extern "C" int64_t qg_linear_decoder_params(const int32_t* dims) {
    LinDims d;
    if (!lin_dims(dims, &d)) return -1;
    return d.total_P;
}

extern "C" int64_t qg_decode_linear_blocks(int64_t n) { return std::max<int64_t>(1, ceil_div(n, kLinBlock)); }

extern "C" qg_status qg_decode_linear(int64_t n, int64_t ld, const float* prev_attrs, const float* latents,
                                      const int32_t* dims, const float* D, const float* pos_pre,
                                      const float* gate_logit, const float* gate_noise, float gamma0, float gamma1,
                                      float tau, float* attrs_out, float* gate_out, float* lreg_partial,
                                      qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n, "n=%lld ld=%lld: need 0 <= n <= ld", (long long)n, (long long)ld);
    LinDims dm;
    if (!lin_dims(dims, &dm)) return QG_ERR_ARG;
    qg_status st = check_gate(gamma0, gamma1, tau);
    if (st != QG_OK) return st;
    QG_REQUIRE(n == 0 || (prev_attrs && latents && D && pos_pre && gate_logit && attrs_out), "a required pointer is NULL");
    QG_REQUIRE(attrs_out != prev_attrs, "attrs_out may not alias prev_attrs");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = qg_decode_linear_blocks(n);
    if (n == 0) return lreg_partial ? qg_zero(lreg_partial, 4 * nb, stream) : QG_OK;
    const float shift = tau * logf(-gamma0 / gamma1);
    {
        QG_TIMED("decode_linear", s);
        k_decode_linear<<<(unsigned)nb, kLinBlock, 0, s>>>(n, ld, prev_attrs, latents, dm, D, pos_pre, gate_logit,
                                                           gate_noise, gamma0, gamma1, tau, shift, attrs_out, gate_out,
                                                           lreg_partial);
    }
    QG_LAUNCH_CHECK("qg_decode_linear");
    return QG_OK;
}

extern "C" size_t qg_decode_linear_bwd_workspace_size(int64_t n, const int32_t* dims) {
    LinDims dm;
    if (n < 0 || !lin_dims(dims, &dm)) return 0;
    return align_up((size_t)qg_decode_linear_blocks(n) * dm.total_P * sizeof(float));
}

extern "C" qg_status qg_decode_linear_bwd(int64_t n, int64_t ld, const float* latents, const int32_t* dims,
                                          const float* D, const float* pos_pre, const float* gate_logit,
                                          const float* gate_noise, float gamma0, float gamma1, float tau,
                                          const float* grad_attrs, float lambda_reg, float* grad_latents,
                                          float* grad_D, float* grad_pos_pre, float* grad_gate_logit, void* ws,
                                          size_t ws_bytes, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n, "n=%lld ld=%lld: need 0 <= n <= ld", (long long)n, (long long)ld);
    LinDims dm;
    if (!lin_dims(dims, &dm)) return QG_ERR_ARG;
    qg_status st = check_gate(gamma0, gamma1, tau);
    if (st != QG_OK) return st;
    QG_REQUIRE(n == 0 || (latents && D && pos_pre && gate_logit && grad_attrs && grad_latents && grad_D &&
                          grad_pos_pre && grad_gate_logit),
               "a required pointer is NULL");
    const size_t need = qg_decode_linear_bwd_workspace_size(n, dims);
    QG_REQUIRE(ws && ws_bytes >= need, "workspace too small: %zu < %zu", ws_bytes, need);
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = qg_decode_linear_blocks(n);
    const float shift = tau * logf(-gamma0 / gamma1);
    {
        QG_TIMED("decode_linear_bwd", s);
        k_decode_linear_bwd<<<(unsigned)nb, kLinBlock, 0, s>>>(n, ld, latents, dm, D, pos_pre, gate_logit, gate_noise,
                                                               gamma0, gamma1, tau, shift, lambda_reg / (float)n,
                                                               grad_attrs, grad_latents, grad_pos_pre, grad_gate_logit,
                                                               (float*)ws);
        k_linear_reduce<<<(unsigned)ceil_div(dm.total_P, 4), 256, 0, s>>>((const float*)ws, nb, dm.total_P, grad_D);
    }
    QG_LAUNCH_CHECK("qg_decode_linear_bwd");
    return QG_OK;
}
