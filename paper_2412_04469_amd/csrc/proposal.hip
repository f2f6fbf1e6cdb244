// Learned residual proposal: a 24 -> 64 -> 64 -> 12 SiLU MLP per Gaussian on BF16 matrix cores
// (v_mfma_f32_16x16x16bf16_1k) with FP32 accumulation, its backward, and its input features.
//
// One wave handles 16 Gaussians at a time.  With q = lane/16 and c = lane%16, the MFMA takes
// A[c][4q+j] and B[4q+j][c] (j = 0..3, four bf16 per lane) and returns D[4q+i][c] (i = 0..3).  Activations
// are kept as (feature, Gaussian) tiles with the Gaussian on c, so the D registers of one layer
// (feature 16b + 4q + i, Gaussian c) are exactly the B operand of the next layer's K-block b: the forward
// never leaves registers.  In the backward the output gradient and dL/d pre-activation tiles are again B
// operands of the transposed weights; the weight gradients contract over Gaussians, so the tiles they need
// are staged through a per-wave LDS area as [row][16 Gaussians] bf16 and read back with the Gaussian on k.
//
// Rounding points (matching the definition of the operands): every matrix operand is rounded to bf16
// from float32, round to nearest even -- the weights, the standardised features, SiLU outputs, the
// output gradient and both dL/d pre-activation tiles; biases, pre-activations and the elementwise
// SiLU-derivative factors stay float32.
#include <cmath>

#include "qg_internal.h"

namespace qg {
namespace {

constexpr int kIn = 24, kHid = 64, kOut = 12;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
              kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kOut * kHid, kParams = kOffB3 + kOut;
static_assert(kParams == QG_PROPOSAL_PARAMS, "parameter layout");

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (short)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(short b) { return __uint_as_float(((uint32_t)(uint16_t)b) << 16); }
__device__ __forceinline__ f4 mma(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
__device__ __forceinline__ float sigm(float x) { return 1.f / (1.f + expf(-x)); }
__device__ __forceinline__ float silu(float x) { return x * sigm(x); }
__device__ __forceinline__ float silu_grad(float x) {
    const float s = sigm(x);
    return s * (1.f + x * (1.f - s));
}

struct Stats {  // [24 in_mean | 24 in_rstd | 12 out_mean | 12 out_std]
    const float* p;
    __device__ float in_mean(int f) const { return p[f]; }
    __device__ float in_rstd(int f) const { return p[kIn + f]; }
    __device__ float out_mean(int o) const { return p[2 * kIn + o]; }
    __device__ float out_std(int o) const { return p[2 * kIn + kOut + o]; }
};

// Forward operands of one wave: weights as A operands (rows on c, k on 4q + j), biases in D layout.
struct FwdW {
    s4 a1[4][2], a2[4][4], a3[4];
    f4 b1[4], b2[4], b3;
};

__device__ __forceinline__ void load_fwd(const float* __restrict__ P, FwdW& w) {
    const int lane = __lane_id(), q = lane / 16, c = lane % 16;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * kb + 4 * q + j;
                w.a1[mb][kb][j] = k < kIn ? bf16(P[kOffW1 + (16 * mb + c) * kIn + k]) : (short)0;
            }
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int j = 0; j < 4; ++j) w.a2[mb][kb][j] = bf16(P[kOffW2 + (16 * mb + c) * kHid + 16 * kb + 4 * q + j]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            w.b1[mb][i] = P[kOffB1 + 16 * mb + 4 * q + i];
            w.b2[mb][i] = P[kOffB2 + 16 * mb + 4 * q + i];
        }
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) w.a3[kb][j] = c < kOut ? bf16(P[kOffW3 + c * kHid + 16 * kb + 4 * q + j]) : (short)0;
#pragma unroll
    for (int i = 0; i < 4; ++i) w.b3[i] = 4 * q + i < kOut ? P[kOffB3 + 4 * q + i] : 0.f;
}

struct Acts {
    s4 x[2];          // standardised features, B operand (feature 16kb + 4q + j, Gaussian c)
    f4 pre1[4], pre2[4];
    s4 h1[4], h2[4];  // B operands of the next layer
    f4 ys;            // standardised outputs (output 4q + i, Gaussian c)
};

// x_at(f) returns raw feature f (< 24) of this lane's Gaussian, or is not called for invalid lanes.
template <class X>
__device__ __forceinline__ void mlp_forward(const FwdW& w, const Stats& st, bool valid, const X& x_at, Acts& a) {
    const int lane = __lane_id(), q = lane / 16;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int f = 16 * kb + 4 * q + j;
            a.x[kb][j] = (valid && f < kIn) ? bf16((x_at(f) - st.in_mean(f)) * st.in_rstd(f)) : (short)0;
        }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        f4 acc = w.b1[mb];
        acc = mma(w.a1[mb][0], a.x[0], acc);
        acc = mma(w.a1[mb][1], a.x[1], acc);
        a.pre1[mb] = acc;
#pragma unroll
        for (int i = 0; i < 4; ++i) a.h1[mb][i] = bf16(silu(acc[i]));
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        f4 acc = w.b2[mb];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mma(w.a2[mb][kb], a.h1[kb], acc);
        a.pre2[mb] = acc;
#pragma unroll
        for (int i = 0; i < 4; ++i) a.h2[mb][i] = bf16(silu(acc[i]));
    }
    f4 acc = w.b3;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = mma(w.a3[kb], a.h2[kb], acc);
    a.ys = acc;
}

__global__ __launch_bounds__(256) void k_proposal_fwd(int64_t n, int64_t ld_in, const float* __restrict__ feat,
                                                      const float* __restrict__ P, const float* __restrict__ stats,
                                                      float* __restrict__ out, int64_t ld_out) {
    FwdW w;
    load_fwd(P, w);
    const Stats st{stats};
    const int lane = threadIdx.x % 64, q = lane / 16, c = lane % 16;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    const int64_t groups = ceil_div(n, 16);
    for (int64_t g = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; g < groups; g += waves) {
        const int64_t col = 16 * g + c;
        const bool valid = col < n;
        Acts a;
        mlp_forward(w, st, valid, [&](int f) { return feat[(int64_t)f * ld_in + col]; }, a);
        if (valid) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = 4 * q + i;
                if (o < kOut) out[(int64_t)o * ld_out + col] = a.ys[i] * st.out_std(o) + st.out_mean(o);
            }
        }
    }
}

// ---- backward ---------------------------------------------------------------------------------------
struct BwdW {
    s4 a3t[4];     // W3^T (rows 16mb + c = hidden, k = output 4q + j)
    s4 a2t[4][4];  // W2^T (rows 16mb + c = hidden-1 unit, k = hidden-2 unit 16kb + 4q + j)
};

__device__ __forceinline__ void load_bwd(const float* __restrict__ P, BwdW& w) {
    const int lane = __lane_id(), q = lane / 16, c = lane % 16;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = 4 * q + j;
            w.a3t[mb][j] = o < kOut ? bf16(P[kOffW3 + o * kHid + 16 * mb + c]) : (short)0;
        }
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int j = 0; j < 4; ++j) w.a2t[mb][kb][j] = bf16(P[kOffW2 + (16 * kb + 4 * q + j) * kHid + 16 * mb + c]);
    }
}

// Per-wave LDS tiles, [row][16 Gaussians] bf16.
struct Tiles {
    short x[32][16], h1[64][16], h2[64][16], dy[16][16], dp2[64][16], dp1[64][16];
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile row r, Gaussians 4q .. 4q + 3 as an operand with k on the Gaussian.
__device__ __forceinline__ s4 tile_k(const short (*t)[16], int r, int q) {
    return *reinterpret_cast<const s4*>(&t[r][4 * q]);
}

constexpr int kBwdWaves = 1024;  // maximum waves (partial slots) of one backward call
constexpr int kPartial = kParams + 1;  // per-wave gradient partials + loss

__global__ __launch_bounds__(256) void k_proposal_bwd(int64_t m, const uint32_t* __restrict__ idx, int64_t n, int64_t ld,
                                                      const float* __restrict__ feat, const float* __restrict__ tgt,
                                                      const float* __restrict__ P, const float* __restrict__ stats,
                                                      float* __restrict__ partial) {
    __shared__ Tiles s_t[4];
    const int wv = threadIdx.x / 64;
    Tiles& T = s_t[wv];
    FwdW w;
    load_fwd(P, w);
    BwdW wb;
    load_bwd(P, wb);
    const Stats st{stats};
    const int lane = threadIdx.x % 64, q = lane / 16, c = lane % 16;
    const float inv_m = 1.f / (float)m;
    f4 gW2[4][4], gW1[4][2], gW3[4], gb1[4], gb2[4], gb3;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = f4{0.f, 0.f, 0.f, 0.f};
        gW1[a][0] = gW1[a][1] = gW3[a] = gb1[a] = gb2[a] = f4{0.f, 0.f, 0.f, 0.f};
    }
    gb3 = f4{0.f, 0.f, 0.f, 0.f};
    float loss = 0.f;
    const int64_t waves = (int64_t)gridDim.x * 4;
    const int64_t wave_id = (int64_t)blockIdx.x * 4 + wv;
    const int64_t groups = ceil_div(m, 16);
    for (int64_t g = wave_id; g < groups; g += waves) {
        const int64_t s = 16 * g + c;
        int64_t col = s < m ? (idx ? (int64_t)idx[s] : s) : 0;
        const bool valid = s < m && col < n;  // an index past n is skipped, not read
        col = valid ? col : 0;
        Acts a;
        mlp_forward(w, st, valid, [&](int f) { return feat[(int64_t)f * ld + col]; }, a);
        // output gradient of L = (1/m) sum (y_s - t_s)^2 (output 4q + i, Gaussian c)
        f4 dy;
        s4 dyb;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = 4 * q + i;
            float d = 0.f;
            if (valid && o < kOut) {
                const float e = a.ys[i] - (tgt[(int64_t)o * ld + col] - st.out_mean(o)) / st.out_std(o);
                loss = __builtin_fmaf(e, e, loss);
                d = 2.f * e * inv_m;
            }
            dy[i] = d;
            dyb[i] = bf16(d);
        }
        gb3 += dy;
        // dL/d pre2 = (W3^T dy) * SiLU'(pre2)
        s4 dp2b[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const f4 dh = mma(wb.a3t[mb], dyb, f4{0.f, 0.f, 0.f, 0.f});
            f4 dp;
#pragma unroll
            for (int i = 0; i < 4; ++i) dp[i] = dh[i] * silu_grad(a.pre2[mb][i]);
            gb2[mb] += dp;
#pragma unroll
            for (int i = 0; i < 4; ++i) dp2b[mb][i] = bf16(dp[i]);
        }
        // dL/d pre1 = (W2^T dpre2) * SiLU'(pre1)
        s4 dp1b[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            f4 dh = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) dh = mma(wb.a2t[mb][kb], dp2b[kb], dh);
            f4 dp;
#pragma unroll
            for (int i = 0; i < 4; ++i) dp[i] = dh[i] * silu_grad(a.pre1[mb][i]);
            gb1[mb] += dp;
#pragma unroll
            for (int i = 0; i < 4; ++i) dp1b[mb][i] = bf16(dp[i]);
        }
        // stage the (row, Gaussian) tiles; the weight gradients contract over Gaussians
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) T.x[16 * kb + 4 * q + i][c] = a.x[kb][i];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                T.h1[16 * mb + 4 * q + i][c] = a.h1[mb][i];
                T.h2[16 * mb + 4 * q + i][c] = a.h2[mb][i];
                T.dp2[16 * mb + 4 * q + i][c] = dp2b[mb][i];
                T.dp1[16 * mb + 4 * q + i][c] = dp1b[mb][i];
            }
            T.dy[4 * q + i][c] = dyb[i];
        }
        wave_sync();
        // dW3[o][f] += dy[o][G] h2[f][G]; dW2[f2][f1] += dp2[f2][G] h1[f1][G]; dW1[f1][x] += dp1[f1][G] x[x][G]
        const s4 ady = tile_k(T.dy, c, q);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) gW3[nb] = mma(ady, tile_k(T.h2, 16 * nb + c, q), gW3[nb]);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const s4 adp2 = tile_k(T.dp2, 16 * mb + c, q);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) gW2[mb][nb] = mma(adp2, tile_k(T.h1, 16 * nb + c, q), gW2[mb][nb]);
            const s4 adp1 = tile_k(T.dp1, 16 * mb + c, q);
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) gW1[mb][nb] = mma(adp1, tile_k(T.x, 16 * nb + c, q), gW1[mb][nb]);
        }
        wave_sync();
    }
    // bias gradients: sum the 16 Gaussian columns of each row (through LDS, reusing the dp2 tile as floats)
    float* red = reinterpret_cast<float*>(&T.dp2[0][0]);  // 64 rows x 16 floats fit in dp2 + dp1 (4 KB)
    float* out = partial + wave_id * kPartial;
    auto row_sum_to = [&](const f4 (&v)[4], int nrow_blocks, int off) {
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
            if (mb < nrow_blocks)
#pragma unroll
                for (int i = 0; i < 4; ++i) red[(16 * mb + 4 * q + i) * 16 + c] = v[mb][i];
        wave_sync();
        for (int r = lane; r < 16 * nrow_blocks; r += 64) {
            float sacc = 0.f;
            for (int k = 0; k < 16; ++k) sacc += red[r * 16 + k];
            out[off + r] = sacc;
        }
        wave_sync();
    };
    row_sum_to(gb1, 4, kOffB1);
    row_sum_to(gb2, 4, kOffB2);
#pragma unroll
    for (int i = 0; i < 4; ++i) red[(4 * q + i) * 16 + c] = gb3[i];
    wave_sync();
    if (lane < kOut) {
        float sacc = 0.f;
        for (int k = 0; k < 16; ++k) sacc += red[lane * 16 + k];
        out[kOffB3 + lane] = sacc;
    }
    wave_sync();
    // weight gradients in the parameter layout (D layout: row 16mb + 4q + i, column 16nb + c)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * mb + 4 * q + i;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) out[kOffW2 + r * kHid + 16 * nb + c] = gW2[mb][nb][i];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const int xk = 16 * nb + c;
                if (xk < kIn) out[kOffW1 + r * kIn + xk] = gW1[mb][nb][i];
            }
        }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int o = 4 * q + i;
        if (o < kOut)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) out[kOffW3 + o * kHid + 16 * nb + c] = gW3[nb][i];
    }
    // wave loss
    for (int off = 32; off >= 1; off >>= 1) loss += __shfl_xor(loss, off);
    if (lane == 0) out[kParams] = loss;
}

// grad[p] += sum over waves (fixed order) of partial[w][p]; loss_out[0] = sum of the wave losses / m.
__global__ void k_proposal_reduce(const float* __restrict__ partial, int nwaves, float inv_m,
                                  float* __restrict__ grad, float* __restrict__ loss_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kParams) return;
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += partial[(int64_t)w * kPartial + p];
    if (p < kParams)
        grad[p] += s;
    else if (loss_out)
        loss_out[0] = s * inv_m;
}

__global__ void k_proposal_features(int64_t n, int64_t ld, const float* __restrict__ A1, const float* __restrict__ A2,
                                    const float* __restrict__ A3, const float* __restrict__ p,
                                    float* __restrict__ out, int64_t ld_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k * ld_out + i] = A1[k * ld + i];
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const float a1 = A1[k * ld + i], a2 = A2[k * ld + i], a3 = A3[k * ld + i];
        out[(3 + k) * ld_out + i] = a1 - a2;
        out[(13 + k) * ld_out + i] = a2 - a3;
    }
    out[23 * ld_out + i] = p[i];
}

int fwd_blocks(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, 64), 1), 2048); }
int bwd_blocks(int64_t m) { return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(m, 64), 1), kBwdWaves / 4); }

}  // namespace
}  // namespace qg

using namespace qg;

extern "C" qg_status qg_proposal_features(int64_t n, int64_t ld, const float* A1, const float* A2, const float* A3,
                                          const float* p, float* out, int64_t ld_out, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n && ld_out >= n, "n=%lld ld=%lld ld_out=%lld invalid", (long long)n, (long long)ld,
               (long long)ld_out);
    if (n == 0) return QG_OK;
    QG_REQUIRE(A1 && A2 && A3 && p && out, "a pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("proposal_features", s);
        k_proposal_features<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, ld, A1, A2, A3, p, out, ld_out);
    }
    QG_LAUNCH_CHECK("qg_proposal_features");
    return QG_OK;
}

extern "C" qg_status qg_proposal_fwd(int64_t n, int64_t ld_in, const float* features, const float* params,
                                     const float* stats, float* out, int64_t ld_out, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld_in >= n && ld_out >= n, "n=%lld ld_in=%lld ld_out=%lld invalid", (long long)n,
               (long long)ld_in, (long long)ld_out);
    if (n == 0) return QG_OK;
    QG_REQUIRE(features && params && stats && out, "a pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("proposal_fwd", s);
        k_proposal_fwd<<<fwd_blocks(n), 256, 0, s>>>(n, ld_in, features, params, stats, out, ld_out);
    }
    QG_LAUNCH_CHECK("qg_proposal_fwd");
    return QG_OK;
}

extern "C" size_t qg_proposal_bwd_workspace_size(void) { return align_up((size_t)kBwdWaves * kPartial * sizeof(float)); }

extern "C" qg_status qg_proposal_bwd(int64_t m, const uint32_t* idx, int64_t n, int64_t ld, const float* features,
                                     const float* targets, const float* params, const float* stats, float* grad,
                                     float* loss_out, void* ws, size_t ws_bytes, qg_stream stream) {
    clear_error();
    QG_REQUIRE(m >= 0 && n >= 0 && ld >= n && m < (1ll << 32), "m=%lld n=%lld ld=%lld invalid", (long long)m,
               (long long)n, (long long)ld);
    QG_REQUIRE(idx || m <= n, "without idx, m must be <= n");
    if (m == 0) return QG_OK;
    QG_REQUIRE(features && targets && params && stats && grad, "a pointer is NULL");
    QG_REQUIRE(ws && ws_bytes >= qg_proposal_bwd_workspace_size(), "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int blocks = bwd_blocks(m);
    float* partial = (float*)ws;
    {
        QG_TIMED("proposal_bwd", s);
        k_proposal_bwd<<<blocks, 256, 0, s>>>(m, idx, n, ld, features, targets, params, stats, partial);
        k_proposal_reduce<<<(unsigned)ceil_div(kParams + 1, 256), 256, 0, s>>>(partial, blocks * 4, 1.f / (float)m,
                                                                              grad, loss_out);
    }
    QG_LAUNCH_CHECK("qg_proposal_bwd");
    return QG_OK;
}
