// The residual decoder's dense products (Eq. 5: r = W2 SiLU(W1 l)) and their backward on FP32 matrix
// cores, one wave per group of 16 Gaussians.  Shared by the standalone decode kernels and the fused
// decode+projection kernels.  Internal to libqg.
//
// MFMA layout (v_mfma_f32_16x16x4f32, wave64): lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// accumulates D[4*(l/16)+i][l%16], i = 0..3.  With q = l/16 and c = l%16:
//   "layout T": register i holds (feature 16b + 4q + i, Gaussian c)
//   "layout N": register i holds (Gaussian 4q + i, feature 16b + c)
// Every product is oriented so that the output registers of one are directly the B operand of the next:
// contraction step i takes the features (or Gaussians) {i, 4+i, 8+i, 12+i} of a 16-block, and the
// constant operand is loaded in that permuted order.
#pragma once

#include "qg_internal.h"

namespace qg {
namespace dec {

constexpr int kL = 8;    // latent width
constexpr int kH = 32;   // hidden width
constexpr int kM = 56;   // outputs: rotation 4, log-scale 3, opacity logit 1, SH 48 (planes 3..58)
constexpr int kMB = 4;   // 56 outputs padded to 4 blocks of 16
constexpr int kGroup = 16;
constexpr int kWidth = kH * kL + kM * kH;  // 2048 weight-gradient entries: W1 [32][8] then W2 [56][32]

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float sigm(float x) { return __builtin_amdgcn_rcpf(1.f + expf(-x)); }
__device__ __forceinline__ float silu(float x) { return x * sigm(x); }
__device__ __forceinline__ float silu_grad(float x) {
    const float s = sigm(x);
    return s * (1.f + x * (1.f - s));
}

// ---- forward ------------------------------------------------------------------------------------
struct FwdOps {
    float aW1[2][2];     // A of pre^T = W1 L^T: (j = 16jb + c, k = 4ks + q)
    float aW2[kMB][2][4];  // A of R^T = W2 H^T, step (jb, i): (m = 16mb + c, j = 16jb + 4q + i)
};

__device__ __forceinline__ void load_fwd_ops(const float* __restrict__ W1, const float* __restrict__ W2, FwdOps& o) {
    const int lane = __lane_id(), q = lane / 16, c = lane % 16;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) o.aW1[jb][ks] = W1[(16 * jb + c) * kL + 4 * ks + q];
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 16 * mb + c;
                o.aW2[mb][jb][i] = m < kM ? W2[m * kH + 16 * jb + 4 * q + i] : 0.f;
            }
}

// Residuals of 16 Gaussians.  lat(k) returns the rounded latent k of Gaussian c (this lane's column);
// out(m, i_of_m, value) receives R[m][Gaussian c] for m = 16mb + 4q + i < 56.
template <class Lat, class Out>
__device__ __forceinline__ void decode_group_fwd(const FwdOps& o, const Lat& lat, const Out& out) {
    const int lane = __lane_id(), q = lane / 16;
    f4 pre[2];
    const float b0 = lat(q), b1 = lat(4 + q);
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(o.aW1[jb][0], b0, acc);
        acc = mfma(o.aW1[jb][1], b1, acc);
        pre[jb] = acc;
    }
    f4 R[kMB];
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb) R[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float h = silu(pre[jb][i]);
#pragma unroll
            for (int mb = 0; mb < kMB; ++mb) R[mb] = mfma(o.aW2[mb][jb][i], h, R[mb]);
        }
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 16 * mb + 4 * q + i;
            if (m < kM) out(m, R[mb][i]);
        }
}

// ---- backward -----------------------------------------------------------------------------------
struct BwdOps {
    float bW1[2][2];   // B of pre = L W1^T: (k = 4ks + q, j = 16jb + c)
    float bW2[14][2];  // B of dH = dR W2: (m = 4ks + q, j = 16jb + c)
    float aW1T[8];     // A of dL^T = W1^T dpre^T: (k = c, j = 4ks + q)
};

__device__ __forceinline__ void load_bwd_ops(const float* __restrict__ W1, const float* __restrict__ W2, BwdOps& o) {
    const int lane = __lane_id(), q = lane / 16, c = lane % 16;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) o.bW1[jb][ks] = W1[(16 * jb + c) * kL + 4 * ks + q];
#pragma unroll
    for (int ks = 0; ks < 14; ++ks)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) o.bW2[ks][jb] = W2[(4 * ks + q) * kH + 16 * jb + c];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) o.aW1T[ks] = c < kL ? W1[(4 * ks + q) * kL + c] : 0.f;
}

// A 16 x 33 LDS array as the transpose buffer of decode_group_bwd.
struct TransposeBuf {
    float (*t)[33];
    __device__ __forceinline__ float& operator()(int r, int j) const { return t[r][j]; }
};

struct BwdAcc {
    f4 W2[kMB][2];  // dW2[16mb + 4q + i][16jb + c]
    f4 W1[2];       // dW1^T[4q + i][16jb + c] (rows < 8 used)
};

__device__ __forceinline__ void zero_acc(BwdAcc& a) {
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb) a.W2[mb][0] = a.W2[mb][1] = f4{0.f, 0.f, 0.f, 0.f};
    a.W1[0] = a.W1[1] = f4{0.f, 0.f, 0.f, 0.f};
}

// Backward of 16 Gaussians (columns/rows as in the layouts above), in two halves so that a caller can run
// the first half of several groups before the second half of any (one LDS barrier between them instead of
// one per group, and the groups' dL chains interleave).
//   latA(k):   rounded latent k of Gaussian c                (row layout of pre = L W1^T)
//   latN(k, i):rounded latent k of Gaussian 4q + i           (A of dW1^T += L^T dpre)
//   drA(m):    dL/dr_m of Gaussian c                         (A of dH = dR W2), m = 4ks + q
//   drN(m, i): dL/dr_m of Gaussian 4q + i                    (A of dW2 += dR^T H), m = 16mb + c (0 if >= 56)
//   dlat(k, v):receives dL/dlatent_k of Gaussian c for k = 4q + i < 8 (lanes q < 2)
// tb(r, j): a float& to LDS owned by this wave, r < 16, j < 32 (transpose of dpre); it is written only after
// every drA/drN/latN read of the group, so it may alias their storage.
// First half: the weight-gradient products into acc and dpre^T into tb.
template <class LatA, class LatN, class DrA, class DrN, class TB>
__device__ __forceinline__ void decode_group_bwd_a(const BwdOps& o, BwdAcc& acc, const LatA& latA, const LatN& latN,
                                                   const DrA& drA, const DrN& drN, const TB& tb) {
    const int lane = __lane_id(), q = lane / 16, c = lane % 16;
    // pre (layout N)
    f4 pre[2];
    {
        const float a0 = latA(q), a1 = latA(4 + q);
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            f4 t = {0.f, 0.f, 0.f, 0.f};
            t = mfma(a0, o.bW1[jb][0], t);
            t = mfma(a1, o.bW1[jb][1], t);
            pre[jb] = t;
        }
    }
    // dH = dR W2 (layout N)
    f4 dH[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int ks = 0; ks < 14; ++ks) {
        const float a = drA(4 * ks + q);
        dH[0] = mfma(a, o.bW2[ks][0], dH[0]);
        dH[1] = mfma(a, o.bW2[ks][1], dH[1]);
    }
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
#pragma unroll
        for (int mb = 0; mb < kMB; ++mb) {
            const float a = drN(16 * mb + c, i);
            acc.W2[mb][0] = mfma(a, H[0][i], acc.W2[mb][0]);
            acc.W2[mb][1] = mfma(a, H[1][i], acc.W2[mb][1]);
        }
        const float al = c < kL ? latN(c, i) : 0.f;
        acc.W1[0] = mfma(al, dP[0][i], acc.W1[0]);
        acc.W1[1] = mfma(al, dP[1][i], acc.W1[1]);
    }
    // dpre transposed to (feature 4ks + q, Gaussian c) through LDS
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int i = 0; i < 4; ++i) tb(4 * q + i, 16 * jb + c) = dP[jb][i];
}

// Second half (after an LDS barrier of the wave): dL^T = W1^T dpre^T from tb.
template <class DLat, class TB>
__device__ __forceinline__ void decode_group_bwd_b(const BwdOps& o, const DLat& dlat, const TB& tb) {
    const int lane = __lane_id(), q = lane / 16, c = lane % 16;
    f4 dL = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) dL = mfma(o.aW1T[ks], tb(c, 4 * ks + q), dL);
    if (q < 2) {
#pragma unroll
        for (int i = 0; i < 4; ++i) dlat(4 * q + i, dL[i]);
    }
}

__device__ __forceinline__ void wave_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Both halves for one group.
template <class LatA, class LatN, class DrA, class DrN, class DLat, class TB>
__device__ __forceinline__ void decode_group_bwd(const BwdOps& o, BwdAcc& acc, const LatA& latA, const LatN& latN,
                                                 const DrA& drA, const DrN& drN, const DLat& dlat, const TB& tb) {
    decode_group_bwd_a(o, acc, latA, latN, drA, drN, tb);
    wave_lds_barrier();
    decode_group_bwd_b(o, dlat, tb);
    wave_lds_barrier();
}

// Adds this wave's accumulators into a block buffer sw[2048] (W1 [32][8] then W2 [56][32]); the caller
// serialises the waves (fixed order) around this call.
__device__ __forceinline__ void add_acc(const BwdAcc& acc, float* sw) {
    const int lane = __lane_id(), q = lane / 16, c = lane % 16;
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 16 * mb + 4 * q + i;
                if (m < kM) sw[kH * kL + m * kH + 16 * jb + c] += acc.W2[mb][jb][i];
            }
    if (q < 2) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) sw[(16 * jb + c) * kL + 4 * q + i] += acc.W1[jb][i];
    }
}

// Writes this wave's accumulators to its own row dst[2048] (every element exactly once, by one lane).
__device__ __forceinline__ void store_acc(const BwdAcc& acc, float* __restrict__ dst) {
    const int lane = __lane_id(), q = lane / 16, c = lane % 16;
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 16 * mb + 4 * q + i;
                if (m < kM) dst[kH * kL + m * kH + 16 * jb + c] = acc.W2[mb][jb][i];
            }
    if (q < 2) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) dst[(16 * jb + c) * kL + 4 * q + i] = acc.W1[jb][i];
    }
}

// As add_acc, for a buffer shared by the waves of a block (LDS float atomics; no ordering needed).
__device__ __forceinline__ void add_acc_atomic(const BwdAcc& acc, float* sw) {
    const int lane = __lane_id(), q = lane / 16, c = lane % 16;
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 16 * mb + 4 * q + i;
                if (m < kM) atomicAdd(&sw[kH * kL + m * kH + 16 * jb + c], acc.W2[mb][jb][i]);
            }
    if (q < 2) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) atomicAdd(&sw[(16 * jb + c) * kL + 4 * q + i], acc.W1[jb][i]);
    }
}

// Gate of Eq. 6-7.
__device__ __forceinline__ float gate_of(float a, float g0, float g1, float tau, float* gh_out, float* gt_out) {
    const float gh = sigm(a / tau);
    const float gt = gh * (g1 - g0) + g0;
    if (gh_out) *gh_out = gh;
    if (gt_out) *gt_out = gt;
    return fminf(1.f, fmaxf(0.f, gt));
}

}  // namespace dec
}  // namespace qg
