// D-SSIM term of the image loss (Eq. 3): SSIM under an 11 x 11 Gaussian window (sigma 1.5, zero padding,
// C1 = 0.01^2, C2 = 0.03^2), its mean over pixels and channels, and the gradient of weight * (1 - mean SSIM)
// with respect to the rendered image.
//
// Forward (k_ssim_fwd): a block owns a 32 x 32 tile of one channel.  It stages x and y with a 5-pixel halo in
// LDS (zero outside the image), runs the window's horizontal pass for the four moments (x, y, x^2 + y^2, xy)
// over the halo rows (a thread makes 4 adjacent columns from 16 staged values read as four 16-byte words),
// then the vertical pass (a thread makes 4 rows of one column from the 14 staged rows they read).  From mu_x,
// mu_y, E[x^2] + E[y^2] and E[xy] it forms SSIM and the per-pixel partials of the loss with respect to mu_x,
// E[x^2] and E[xy]:
//   dS/dmu_x = 2 mu_y (A2 - A1) / (B1 B2) - 2 mu_x S (1/B1 - 1/B2),  dS/dE[x^2] = -S / B2,
//   dS/dE[xy] = 2 A1 / (B1 B2),
// with A1 = 2 mu_x mu_y + C1, A2 = 2 sigma_xy + C2, B1 = mu_x^2 + mu_y^2 + C1, B2 = sigma_x^2 + sigma_y^2 + C2.
// Backward (k_ssim_bwd): each moment is a zero-padded correlation with the symmetric window, so its adjoint
// blurs the partial maps with the same window; dL/dx = blur(P_mu) + 2 x blur(P_xx) + y blur(P_xy).
#include <cmath>

#include "qg_internal.h"

namespace qg {
namespace {

constexpr int kSR = 5;             // window radius (11 taps)
constexpr int kSW = 2 * kSR + 1;
constexpr int kSTW = 32, kSTH = 32;  // output tile
constexpr int kSIW = kSTW + 2 * kSR, kSIH = kSTH + 2 * kSR;  // staged input tile (42 x 42)
constexpr int kSIWP = 44;          // staged row stride: a multiple of 4 floats, for 16-byte LDS reads
constexpr int kThreads = 256;
constexpr int kStageIters = (kSIH * kSIW + kThreads - 1) / kThreads;
constexpr int kQuads = kSTW / 4;   // horizontal pass: one thread makes 4 adjacent columns of a staged row
constexpr int kRowsPT = kSTH / (kThreads / kSTW);  // vertical pass: one thread makes 4 rows of a column
constexpr int kVRows = kRowsPT + kSW - 1;          // staged rows those 4 outputs read
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;
static_assert(kRowsPT == 4 && kSTW % 4 == 0 && kSIWP >= 4 * kQuads + 4 * 3, "tile shape");

struct Taps {
    float g[kSW];
};

// Stage n planes of a tile with halo into s[n][kSIH][kSIWP] (zero outside the image).  All loads are issued
// before the first LDS store, so the block waits on one memory latency rather than one per row of threads.
template <int N>
__device__ __forceinline__ void stage(const float* const (&src)[N], float (*s)[kSIH][kSIWP], int x0, int y0, int W,
                                      int H) {
    float v[kStageIters][N];
#pragma unroll
    for (int j = 0; j < kStageIters; ++j) {
        const int i = threadIdx.x + kThreads * j;
        const int r = i / kSIW, c = i % kSIW;
        const int x = x0 - kSR + c, y = y0 - kSR + r;
        const bool in = i < kSIH * kSIW && x >= 0 && x < W && y >= 0 && y < H;
        const uint32_t o = in ? (uint32_t)(y * W + x) : 0u;  // a plane holds fewer than 2^31 pixels
#pragma unroll
        for (int k = 0; k < N; ++k) v[j][k] = in ? src[k][o] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kStageIters; ++j) {
        const int i = threadIdx.x + kThreads * j;
        if (i < kSIH * kSIW) {
            const int r = i / kSIW, c = i % kSIW;
#pragma unroll
            for (int k = 0; k < N; ++k) s[k][r][c] = v[j][k];
        }
    }
}

// 16 consecutive staged values of row r from column c0 (a multiple of 4); the window of output column
// c0 + o reads entries o .. o + 10.
__device__ __forceinline__ void row16(const float (*row)[kSIWP], int r, int c0, float (&x)[16]) {
    const float4* p = reinterpret_cast<const float4*>(&row[r][c0]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float4 q = p[j];
        x[4 * j] = q.x;
        x[4 * j + 1] = q.y;
        x[4 * j + 2] = q.z;
        x[4 * j + 3] = q.w;
    }
}

__device__ __forceinline__ void store4(float* p, const float (&v)[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}

__global__ __launch_bounds__(kThreads) void k_ssim_fwd(int C, int H, int W, const float* __restrict__ img,
                                                       const float* __restrict__ gt, Taps t, float dscale,
                                                       float* __restrict__ pmu, float* __restrict__ pxx,
                                                       float* __restrict__ pxy, double* __restrict__ part) {
    __shared__ __align__(16) float s_in[2][kSIH][kSIWP];
    // SSIM needs E[x^2] and E[y^2] only as their sum (sigma_x^2 + sigma_y^2 in B2), so four moments are blurred
    __shared__ __align__(16) float s_h[4][kSIH][kSTW];
    __shared__ double s_red[kThreads / 64];
    const int gx = (W + kSTW - 1) / kSTW;
    const int tile = blockIdx.x, ch = blockIdx.y;
    const int x0 = (tile % gx) * kSTW, y0 = (tile / gx) * kSTH;
    const size_t plane = (size_t)H * W, base = (size_t)ch * plane;
    const float* const src[2] = {img + base, gt + base};
    stage<2>(src, s_in, x0, y0, W, H);
    __syncthreads();
    // horizontal pass over all staged rows, output columns only
    for (int i = threadIdx.x; i < kSIH * kQuads; i += kThreads) {
        const int r = i / kQuads, c0 = (i % kQuads) * 4;
        float x[16], y[16];
        row16(s_in[0], r, c0, x);
        row16(s_in[1], r, c0, y);
        float a[4] = {}, b[4] = {}, sq[4] = {}, ab[4] = {};
#pragma unroll
        for (int k = 0; k < kSW; ++k) {
            const float w = t.g[k];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const float xv = x[o + k], yv = y[o + k];
                a[o] = __builtin_fmaf(w, xv, a[o]);
                b[o] = __builtin_fmaf(w, yv, b[o]);
                sq[o] = __builtin_fmaf(w, __builtin_fmaf(xv, xv, yv * yv), sq[o]);
                ab[o] = __builtin_fmaf(w, xv * yv, ab[o]);
            }
        }
        store4(&s_h[0][r][c0], a);
        store4(&s_h[1][r][c0], b);
        store4(&s_h[2][r][c0], sq);
        store4(&s_h[3][r][c0], ab);
    }
    __syncthreads();
    // vertical pass: column c, output rows r0 .. r0 + 3 from staged rows r0 .. r0 + 13
    const int c = threadIdx.x % kSTW, r0 = (threadIdx.x / kSTW) * kRowsPT;
    float m[kRowsPT][4] = {};
#pragma unroll
    for (int j = 0; j < kVRows; ++j) {
        float h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = s_h[q][r0 + j][c];
#pragma unroll
        for (int o = 0; o < kRowsPT; ++o) {
            const int k = j - o;
            if (k >= 0 && k < kSW) {
#pragma unroll
                for (int q = 0; q < 4; ++q) m[o][q] = __builtin_fmaf(t.g[k], h[q], m[o][q]);
            }
        }
    }
    double sv = 0.0;
    const int x = x0 + c;
#pragma unroll
    for (int o = 0; o < kRowsPT; ++o) {
        const int y = y0 + r0 + o;
        if (x >= W || y >= H) continue;
        const float mx = m[o][0], my = m[o][1];
        const float sxy = m[o][3] - mx * my;
        const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
        const float B1 = mx * mx + my * my + kC1, B2 = (m[o][2] - (mx * mx + my * my)) + kC2;
        // one division: 1/B1 = B2 iD, 1/B2 = B1 iD
        const float iD = 1.f / (B1 * B2);
        const float S = A1 * A2 * iD;
        sv += (double)S;
        if (pmu) {
            const size_t off = base + (size_t)y * W + x;
            // dL/dS = -dscale (dscale = weight / (C H W))
            pmu[off] = -dscale * (2.f * my * (A2 - A1) * iD - 2.f * mx * S * ((B2 - B1) * iD));
            pxx[off] = dscale * (S * (B1 * iD));
            pxy[off] = -dscale * (2.f * A1 * iD);
        }
    }
    // block sum of SSIM (fixed order)
    for (int o = 32; o >= 1; o >>= 1) sv += __shfl_xor(sv, o);
    if (__lane_id() == 0) s_red[threadIdx.x / 64] = sv;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(size_t)ch * gridDim.x + tile] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

__global__ __launch_bounds__(kThreads) void k_ssim_bwd(int C, int H, int W, const float* __restrict__ img,
                                                       const float* __restrict__ gt, Taps t,
                                                       const float* __restrict__ pmu, const float* __restrict__ pxx,
                                                       const float* __restrict__ pxy, float* __restrict__ grad) {
    __shared__ __align__(16) float s_in[3][kSIH][kSIWP];
    __shared__ __align__(16) float s_h[3][kSIH][kSTW];
    const int gx = (W + kSTW - 1) / kSTW;
    const int tile = blockIdx.x, ch = blockIdx.y;
    const int x0 = (tile % gx) * kSTW, y0 = (tile / gx) * kSTH;
    const size_t plane = (size_t)H * W, base = (size_t)ch * plane;
    const float* const src[3] = {pmu + base, pxx + base, pxy + base};
    stage<3>(src, s_in, x0, y0, W, H);
    __syncthreads();
    for (int i = threadIdx.x; i < kSIH * kQuads; i += kThreads) {
        const int r = i / kQuads, c0 = (i % kQuads) * 4;
        float u[16], v[16], z[16];
        row16(s_in[0], r, c0, u);
        row16(s_in[1], r, c0, v);
        row16(s_in[2], r, c0, z);
        float a[4] = {}, b[4] = {}, d[4] = {};
#pragma unroll
        for (int k = 0; k < kSW; ++k) {
            const float w = t.g[k];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                a[o] = __builtin_fmaf(w, u[o + k], a[o]);
                b[o] = __builtin_fmaf(w, v[o + k], b[o]);
                d[o] = __builtin_fmaf(w, z[o + k], d[o]);
            }
        }
        store4(&s_h[0][r][c0], a);
        store4(&s_h[1][r][c0], b);
        store4(&s_h[2][r][c0], d);
    }
    __syncthreads();
    const int c = threadIdx.x % kSTW, r0 = (threadIdx.x / kSTW) * kRowsPT;
    float m[kRowsPT][3] = {};
#pragma unroll
    for (int j = 0; j < kVRows; ++j) {
        float h[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) h[q] = s_h[q][r0 + j][c];
#pragma unroll
        for (int o = 0; o < kRowsPT; ++o) {
            const int k = j - o;
            if (k >= 0 && k < kSW) {
#pragma unroll
                for (int q = 0; q < 3; ++q) m[o][q] = __builtin_fmaf(t.g[k], h[q], m[o][q]);
            }
        }
    }
    const int x = x0 + c;
#pragma unroll
    for (int o = 0; o < kRowsPT; ++o) {
        const int y = y0 + r0 + o;
        if (x >= W || y >= H) continue;
        const size_t off = base + (size_t)y * W + x;
        grad[off] += m[o][0] + 2.f * img[off] * m[o][1] + gt[off] * m[o][2];
    }
}

// out[0] = 1 - (sum of the block sums) / count, in a fixed order: thread t adds parts t, t + 256, ... in turn,
// then a pairwise tree over the 256 thread sums.
__global__ __launch_bounds__(256) void k_ssim_reduce(int64_t nparts, int64_t count, const double* __restrict__ part,
                                                     double* __restrict__ out) {
    __shared__ double s[256];
    double a = 0.0;
    for (int64_t k = threadIdx.x; k < nparts; k += 256) a += part[k];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 1.0 - s[0] / (double)count;
}

int64_t ssim_tiles(int H, int W) { return (int64_t)((W + kSTW - 1) / kSTW) * ((H + kSTH - 1) / kSTH); }

}  // namespace
}  // namespace qg

using namespace qg;

extern "C" size_t qg_ssim_workspace_size(int32_t C, int32_t H, int32_t W) {
    if (C < 1 || H < 1 || W < 1) return 0;
    const size_t n = (size_t)C * H * W;
    return 3 * align_up(n * sizeof(float)) + align_up((size_t)C * ssim_tiles(H, W) * sizeof(double));
}

extern "C" qg_status qg_ssim_loss(int32_t C, int32_t H, int32_t W, const float* image, const float* gt, float weight,
                                  float* grad_image, double* dssim_out, void* ws, size_t ws_bytes,
                                  qg_stream stream) {
    clear_error();
    QG_REQUIRE(C >= 1 && C <= 65535 && H >= 1 && W >= 1, "C=%d H=%d W=%d invalid", C, H, W);
    QG_REQUIRE(image && gt, "image/gt NULL");
    QG_REQUIRE(grad_image || dssim_out, "nothing to compute: grad_image and dssim_out are both NULL");
    const size_t need = qg_ssim_workspace_size(C, H, W);
    QG_REQUIRE(ws && ws_bytes >= need, "workspace too small: %zu < %zu", ws_bytes, need);
    const int64_t ntiles = ssim_tiles(H, W);
    QG_REQUIRE((int64_t)H * W < (1ll << 31), "image too large: H*W=%lld", (long long)H * W);
    hipStream_t s = (hipStream_t)stream;
    Taps t;
    {
        double g[kSW], sum = 0.0;
        for (int k = 0; k < kSW; ++k) {
            const double d = (double)(k - kSR);
            g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
            sum += g[k];
        }
        for (int k = 0; k < kSW; ++k) t.g[k] = (float)(g[k] / sum);
    }
    const size_t n = (size_t)C * H * W;
    float* pmu = (float*)ws;
    float* pxx = (float*)((char*)ws + align_up(n * sizeof(float)));
    float* pxy = (float*)((char*)ws + 2 * align_up(n * sizeof(float)));
    double* part = (double*)((char*)ws + 3 * align_up(n * sizeof(float)));
    const float dscale = (float)((double)weight / (double)n);
    const dim3 grid((unsigned)ntiles, (unsigned)C);
    {
        QG_TIMED("ssim", s);
        k_ssim_fwd<<<grid, 256, 0, s>>>(C, H, W, image, gt, t, dscale, grad_image ? pmu : nullptr, pxx, pxy, part);
        if (grad_image) k_ssim_bwd<<<grid, 256, 0, s>>>(C, H, W, image, gt, t, pmu, pxx, pxy, grad_image);
        if (dssim_out) k_ssim_reduce<<<1, 256, 0, s>>>((int64_t)C * ntiles, (int64_t)n, part, dssim_out);
    }
    QG_LAUNCH_CHECK("qg_ssim_loss");
    return QG_OK;
}
