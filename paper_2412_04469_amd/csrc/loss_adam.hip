// L1 loss with its image gradient and the clamped-image MSE used for PSNR; Adam.
#include <cmath>

#include "l1_term.h"
#include "qg_internal.h"

namespace qg {
namespace {

constexpr int kLBlock = 256;
constexpr int kLIPT = 16;
constexpr int64_t kLTile = (int64_t)kLBlock * kLIPT;

// The block's two sums (in double) to part[2b], part[2b + 1], in a fixed order.
__device__ __forceinline__ void l1_block_partials(float sa, float sb, double* s_a, double* s_b, double* part) {
    double da = sa, db = sb;
    for (int o = 32; o >= 1; o >>= 1) {
        da += __shfl_xor(da, o);
        db += __shfl_xor(db, o);
    }
    if (__lane_id() == 0) {
        s_a[threadIdx.x / kWave] = da;
        s_b[threadIdx.x / kWave] = db;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0, tb = 0;
        for (int w = 0; w < kLBlock / kWave; ++w) {
            ta += s_a[w];
            tb += s_b[w];
        }
        part[2 * blockIdx.x] = ta;
        part[2 * blockIdx.x + 1] = tb;
    }
}

// A block covers kLTile consecutive elements.  vec: every pointer is 16-byte aligned; a block lying wholly
// inside the range then moves them as float4 (thread t takes quads t, t + 256, ...).
__global__ __launch_bounds__(kLBlock) void k_l1(int64_t count, const float* __restrict__ img,
                                                const float* __restrict__ gt, float gscale,
                                                float* __restrict__ grad, double* __restrict__ part, int vec) {
    __shared__ double s_a[kLBlock / kWave], s_b[kLBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kLTile;
    float sa = 0.f, sb = 0.f;
    if (vec && base + kLTile <= count) {
        const float4* I = reinterpret_cast<const float4*>(img + base);
        const float4* T = reinterpret_cast<const float4*>(gt + base);
        float4* D = reinterpret_cast<float4*>(grad + base);
        float4 x[kLIPT / 4], y[kLIPT / 4];
#pragma unroll
        for (int r = 0; r < kLIPT / 4; ++r) {
            x[r] = I[r * kLBlock + threadIdx.x];
            y[r] = T[r * kLBlock + threadIdx.x];
        }
#pragma unroll
        for (int r = 0; r < kLIPT / 4; ++r) {
            float4 gr;
            gr.x = l1_term(x[r].x, y[r].x, gscale, sa, sb);
            gr.y = l1_term(x[r].y, y[r].y, gscale, sa, sb);
            gr.z = l1_term(x[r].z, y[r].z, gscale, sa, sb);
            gr.w = l1_term(x[r].w, y[r].w, gscale, sa, sb);
            if (grad) D[r * kLBlock + threadIdx.x] = gr;
        }
    } else {
#pragma unroll
        for (int r = 0; r < kLIPT; ++r) {
            const int64_t i = base + (int64_t)r * kLBlock + threadIdx.x;
            if (i < count) {
                const float gr = l1_term(img[i], gt[i], gscale, sa, sb);
                if (grad) grad[i] = gr;
            }
        }
    }
    l1_block_partials(sa, sb, s_a, s_b, part);
}

// As k_l1 over the elements whose pixel (index mod plane) is set in mask; the others get a zero gradient and
// add nothing to the sums.  The scale stays 1/count (the masked-iteration reading of Sec. 3.3: the loss of
// the rendered pixels at the full image's normalisation).  vec: as in k_l1, and in addition plane is a
// multiple of 4 and mask 4-byte aligned, so a float4 of elements never crosses a plane boundary and its four
// mask bytes are one aligned word (byte k for element k).  The elements are visited in k_l1's order, so with
// every pixel set the sums are k_l1's.
__global__ __launch_bounds__(kLBlock) void k_l1_masked(int64_t count, int64_t plane, const float* __restrict__ img,
                                                       const float* __restrict__ gt,
                                                       const uint8_t* __restrict__ mask, float gscale,
                                                       float* __restrict__ grad, double* __restrict__ part, int vec) {
    __shared__ double s_a[kLBlock / kWave], s_b[kLBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kLTile;
    float sa = 0.f, sb = 0.f;
    if (vec && base + kLTile <= count) {
        const float4* I = reinterpret_cast<const float4*>(img + base);
        const float4* T = reinterpret_cast<const float4*>(gt + base);
        float4* D = reinterpret_cast<float4*>(grad + base);
        float4 x[kLIPT / 4], y[kLIPT / 4];
        uint32_t mk[kLIPT / 4];
#pragma unroll
        for (int r = 0; r < kLIPT / 4; ++r) {
            const int q = r * kLBlock + threadIdx.x;
            x[r] = I[q];
            y[r] = T[q];
            const uint32_t pix = (uint32_t)(base + 4 * q) % (uint32_t)plane;  // count < 2^32
            mk[r] = *reinterpret_cast<const uint32_t*>(mask + pix);
        }
#pragma unroll
        for (int r = 0; r < kLIPT / 4; ++r) {
            float4 gr;
            gr.x = (mk[r] & 0xffu) ? l1_term(x[r].x, y[r].x, gscale, sa, sb) : 0.f;
            gr.y = (mk[r] & 0xff00u) ? l1_term(x[r].y, y[r].y, gscale, sa, sb) : 0.f;
            gr.z = (mk[r] & 0xff0000u) ? l1_term(x[r].z, y[r].z, gscale, sa, sb) : 0.f;
            gr.w = (mk[r] & 0xff000000u) ? l1_term(x[r].w, y[r].w, gscale, sa, sb) : 0.f;
            if (grad) D[r * kLBlock + threadIdx.x] = gr;
        }
    } else {
#pragma unroll
        for (int r = 0; r < kLIPT; ++r) {
            const int64_t i = base + (int64_t)r * kLBlock + threadIdx.x;
            if (i < count) {
                const float gr = mask[(uint32_t)i % (uint32_t)plane] ? l1_term(img[i], gt[i], gscale, sa, sb) : 0.f;
                if (grad) grad[i] = gr;
            }
        }
    }
    l1_block_partials(sa, sb, s_a, s_b, part);
}

__global__ void k_loss_reduce(int64_t nb, int64_t count, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0, b = 0;
    for (int64_t k = 0; k < nb; ++k) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    out[0] = count > 0 ? a / (double)count : 0.0;
    out[1] = count > 0 ? b / (double)count : 0.0;
}

__global__ void k_adam(int64_t count, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

struct AdamSegs {
    float* p[8];
    float* g[8];
    float* m[8];
    float* v[8];
    float lr[8];
    int64_t count[8];
    int64_t qstart[9];  // prefix of the segment lengths in quads of 4 elements
    int vec[8];         // all four arrays of the segment 16-byte aligned: whole quads move as float4
    int nseg;
};

// All parameter groups of one optimiser step in one launch; the gradient is cleared after it is read so the
// next backward can accumulate into it without a separate zeroing pass.
// Device step counter: state[0] (int) is incremented, state[1], state[2] receive the bias corrections
// 1 - b1^t, 1 - b2^t of the new step (computed in double, rounded once, as on the host path).
__global__ void k_adam_tick(int32_t* __restrict__ state, float b1, float b2) {
    const int32_t t = state[0] + 1;
    state[0] = t;
    reinterpret_cast<float*>(state)[1] = (float)(1.0 - pow((double)b1, (double)t));
    reinterpret_cast<float*>(state)[2] = (float)(1.0 - pow((double)b2, (double)t));
}

__device__ __forceinline__ void adam_one(float& p, float& m, float& v, float g, float lr, float b1, float b2, float eps,
                                         float c1, float c2) {
    m = b1 * m + (1.f - b1) * g;
    v = b2 * v + (1.f - b2) * g * g;
    p -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// One thread per quad of 4 consecutive elements of a segment (16-byte loads and stores where aligned).
__global__ void k_adam_multi(AdamSegs S, float b1, float b2, float eps, float c1, float c2, int zero_grad,
                             const int32_t* __restrict__ state) {
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= S.qstart[S.nseg]) return;
    if (state) {
        c1 = reinterpret_cast<const float*>(state)[1];
        c2 = reinterpret_cast<const float*>(state)[2];
    }
    int s = 0;
#pragma unroll 1
    while (s + 1 < S.nseg && qi >= S.qstart[s + 1]) ++s;
    const int64_t j0 = (qi - S.qstart[s]) * 4;
    const float lr = S.lr[s];
    if (S.vec[s] && j0 + 4 <= S.count[s]) {
        float4* P = reinterpret_cast<float4*>(S.p[s] + j0);
        float4* G = reinterpret_cast<float4*>(S.g[s] + j0);
        float4* M = reinterpret_cast<float4*>(S.m[s] + j0);
        float4* V = reinterpret_cast<float4*>(S.v[s] + j0);
        const float4 g = *G;
        float4 p = *P, m = *M, v = *V;
        adam_one(p.x, m.x, v.x, g.x, lr, b1, b2, eps, c1, c2);
        adam_one(p.y, m.y, v.y, g.y, lr, b1, b2, eps, c1, c2);
        adam_one(p.z, m.z, v.z, g.z, lr, b1, b2, eps, c1, c2);
        adam_one(p.w, m.w, v.w, g.w, lr, b1, b2, eps, c1, c2);
        *P = p;
        *M = m;
        *V = v;
        if (zero_grad) *G = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
        const int64_t j1 = j0 + 4 < S.count[s] ? j0 + 4 : S.count[s];
        for (int64_t j = j0; j < j1; ++j) {
            float p = S.p[s][j], m = S.m[s][j], v = S.v[s][j];
            adam_one(p, m, v, S.g[s][j], lr, b1, b2, eps, c1, c2);
            S.p[s][j] = p;
            S.m[s][j] = m;
            S.v[s][j] = v;
            if (zero_grad) S.g[s][j] = 0.f;
        }
    }
}

}  // namespace
}  // namespace qg

using namespace qg;

extern "C" qg_status qg_adam_multi(int32_t nseg, const qg_adam_segment* segs, float b1, float b2, float eps, int32_t t,
                                   int32_t* step_state, int32_t zero_grad, qg_stream stream) {
    clear_error();
    QG_REQUIRE(nseg >= 1 && nseg <= 8 && segs, "nseg must be in [1, 8]");
    QG_REQUIRE(step_state || t >= 1, "t >= 1 required");
    QG_REQUIRE(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f && eps >= 0.f, "bad Adam constants");
    AdamSegs S = {};
    S.nseg = nseg;
    S.qstart[0] = 0;
    for (int k = 0; k < nseg; ++k) {
        const qg_adam_segment& q = segs[k];
        QG_REQUIRE(q.count >= 0, "segment %d: count < 0", k);
        QG_REQUIRE(q.count == 0 || (q.param && q.grad && q.m && q.v), "segment %d: a pointer is NULL", k);
        S.p[k] = q.param;
        S.g[k] = q.grad;
        S.m[k] = q.m;
        S.v[k] = q.v;
        S.lr[k] = q.lr;
        S.count[k] = q.count;
        S.qstart[k + 1] = S.qstart[k] + ceil_div(q.count, (int64_t)4);
        auto al16 = [](const float* x) { return ((uintptr_t)x & 15u) == 0; };
        S.vec[k] = al16(q.param) && al16(q.grad) && al16(q.m) && al16(q.v);
    }
    const int64_t total = S.qstart[nseg];
    const float c1 = step_state ? 1.f : (float)(1.0 - std::pow((double)b1, t));
    const float c2 = step_state ? 1.f : (float)(1.0 - std::pow((double)b2, t));
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("adam", s);
        if (step_state) k_adam_tick<<<1, 1, 0, s>>>(step_state, b1, b2);
        if (total > 0)
            k_adam_multi<<<(unsigned)ceil_div(total, 256), 256, 0, s>>>(S, b1, b2, eps, c1, c2, zero_grad, step_state);
    }
    QG_LAUNCH_CHECK("qg_adam_multi");
    return QG_OK;
}

extern "C" int64_t qg_loss_blocks(int64_t count) { return std::max<int64_t>(1, ceil_div(count, kLTile)); }

extern "C" qg_status qg_l1_loss(int64_t count, const float* image, const float* gt, float scale, float* grad_image,
                                double* partials, qg_stream stream) {
    clear_error();
    QG_REQUIRE(count >= 0, "count < 0");
    QG_REQUIRE(partials, "partials is NULL");
    QG_REQUIRE(count == 0 || (image && gt), "image/gt NULL");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = qg_loss_blocks(count);
    const float gs = count > 0 ? scale / (float)count : 0.f;
    {
        QG_TIMED("l1", s);
        auto al16 = [](const void* x) { return ((uintptr_t)x & 15u) == 0; };
        const int vec = al16(image) && al16(gt) && al16(grad_image);
        k_l1<<<(unsigned)nb, kLBlock, 0, s>>>(count, image, gt, gs, grad_image, partials, vec);
    }
    QG_LAUNCH_CHECK("qg_l1_loss");
    return QG_OK;
}

extern "C" qg_status qg_l1_loss_masked(int64_t count, int64_t plane, const float* image, const float* gt,
                                       const uint8_t* mask, float scale, float* grad_image, double* partials,
                                       qg_stream stream) {
    clear_error();
    QG_REQUIRE(count >= 0 && plane >= 1 && count % plane == 0, "count=%lld must be a multiple of plane=%lld >= 1",
               (long long)count, (long long)plane);
    QG_REQUIRE(count < (1ll << 32), "count=%lld must be < 2^32", (long long)count);
    QG_REQUIRE(partials, "partials is NULL");
    QG_REQUIRE(count == 0 || (image && gt && mask), "image/gt/mask NULL");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = qg_loss_blocks(count);
    const float gs = count > 0 ? scale / (float)count : 0.f;
    {
        QG_TIMED("l1", s);
        auto al16 = [](const void* x) { return ((uintptr_t)x & 15u) == 0; };
        const int vec = al16(image) && al16(gt) && al16(grad_image) && plane % 4 == 0 &&
                        ((uintptr_t)mask & 3u) == 0;
        k_l1_masked<<<(unsigned)nb, kLBlock, 0, s>>>(count, plane, image, gt, mask, gs, grad_image, partials, vec);
    }
    QG_LAUNCH_CHECK("qg_l1_loss_masked");
    return QG_OK;
}

extern "C" qg_status qg_loss_reduce(int64_t count, const double* partials, double* out, qg_stream stream) {
    clear_error();
    QG_REQUIRE(count >= 0 && partials && out, "bad arguments");
    {
        QG_TIMED("loss_reduce", (hipStream_t)stream);
        k_loss_reduce<<<1, 64, 0, (hipStream_t)stream>>>(qg_loss_blocks(count), count, partials, out);
    }
    QG_LAUNCH_CHECK("qg_loss_reduce");
    return QG_OK;
}

extern "C" qg_status qg_loss_reduce_parts(int64_t nparts, int64_t count, const double* partials, double* out,
                                          qg_stream stream) {
    clear_error();
    QG_REQUIRE(nparts >= 0 && count >= 0 && (nparts == 0 || partials) && out, "bad arguments");
    {
        QG_TIMED("loss_reduce", (hipStream_t)stream);
        k_loss_reduce<<<1, 64, 0, (hipStream_t)stream>>>(nparts, count, partials, out);
    }
    QG_LAUNCH_CHECK("qg_loss_reduce_parts");
    return QG_OK;
}

extern "C" qg_status qg_adam(int64_t count, float* param, const float* grad, float* m, float* v, float lr, float b1,
                             float b2, float eps, int32_t t, qg_stream stream) {
    clear_error();
    QG_REQUIRE(count >= 0 && t >= 1, "count >= 0 and t >= 1 required");
    QG_REQUIRE(count == 0 || (param && grad && m && v), "a pointer is NULL");
    QG_REQUIRE(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f && eps >= 0.f, "bad Adam constants");
    if (count == 0) return QG_OK;
    const float c1 = (float)(1.0 - std::pow((double)b1, t));
    const float c2 = (float)(1.0 - std::pow((double)b2, t));
    {
        QG_TIMED("adam", (hipStream_t)stream);
        k_adam<<<(unsigned)ceil_div(count, 256), 256, 0, (hipStream_t)stream>>>(count, param, grad, m, v, lr, b1, b2,
                                                                              eps, c1, c2);
    }
    QG_LAUNCH_CHECK("qg_adam");
    return QG_OK;
}
