// Fused per-Gaussian passes: decode + projection (forward) and projection adjoint + decode backward.
//
// The per-Gaussian chain is bound by HBM traffic.  Run as separate calls it writes the decoded 59-plane
// attribute tensor, reads it back in the projection, and in the backward writes and re-reads its
// gradient.  Here one wave owns 64 consecutive Gaussians: the decoder's products run on the matrix cores
// for the 64 Gaussians (decoder_mfma.h), the residuals land in LDS, and each lane then projects its own
// Gaussian (gauss_math.h) from prev + residual.  The backward stages the chunk's attribute planes in LDS
// (the forward's decoded attributes when the caller kept them, else prev with the residuals decoded again),
// projects back through them per lane, keeps the attribute gradient in the same LDS slots and feeds it
// straight to the decoder backward.  Results equal qg_decode_residuals + qg_project and qg_render_bwd +
// qg_decode_residuals_bwd.
#include <cmath>

#include "decoder_mfma.h"
#include "gauss_math.h"

namespace qg {

qg_status blend_bwd_launch(const ViewTable& vt, qg_tiling tiling, const uint32_t* vals, const uint32_t* ranges,
                           const float* bg, const float* const* T_final, const uint32_t* const* last,
                           const float* const* grad_image, float* grad2d, int64_t stride, int64_t n, PairPart pp,
                           hipStream_t s);
qg_status decode_reduce_launch(const float* part, int64_t nblocks, float* gW1, float* gW2, hipStream_t s);

namespace {

using namespace dec;

constexpr int kChunk = 64;

// Element offset of plane k of Gaussian g in a [planes][ld] array, in 32 bits (the entry points check that
// every plane offset fits): the loads then use an SGPR base and a 32-bit VGPR offset.
__device__ __forceinline__ uint32_t pidx(int k, uint32_t ld, uint32_t g) { return (uint32_t)k * ld + g; }

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Two waves per block, one chunk of 64 Gaussians per wave (straight-line code).  The decoder's output reaches
// the lanes one group of 16 Gaussians at a time through a 16-row LDS buffer (7 KB per block), so LDS no longer
// bounds the occupancy; the registers allow three waves per SIMD.
__global__ __launch_bounds__(128) void k_decode_project(int64_t n, int64_t ld, const float* __restrict__ prev,
                                                        const float* __restrict__ lat, const float* __restrict__ W1,
                                                        const float* __restrict__ W2, const float* __restrict__ lp,
                                                        const float* __restrict__ ga,
                                                        const float* __restrict__ gnoise, float g0, float g1,
                                                        float tau, float reg_shift, int sh_deg, ViewTable vt,
                                                        float dilation,
                                                        int tile_w, int tile_h, float* __restrict__ attrs_out,
                                                        float* __restrict__ gate_out, float* __restrict__ lreg_part) {
    __shared__ float s_res[2][16][kM + 1];
    __shared__ float s_red[2];
    const int lane = __lane_id(), w = threadIdx.x / 64, c = lane % 16;
    const int64_t nchunks = ceil_div(n, kChunk);
    const uint32_t ld32 = (uint32_t)ld;
    float preg = 0.f;
    const int64_t ch = (int64_t)blockIdx.x * 2 + w;
    if (ch < nchunks) {
        const int64_t base = ch * kChunk;
        const int64_t g = base + lane;
        const bool gv = g < n;
        const uint32_t g32 = (uint32_t)g;
        // issue every attribute load of this lane's Gaussian first; they land while the decoder runs
        float at[QG_N_PLANES];
#pragma unroll
        for (int k = 0; k < QG_N_PLANES; ++k) at[k] = gv ? prev[pidx(k, ld32, g32)] : 0.f;
        float lpv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) lpv[k] = gv ? lp[pidx(k, ld32, g32)] : 0.f;
        const float a = gv ? ga[g] : 0.f;
        const float an = (gv && gnoise) ? a + gnoise[g] : a;  // stochastic gate: log(alpha) + logistic sample
        {
            FwdOps ops;
            load_fwd_ops(W1, W2, ops);
            // one group of 16 Gaussians at a time through a 16-row buffer; the group's own lanes add its rows
#pragma unroll
            for (int sg = 0; sg < 4; ++sg) {
                const int64_t gs = base + 16 * sg + c;
                const bool vs = gs < n;
                auto latf = [&](int k) { return vs ? rintf(lat[pidx(k, ld32, (uint32_t)gs)]) : 0.f; };
                auto outf = [&](int m, float v) { s_res[w][c][m] = v; };
                decode_group_fwd(ops, latf, outf);
                wave_sync_lds();
                if (lane / 16 == sg) {
#pragma unroll
                    for (int k = 3; k < QG_N_PLANES; ++k) at[k] = at[k] + s_res[w][c][k - 3];
                }
                wave_sync_lds();
            }
        }
        if (gv) {
            const float gg = gate_of(an, g0, g1, tau, nullptr, nullptr);
#pragma unroll
            for (int k = 0; k < 3; ++k) at[k] = __builtin_fmaf(gg, lpv[k], at[k]);
            if (attrs_out) {
#pragma unroll
                for (int k = 0; k < QG_N_PLANES; ++k) attrs_out[pidx(k, ld32, g32)] = at[k];
            }
            auto get = [&](int k) { return at[k]; };
            project_gauss(g, get, sh_deg, vt, dilation, tile_w, tile_h);
            if (gate_out) gate_out[g] = gg;
            preg += sigm(a - reg_shift);
        }
    }
    if (lreg_part) {
        for (int o = 32; o >= 1; o >>= 1) preg += __shfl_xor(preg, o);
        if (lane == 0) s_red[w] = preg;
        __syncthreads();
        if (threadIdx.x == 0) lreg_part[blockIdx.x] = s_red[0] + s_red[1];
    }
}

// ---- backward: staging through LDS DMA ----------------------------------------------------------
// The backward keeps a chunk's per-Gaussian inputs in LDS, plane by plane (64 floats a plane).  They are
// copied there by global->LDS loads, which take no registers, so every plane of a chunk is in flight at once
// and the chunk waits on memory once.  A plane is stored rotated by a multiple of 16 slots (slot
// (g + rot) % 64 holds Gaussian g of the chunk): the decoder's column accesses, 16 Gaussians x 4 planes per
// instruction, then spread over the banks instead of landing four deep on one.
__device__ __forceinline__ int rot_at(int m) { return 16 * ((m + (m >> 2)) & 3); }
__device__ __forceinline__ int slot_at(int m, int g) { return m * kChunk + ((g + rot_at(m)) & (kChunk - 1)); }
__device__ __forceinline__ int slot_lat(int k, int g) { return k * kChunk + ((g + 16 * (k & 3)) & (kChunk - 1)); }

typedef __attribute__((address_space(3))) void* lds_ptr;

// The lane index, opaque to the optimiser: the LDS addresses derived from it are formed in the phase that uses
// them instead of all at once at the top of the kernel.
__device__ __forceinline__ int lane_here() {
    int l = __lane_id();
    asm volatile("" : "+v"(l));
    return l;
}

// Plane `plane` of the chunk's 64 Gaussians from src ([planes][ld]) into dst[0..63], rotated by rot: lane l
// fetches Gaussian base + ((l - rot) mod 64), at a uniform address plus a lane offset.  In the last, partial
// chunk (kFull == false) lanes past the last Gaussian fetch Gaussian n - 1 instead (their results are never
// stored, but their values reach the decoder's products, so they must be finite data).
template <bool kFull>
__device__ __forceinline__ void stage_plane(const float* __restrict__ src, int64_t ld, int plane, int64_t base,
                                            int64_t n, int lane, int rot, float* dst) {
    const uint32_t off = (uint32_t)(lane - rot) & (kChunk - 1);
    const float* row = src + (int64_t)plane * ld + base;
    const float* p = kFull ? row + off : row + (base + off < n ? off : n - 1 - base);
    __builtin_amdgcn_global_load_lds(p, (lds_ptr)dst, 4, 0, 0);
}

// Every input plane of a chunk: attribute planes 3..58 (of prev, or of the decoded attributes), the latents,
// the incoming g_lp and g_ga.
template <bool kFull>
__device__ __forceinline__ void stage_chunk(const float* __restrict__ prev, const float* __restrict__ lat,
                                            const float* g_lp, const float* g_ga, int64_t ld, int64_t base, int64_t n,
                                            float* at, float* sl, float* so) {
    const int l0 = lane_here();
#pragma unroll
    for (int m = 0; m < kM; ++m) stage_plane<kFull>(prev, ld, 3 + m, base, n, l0, rot_at(m), at + m * kChunk);
#pragma unroll
    for (int k = 0; k < kL; ++k) stage_plane<kFull>(lat, ld, k, base, n, l0, 16 * (k & 3), sl + k * kChunk);
#pragma unroll
    for (int k = 0; k < 3; ++k) stage_plane<kFull>(g_lp, ld, k, base, n, l0, 0, so + k * kChunk);
    stage_plane<kFull>(g_ga, ld, 0, base, n, l0, 0, so + 3 * kChunk);
}

// Pins the loaded values in registers, so that the compiler cannot fold a later choice between them and a
// load from memory into a load through a chosen pointer (which would put them in scratch memory).
__device__ __forceinline__ void in_vgprs(BwdPre& p) {
    float* f[] = {&p.r0.g0.x, &p.r0.g0.y, &p.r0.g0.z, &p.r0.g0.w, &p.r0.g1.x, &p.r0.g1.y, &p.r0.g1.z,
                  &p.r0.g1.w, &p.r0.g2.x, &p.r0.g2.y, &p.r0.g2.z, &p.r0.g2.w, &p.gabs};
#pragma unroll
    for (float* x : f) asm volatile("" : "+v"(*x));
    asm volatile("" : "+v"(p.r0.flags));
}

// kDecoded: `prev` holds the decoded attributes of this step (prev + residual, positions with the gate
// applied), so the residuals are not decoded again.
// kDet: each wave writes its weight-gradient accumulators to its own row of wpart (row = chunk) instead of adding
// them into the block's LDS sums with float atomics, so the fixed-order reduce over the rows is deterministic.
template <bool kDecoded, bool kDet>
__global__ __launch_bounds__(256, 2) void k_project_decode_bwd(
    int64_t n, int64_t ld, const float* __restrict__ prev, const float* __restrict__ lat, const float* __restrict__ W1,
    const float* __restrict__ W2, const float* __restrict__ lp, const float* __restrict__ ga,
    const float* __restrict__ gnoise, float g0, float g1, float tau, float reg_shift, float reg_scale, int sh_deg,
    ViewTable vt, float dilation,
    const float* __restrict__ grad2d, int64_t stride, float* __restrict__ gxy_abs, ViewPtrs gxyv,
    float* __restrict__ g_lat, float* __restrict__ g_lp, float* __restrict__ g_ga, float* __restrict__ wpart) {
    // per wave:
    //   s_at:  attribute planes 3..58 (prev + residual while projecting), then dL/dr in the same slots
    //   s_lat: the latents as stored, then dL/dlatent
    //   s_old: the incoming g_lp (3 planes) and g_ga (1 plane), slot = Gaussian
    __shared__ float s_at[4][kM * kChunk];
    __shared__ float s_lat[4][kL * kChunk];
    __shared__ float s_old[4][4 * kChunk];
    __shared__ float s_acc[kWidth];  // the block's decoder weight-gradient sums (LDS float atomics)
    const int lane = __lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    float* const at = s_at[w];
    float* const sl = s_lat[w];
    float* const so = s_old[w];
    for (int i = threadIdx.x; i < kWidth; i += 256) s_acc[i] = 0.f;
    __syncthreads();
    const int64_t nchunks = ceil_div(n, kChunk);
    const uint32_t ld32 = (uint32_t)ld;
    // one chunk per wave: straight-line code, so nothing is kept in registers across chunks
    const int64_t ch = (int64_t)blockIdx.x * 4 + w;
    if (ch < nchunks) {
        const int64_t base = ch * kChunk;
        const int64_t g = base + lane;
        const bool gv = g < n;
        const uint32_t g32 = (uint32_t)g;
        // 0. stage the chunk
        if (base + kChunk <= n)
            stage_chunk<true>(prev, lat, g_lp, g_ga, ld, base, n, at, sl, so);
        else
            stage_chunk<false>(prev, lat, g_lp, g_ga, ld, base, n, at, sl, so);
        float pos[3], lpv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            pos[k] = gv ? prev[pidx(k, ld32, g32)] : 0.f;
            lpv[k] = gv ? lp[pidx(k, ld32, g32)] : 0.f;
        }
        const float a = gv ? ga[g] : 0.f;
        const float an = (gv && gnoise) ? a + gnoise[g] : a;  // stochastic gate: log(alpha) + logistic sample
        // view 0's gradient record and the old |grad xy| sum, loaded with the chunk (one wait for HBM)
        BwdPre pre{};
        if (gv) pre = load_bwd_pre(vt, grad2d, stride, gxy_abs, g);
        // the incoming dL/dlatent, from a clamped index (a lane past n loads Gaussian n-1 and stores nothing)
        float glat[kL];
        const uint32_t gc = gv ? g32 : (uint32_t)(n - 1);
#pragma unroll
        for (int k = 0; k < kL; ++k) glat[k] = g_lat[pidx(k, ld32, gc)];
        __builtin_amdgcn_s_waitcnt(0);
        in_vgprs(pre);
#pragma unroll
        for (int k = 0; k < kL; ++k) asm volatile("" : "+v"(glat[k]));
        wave_sync_lds();
        // 1. add the decoded residuals in place
        if (!kDecoded) {
            const int c1 = lane_here() % 16;
            FwdOps ops;
            load_fwd_ops(W1, W2, ops);
#pragma unroll
            for (int sg = 0; sg < 4; ++sg) {
                const int gs = 16 * sg + c1;
                auto latf = [&](int k) { return rintf(sl[slot_lat(k, gs)]); };
                auto outf = [&](int m, float v) { at[slot_at(m, gs)] += v; };
                decode_group_fwd(ops, latf, outf);
            }
        }
        wave_sync_lds();
        // 2. projection adjoint per Gaussian; position and gate gradients
        if (gv) {
            const int l2 = lane_here();
            float gh, gt;
            const float gg = gate_of(an, g0, g1, tau, &gh, &gt);
            if (!kDecoded) {
#pragma unroll
                for (int k = 0; k < 3; ++k) pos[k] = __builtin_fmaf(gg, lpv[k], pos[k]);
            }
            auto get = [&](int k) { return k < 3 ? pos[k] : at[slot_at(k - 3, l2)]; };
            float dpos[3] = {0.f, 0.f, 0.f};
            auto put = [&](int k, float v) {
                if (k < 3)
                    dpos[k] = v;
                else
                    at[slot_at(k - 3, l2)] = v;
            };
            project_bwd_gauss<true, true>(n, g, get, put, sh_deg, vt, dilation, grad2d, stride, gxy_abs, gxyv, pre);
            const int nb = (sh_deg + 1) * (sh_deg + 1);
            for (int m = 8 + 3 * nb; m < kM; ++m) at[slot_at(m, l2)] = 0.f;  // SH planes above the degree
            float dot = 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                dot = __builtin_fmaf(dpos[k], lpv[k], dot);
                g_lp[pidx(k, ld32, g32)] = so[k * kChunk + l2] + gg * dpos[k];
            }
            float da = (gt > 0.f && gt < 1.f) ? dot * (g1 - g0) * gh * (1.f - gh) / tau : 0.f;
            const float pr = sigm(a - reg_shift);
            g_ga[g] = so[3 * kChunk + l2] + __builtin_fmaf(reg_scale, pr * (1.f - pr), da);
        } else {
            const int l2 = lane_here();
#pragma unroll
            for (int m = 0; m < kM; ++m) at[slot_at(m, l2)] = 0.f;
        }
        wave_sync_lds();
        // 3. decoder backward from the gradient in LDS; this chunk's weight gradients are added to s_acc and
        //    dL/dlatent replaces the latents in s_lat
        {
            const int l3 = lane_here(), q3 = l3 / 16, c3 = l3 % 16;
            BwdOps ops;
            load_bwd_ops(W1, W2, ops);
            BwdAcc acc;
            zero_acc(acc);
            // first halves of the four groups, one barrier, then the four dL chains together.  The transpose
            // buffer of group sg is planes 0..31 of its own Gaussians' slots, dead once that group's reads are
            // done; dL/dlatent goes to the group's own latent slots, read by nothing after its first half.
#pragma unroll
            for (int sg = 0; sg < 4; ++sg) {
                const int gA = 16 * sg + c3;
                auto latA = [&](int k) { return rintf(sl[slot_lat(k, gA)]); };
                auto latN = [&](int k, int i) { return rintf(sl[slot_lat(k, 16 * sg + 4 * q3 + i)]); };
                auto drA = [&](int m) { return at[slot_at(m, gA)]; };
                auto drN = [&](int m, int i) { return m < kM ? at[slot_at(m, 16 * sg + 4 * q3 + i)] : 0.f; };
                auto tb = [&](int r, int j) -> float& { return at[slot_at(j, 16 * sg + r)]; };
                decode_group_bwd_a(ops, acc, latA, latN, drA, drN, tb);
            }
            wave_sync_lds();
#pragma unroll
            for (int sg = 0; sg < 4; ++sg) {
                const int gA = 16 * sg + c3;
                auto dlat = [&](int k, float v) { sl[slot_lat(k, gA)] = v; };
                auto tb = [&](int r, int j) -> float& { return at[slot_at(j, 16 * sg + r)]; };
                decode_group_bwd_b(ops, dlat, tb);
            }
            if constexpr (kDet)
                store_acc(acc, wpart + (size_t)ch * kWidth);
            else
                add_acc_atomic(acc, s_acc);
        }
        wave_sync_lds();
        if (gv) {
            const int l4 = lane_here();
#pragma unroll
            for (int k = 0; k < kL; ++k) g_lat[pidx(k, ld32, g32)] = glat[k] + sl[slot_lat(k, l4)];
        }
    }
    if constexpr (!kDet) {
        __syncthreads();
        for (int i = threadIdx.x; i < kWidth; i += 256) wpart[(size_t)blockIdx.x * kWidth + i] = s_acc[i];
    }
}

int64_t fused_fwd_blocks(int64_t n) { return std::max<int64_t>(1, ceil_div(ceil_div(n, kChunk), 2)); }
int64_t fused_bwd_blocks(int64_t n) { return std::max<int64_t>(1, ceil_div(ceil_div(n, kChunk), 4)); }

qg_status check_dec(int32_t L, int32_t Hd, int32_t M, float g0, float g1, float tau) {
    QG_REQUIRE(L >= 1 && L <= 16, "L=%d outside [1, 16]", L);
    QG_REQUIRE(Hd == 0 || Hd == 32, "Hd=%d must be 0 or 32", Hd);
    QG_REQUIRE(M == 56, "M=%d must be 56", M);
    QG_REQUIRE(g0 < 0.f && g1 > 1.f && tau > 0.f, "need gamma0 < 0, gamma1 > 1, tau > 0");
    if (!(L == kL && Hd == kH)) {
        set_error("decoder shape L=%d Hd=%d not built (supported: L=8, Hd=32)", L, Hd);
        return QG_ERR_UNSUPPORTED;
    }
    return QG_OK;
}

}  // namespace
}  // namespace qg

using namespace qg;

extern "C" int64_t qg_decode_project_lreg_blocks(int64_t n) { return fused_fwd_blocks(n); }

extern "C" qg_status qg_decode_project(int64_t n, int64_t ld, const float* prev_attrs, const float* latents,
                                       int32_t L, const float* W1, const float* W2, int32_t Hd, int32_t M,
                                       const float* pos_pre, const float* gate_logit, const float* gate_noise,
                                       float gamma0, float gamma1, float tau, int32_t sh_degree,
                                       const qg_camera* cams, int32_t V,
                                       qg_tiling tiling, float dilation, const qg_projected* out, float* attrs_out,
                                       float* gate_out, float* lreg_partial, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n && n < (1ll << 31), "n=%lld ld=%lld invalid", (long long)n, (long long)ld);
    qg_status st = check_dec(L, Hd, M, gamma0, gamma1, tau);
    if (st != QG_OK) return st;
    QG_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "sh_degree=%d outside [0, 3]", sh_degree);
    QG_REQUIRE(dilation >= 0.f && std::isfinite(dilation), "dilation must be finite and >= 0");
    QG_REQUIRE(n == 0 || (prev_attrs && latents && W1 && W2 && pos_pre && gate_logit), "a required pointer is NULL");
    QG_REQUIRE(attrs_out != prev_attrs, "attrs_out may not alias prev_attrs");
    QG_REQUIRE((int64_t)QG_N_PLANES * ld < (1ll << 31), "59 * ld must be < 2^31 for the fused kernels");
    ViewTable vt;
    if (!make_view_table(cams, out, V, tiling, true, &vt)) return QG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = fused_fwd_blocks(n);
    if (n == 0) return lreg_partial ? qg_zero(lreg_partial, 4 * nb, stream) : QG_OK;
    const float shift = tau * logf(-gamma0 / gamma1);
    {
        QG_TIMED("decode_project", s);
        k_decode_project<<<(unsigned)nb, 128, 0, s>>>(n, ld, prev_attrs, latents, W1, W2, pos_pre, gate_logit,
                                                      gate_noise, gamma0, gamma1, tau, shift, sh_degree, vt, dilation, tiling.tile_w,
                                                      tiling.tile_h, attrs_out, gate_out, lreg_partial);
    }
    QG_LAUNCH_CHECK("qg_decode_project");
    return QG_OK;
}

namespace qg {
size_t det_weight_part_bytes(int64_t n) {
    return align_up((size_t)std::max<int64_t>(1, ceil_div(n, kChunk)) * kWidth * sizeof(float));
}
}  // namespace qg

// Deterministic-mode workspace after an adjoint call's own: the fused adjoint's weight-gradient rows, the slot
// bases [n * V] and their block sums, then the pair partials (as many slots as fit: the bin capacity).
static size_t det_fixed_bytes(int64_t n, int32_t V) {
    const int64_t items = std::max<int64_t>(n * V, 1);
    return det_weight_part_bytes(n) + align_up((size_t)items * 4) + align_up((size_t)ceil_div(items, 1024) * 4);
}

namespace qg {
qg_status det_layout(char* base, size_t bytes, int64_t n, int32_t V, float** wdet, PairPart* pp) {
    const size_t fixed = det_fixed_bytes(n, V);
    QG_REQUIRE(bytes >= fixed + align_up(kPairPart * 4), "deterministic mode: the workspace has %zu bytes past the "
               "call's own, fewer than the %zu its partials need (add qg_deterministic_workspace_size)", bytes,
               fixed + align_up(kPairPart * 4));
    if (wdet) *wdet = (float*)base;
    const size_t wb = det_weight_part_bytes(n);
    pp->base = (uint32_t*)(base + wb);
    pp->part = (float*)(base + fixed);
    const size_t c = (bytes - fixed) / (kPairPart * sizeof(float));
    pp->cap = (uint32_t)(c < 0xFFFFFFFFull ? c : 0xFFFFFFFFull);
    pp->n = n;
    return QG_OK;
}
}  // namespace qg

extern "C" size_t qg_deterministic_workspace_size(int64_t n, int32_t V, int64_t capacity) {
    if (n < 0 || V < 1 || capacity < 0) return 0;
    return det_fixed_bytes(n, V) + align_up((size_t)std::max<int64_t>(capacity, 1) * kPairPart * sizeof(float));
}

extern "C" size_t qg_render_decode_bwd_workspace_size(int64_t n, int32_t V) {
    if (n < 0 || V < 1) return 0;
    const size_t g2 = align_up((size_t)V * (size_t)(n > 0 ? n : 1) * QG_GRAD2D_STRIDE * sizeof(float));
    return g2 + align_up((size_t)fused_bwd_blocks(n) * kWidth * sizeof(float));
}

extern "C" qg_status qg_render_decode_bwd(
    int64_t n, int64_t ld, const float* prev_attrs, const float* attrs, const float* latents, int32_t L,
    const float* W1, const float* W2,
    int32_t Hd, int32_t M, const float* pos_pre, const float* gate_logit, const float* gate_noise, float gamma0,
    float gamma1, float tau, float lambda_reg, int32_t sh_degree, const qg_camera* cams, int32_t V, qg_tiling tiling,
    float dilation,
    const qg_projected* proj, const uint32_t* vals, const uint32_t* tile_ranges, const float* bg,
    const float* const* T_final, const uint32_t* const* last, const float* const* grad_image, float* grad_latents,
    float* grad_W1, float* grad_W2, float* grad_pos_pre, float* grad_gate_logit, float* grad_xy_abs,
    float* const* grad_xy, void* ws, size_t ws_bytes, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n && n < (1ll << 31), "n=%lld ld=%lld invalid", (long long)n, (long long)ld);
    qg_status st = check_dec(L, Hd, M, gamma0, gamma1, tau);
    if (st != QG_OK) return st;
    QG_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "sh_degree=%d outside [0, 3]", sh_degree);
    QG_REQUIRE(dilation >= 0.f, "dilation < 0");
    QG_REQUIRE((int64_t)QG_N_PLANES * ld < (1ll << 31), "59 * ld must be < 2^31 for the fused kernels");
    ViewTable vt;
    if (!make_view_table(cams, proj, V, tiling, true, &vt)) return QG_ERR_ARG;
    QG_REQUIRE(tile_ranges && bg && T_final && last && grad_image, "a required pointer is NULL");
    QG_REQUIRE(n == 0 || ((prev_attrs || attrs) && latents && W1 && W2 && pos_pre && gate_logit && grad_latents &&
                          grad_W1 && grad_W2 && grad_pos_pre && grad_gate_logit),
               "a required pointer is NULL");
    for (int v = 0; v < V; ++v)
        QG_REQUIRE(T_final[v] && last[v] && grad_image[v], "view %d: an input pointer is NULL", v);
    const size_t need = qg_render_decode_bwd_workspace_size(n, V);
    QG_REQUIRE(ws && ws_bytes >= need, "workspace too small: %zu < %zu", ws_bytes, need);
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    float* grad2d = (float*)ws;
    const int64_t stride = n * QG_GRAD2D_STRIDE;
    float* wpart = (float*)((char*)ws + align_up((size_t)V * (size_t)n * QG_GRAD2D_STRIDE * sizeof(float)));
    const bool det = deterministic_mode();
    PairPart pp{nullptr, 0, nullptr, n};
    float* wdet = nullptr;
    if (det) {
        st = det_layout((char*)ws + need, ws_bytes - need, n, V, &wdet, &pp);
        if (st != QG_OK) return st;
    }
    st = qg_zero(grad2d, (int64_t)V * stride * 4, stream);
    if (st != QG_OK) return st;
    st = blend_bwd_launch(vt, tiling, vals, tile_ranges, bg, T_final, last, grad_image, grad2d, stride, n, pp, s);
    if (st != QG_OK) return st;
    ViewPtrs gv = {};
    if (grad_xy)
        for (int v = 0; v < V; ++v) gv.p[v] = grad_xy[v];
    const int64_t nb = fused_bwd_blocks(n);
    const float shift = tau * logf(-gamma0 / gamma1);
    const float reg_scale = lambda_reg / (float)n;
    {
        QG_TIMED("project_decode_bwd", s);
        const float* src = attrs ? attrs : prev_attrs;
        float* wp = det ? wdet : wpart;
#define QG_PDB_ARGS                                                                                                 \
    n, ld, src, latents, W1, W2, pos_pre, gate_logit, gate_noise, gamma0, gamma1, tau, shift, reg_scale, sh_degree,   \
        vt, dilation,                                                                                                 \
        grad2d, stride, grad_xy_abs, gv, grad_latents, grad_pos_pre, grad_gate_logit, wp
        if (attrs && !det)
            k_project_decode_bwd<true, false><<<(unsigned)nb, 256, 0, s>>>(QG_PDB_ARGS);
        else if (attrs)
            k_project_decode_bwd<true, true><<<(unsigned)nb, 256, 0, s>>>(QG_PDB_ARGS);
        else if (!det)
            k_project_decode_bwd<false, false><<<(unsigned)nb, 256, 0, s>>>(QG_PDB_ARGS);
        else
            k_project_decode_bwd<false, true><<<(unsigned)nb, 256, 0, s>>>(QG_PDB_ARGS);
#undef QG_PDB_ARGS
    }
    QG_LAUNCH_CHECK("qg_render_decode_bwd");
    // deterministic mode: one row per 64-Gaussian chunk, reduced in a fixed order like the block rows
    return decode_reduce_launch(det ? wdet : wpart, det ? ceil_div(n, kChunk) : nb, grad_W1, grad_W2, s);
}
