// Front-to-back alpha compositing (Eq. 2) over tiles, and its reverse-order adjoint.
//
// Layout: one 64-lane wavefront per tile (one workgroup = one wave, so no cross-wave reduction is
// ever needed).  A tile of TW x TH pixels gives each lane PPL = TW*TH/64 pixels that all lie in one
// column: the lane's x offset (and every term of the conic form that only depends on dx) is shared
// by its PPL pixels.  The tile's depth-ordered entries are staged 64 at a time in LDS (one record per
// lane, gathered from the 48-byte splat records) and read back as wave-uniform broadcasts.  A ballot
// over the pixels still running ends the loop early.
//
// The adjoint walks the entries backwards from each pixel's last contributor and recomputes the
// transmittance in reverse, T_i = T_{i+1} / (1 - alpha_i), starting from the stored final T, so no
// per-pixel lists are kept.  Per entry, each lane first sums its PPL pixels, then the wave sums its
// 64 lanes (DPP scans inside each 16-lane row, then the four row totals through LDS), and 9 lanes
// issue one float atomic each into the Gaussian's 2D gradient record.
//
// The blend alpha is evaluated by one inline function used by both kernels, with explicit fused
// multiply-adds, so the forward's skip/clamp/termination decisions are reproduced exactly.

#include "l1_term.h"
#include "qg_internal.h"

namespace qg {

qg_status project_bwd_launch(int64_t n, int64_t ld, const float* attrs, int sh_degree, const ViewTable& vt,
                             float dilation, const float* grad2d, int64_t g2d_view_stride, float* grad_attrs,
                             float* grad_xy_abs, float* const* grad_xy, hipStream_t s);

namespace {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
// -0.5 * log2(e): exp(-q/2) = exp2(kFold * q)
constexpr float kFold = -0.72134752044448170f;
// Per-entry factor of the adjoint's sum number k (x, y, A, B, C, opacity, r, g, b): the position sums carry
// m (B dy + A dx) and m (C dy + B dx) with dL/dx, dL/dy = +sum; the conic sums carry m dx^2, m dx dy, m dy^2
// with dL/dA = -sum/2, dL/dB = -sum (B enters q twice), dL/dC = -sum/2.
__device__ __forceinline__ float geom_scale(int k) { return k == 3 ? -1.f : ((k == 2 || k == 4) ? -0.5f : 1.f); }

struct ViewPtrsF {
    float* p[QG_MAX_VIEWS];
};
struct ViewPtrsCF {
    const float* p[QG_MAX_VIEWS];
};
struct ViewPtrsU {
    uint32_t* p[QG_MAX_VIEWS];
};
struct ViewPtrsCU {
    const uint32_t* p[QG_MAX_VIEWS];
};

// The L1 term of Eq. 3 in the blend forward's epilogue (qg_render_fwd_l1): per view the ground truth, the
// gradient image and the gradient scale (scale / element count); per tile two partial sums.
struct FwdL1 {
    const float* gt[QG_MAX_VIEWS];
    float* grad[QG_MAX_VIEWS];
    float gscale[QG_MAX_VIEWS];
    double* part;  // [2 * total_tiles]
};

// Map workgroup -> tile so that each of the 8 XCDs (which take workgroups round-robin) gets a contiguous
// run of tiles: neighbouring tiles share splats, so they should share an L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t per_xcd) { return (b % 8) * per_xcd + b / 8; }

// Tile order of the blend kernels' plain grid.  Workgroups are dispatched to the 8 XCDs round-robin (block b
// runs on XCD b % 8), and each XCD has its own L2.  Tiles are grouped into super-tiles of S x S tiles (per
// view, padded at the right and bottom edges); super-tile j goes to XCD j % 8, and its S*S tiles run as
// consecutive workgroups of that XCD.  Neighbouring tiles, which share most of their Gaussians, thus share an
// L2, while every XCD gets super-tiles from all over the image: the dense middle of a view is spread over
// all eight XCDs instead of falling to the one or two that a contiguous band of tiles would give it.
struct TileMap {
    int32_t S;                         // super-tile side in tiles
    int32_t V;
    int64_t supers;                    // super-tiles over all views
    int32_t sup_off[QG_MAX_VIEWS + 1];  // first super-tile of each view
    int32_t sw[QG_MAX_VIEWS];          // super-tiles per row of each view
};

// XCD of a tile under that order: its super-tile's index mod 8.
__device__ __forceinline__ uint32_t xcd_of_tile(const TileMap& m, const ViewTable& vt, int v, int tx, int ty) {
    return (uint32_t)((m.sup_off[v] + (int64_t)(ty / m.S) * m.sw[v] + tx / m.S) & 7);
}

// Global tile of workgroup b, or -1 for a workgroup that falls on padding.
__device__ __forceinline__ int64_t map_tile(const TileMap& m, const ViewTable& vt, int64_t b) {
    const int S2 = m.S * m.S;
    const int64_t k = b >> 3;
    const int64_t j = (k / S2) * 8 + (b & 7);
    if (j >= m.supers) return -1;
    const int mm = (int)(k % S2);
    int v = 0;
    while (v + 1 < m.V && j >= m.sup_off[v + 1]) ++v;
    const int64_t jl = j - m.sup_off[v];
    const int tx = (int)(jl % m.sw[v]) * m.S + mm % m.S;
    const int ty = (int)(jl / m.sw[v]) * m.S + mm / m.S;
    const CamDev& c = vt.cam[v];
    if (tx >= c.grid_w || ty >= c.grid_h) return -1;
    return (int64_t)c.tile_off + (int64_t)ty * c.grid_w + tx;
}

__device__ __forceinline__ int view_of_tile(const ViewTable& vt, uint32_t t) {
    int v = 0;
    for (int k = 1; k < vt.V; ++k)
        if (t >= vt.cam[k].tile_off) v = k;
    return v;
}

// Folded conic: q' = kFold * q = A' dx^2 + 2 B' dx dy + C' dy^2; returns exp(-q/2) = exp2(q').
// The blend alpha is min(0.99, o * blend_e(...)).
__device__ __forceinline__ float blend_e(float fa, float fb2, float fc, float dx, float dy) {
    const float adx2 = (fa * dx) * dx;
    const float bdx = fb2 * dx;
    const float qf = __builtin_fmaf(__builtin_fmaf(fc, dy, bdx), dy, adx2);
    return __builtin_amdgcn_exp2f(qf);
}

// Entry culling against the tile: false only if no pixel centre of the box [bx0, bx1] x [by0, by1] can get
// alpha >= 1/255 from this splat, i.e. min over the box of q = A dx^2 + 2 B dx dy + C dy^2 exceeds
// k^2 = 2 ln(255 o) (with a margin far above the float32 error of the blend's own evaluation of q).  The
// minimum of a positive-definite quadratic over a box is 0 if the centre is inside, else it lies on an
// edge, where the 1D minimiser is clamped to the edge.  Anything not finite or degenerate counts as a hit.
__device__ __forceinline__ bool tile_hit(float x, float y, float o, float A, float B, float C, float bx0, float bx1,
                                         float by0, float by1) {
    if (255.f * o < 0.999f) return false;  // alpha <= o < 1/255 everywhere
    if (!(A > 0.f && C > 0.f && A * C - B * B > 0.f)) return true;
    const float lim = 2.f * __logf(fmaxf(255.f * o, 1.f)) * 1.002f + 0.02f;
    const float dx0 = bx0 - x, dx1 = bx1 - x, dy0 = by0 - y, dy1 = by1 - y;
    if (dx0 <= 0.f && dx1 >= 0.f && dy0 <= 0.f && dy1 >= 0.f) return true;
    const float rc = -B / C, ra = -B / A;
    float qmin = __builtin_huge_valf();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const float ex = s ? dx1 : dx0;  // edge x = const
        const float ey_ = fminf(fmaxf(rc * ex, dy0), dy1);
        qmin = fminf(qmin, __builtin_fmaf(__builtin_fmaf(C, ey_, 2.f * B * ex), ey_, A * ex * ex));
        const float ey = s ? dy1 : dy0;  // edge y = const
        const float ex_ = fminf(fmaxf(ra * ey, dx0), dx1);
        qmin = fminf(qmin, __builtin_fmaf(__builtin_fmaf(A, ex_, 2.f * B * ey), ex_, C * ey * ey));
    }
    return !(qmin > lim);
}

template <int TW, int TH>
struct TileGeom {
    static constexpr int PPL = TW * TH / 64;
    static constexpr int ROWS_PER_K = 64 / TW;  // rows advanced per pixel slot
};

// Blend of one tile (one wave); BD entries are staged per LDS batch.  kL1: the epilogue also writes the L1
// gradient of each output value and the tile's two partial sums (l1).
template <int TW, int TH, int BD, bool kL1>
__device__ __forceinline__ void fwd_tile(const ViewTable& vt, const uint32_t* __restrict__ vals,
                                         const uint32_t* __restrict__ ranges, float bg0, float bg1, float bg2,
                                         const ViewPtrsF& image, const ViewPtrsF& tfinal, const ViewPtrsU& lastp,
                                         const FwdL1& l1, int64_t tile, float4* s_a, float4* s_b, float* s_c,
                                         uint32_t* s_pos) {
    constexpr int PPL = TileGeom<TW, TH>::PPL;
    constexpr int RPK = TileGeom<TW, TH>::ROWS_PER_K;
    const int v = view_of_tile(vt, (uint32_t)tile);
    const CamDev& cam = vt.cam[v];
    const int local = (int)(tile - cam.tile_off);
    const int tx = local % cam.grid_w, ty = local / cam.grid_w;
    const int lane = threadIdx.x;
    const int px = tx * TW + (lane % TW);
    const int py0 = ty * TH + lane / TW;
    const float fx = (float)px + 0.5f;
    // T > 0: the pixel is still compositing; the sign flips when it stops (or for pixels outside the image),
    // so the running state needs no register of its own.  The final transmittance is |T|.
    float T[PPL], C0[PPL], C1[PPL], C2[PPL], fy[PPL];
    uint32_t last[PPL];
    const uint32_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        fy[k] = (float)(py0 + k * RPK) + 0.5f;
        T[k] = (px < cam.width && (py0 + k * RPK) < cam.height) ? 1.f : -1.f;
        C0[k] = C1[k] = C2[k] = 0.f;
        last[k] = s;
    }
    const float* __restrict__ splat = vt.proj[v].splat;
    // pixel centres of this tile inside the image
    const float bx0 = (float)(tx * TW) + 0.5f, bx1 = (float)min(tx * TW + TW, cam.width) - 0.5f;
    const float by0 = (float)(ty * TH) + 0.5f, by1 = (float)min(ty * TH + TH, cam.height) - 0.5f;
    for (uint32_t b = s; b < e; b += BD) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < PPL; ++k) any |= T[k] > 0.f;
        if (__ballot(any) == 0) break;
        // stage the batch, keeping (in order) only the entries that can reach alpha >= 1/255 in this tile
        int cnt = 0;
#pragma unroll
        for (int q = 0; q < (BD + 63) / 64; ++q) {
            const int slot = q * 64 + lane;
            const uint32_t j = b + (uint32_t)slot;
            bool hit = false;
            float4 r0, r1, r2;
            if (slot < BD && j < e) {
                const uint32_t gid = vals[j];
                const float4* r = reinterpret_cast<const float4*>(splat) + 3 * (size_t)gid;
                r0 = r[0];
                r1 = r[1];
                r2 = r[2];
                hit = tile_hit(r0.x, r0.y, r0.z, r1.x, r1.y, r1.z, bx0, bx1, by0, by1);
            }
            const uint64_t m = __ballot(hit);
            if (hit) {
                const int dst = cnt + (int)__popcll(m & ((1ull << lane) - 1ull));
                s_a[dst] = make_float4(r0.x, r0.y, r0.z, kFold * r1.x);
                s_b[dst] = make_float4(2.f * kFold * r1.y, kFold * r1.z, r2.x, r2.y);
                s_c[dst] = r2.z;
                s_pos[dst] = j;
            }
            cnt += (int)__popcll(m);
        }
        __syncthreads();
        // two entries per iteration: the wave checks whether any of its pixels still composites once per pair
        // (a stopped pixel takes no entry, so the check only saves work)
        for (int j0 = 0; j0 < cnt; j0 += 2) {
            bool any2 = false;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int jj = j0 + u;
                if (u > 0 && jj >= cnt) break;
                const float4 a = s_a[jj];
                const float4 bb = s_b[jj];
                const float cb = s_c[jj];
                const uint32_t pos1 = s_pos[jj] + 1;
                const float dx = fx - a.x;
                any2 = false;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    // skip if alpha < 1/255; stop before T' < 1e-4.  The branches are on the exec mask: lanes
                    // that skip the entry do no work, and a pixel slot where no lane takes it costs nothing more.
                    const float dy = fy[k] - a.y;
                    const float raw = a.z * blend_e(a.w, bb.x, bb.y, dx, dy);
                    const float al = fminf(kAlphaMax, raw);
                    if (T[k] > 0.f && al >= kAlphaMin) {
                        const float w = al * T[k];
                        const float tn = T[k] - w;  // T (1 - alpha)
                        if (tn < kTMin) {
                            T[k] = -T[k];  // stopped: this entry and all later ones are not taken
                        } else {
                            C0[k] = __builtin_fmaf(bb.z, w, C0[k]);
                            C1[k] = __builtin_fmaf(bb.w, w, C1[k]);
                            C2[k] = __builtin_fmaf(cb, w, C2[k]);
                            T[k] = tn;
                            last[k] = pos1;
                        }
                    }
                    any2 |= T[k] > 0.f;
                }
            }
            if (__ballot(any2) == 0) break;
        }
        __syncthreads();
    }
    const int W = cam.width, H = cam.height;
    float* img = image.p[v];
    float* tf = tfinal.p[v];
    uint32_t* lp = lastp.p[v];
    float sa = 0.f, sb = 0.f;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = py0 + k * RPK;
        if (px < W && py < H) {
            const size_t o = (size_t)py * W + px;
            const size_t plane = (size_t)W * H;
            const float tk = fabsf(T[k]);
            const float c0 = C0[k] + tk * bg0, c1 = C1[k] + tk * bg1, c2 = C2[k] + tk * bg2;
            img[o] = c0;
            img[plane + o] = c1;
            img[2 * plane + o] = c2;
            tf[o] = tk;
            lp[o] = last[k];
            if constexpr (kL1) {
                const float* __restrict__ g = l1.gt[v];
                float* __restrict__ gr = l1.grad[v];
                const float gs = l1.gscale[v];
                gr[o] = l1_term(c0, g[o], gs, sa, sb);
                gr[plane + o] = l1_term(c1, g[plane + o], gs, sa, sb);
                gr[2 * plane + o] = l1_term(c2, g[2 * plane + o], gs, sa, sb);
            }
        }
    }
    if constexpr (kL1) {  // the tile's sums: lane values in double, added over the wave in a fixed order
        double da = sa, db = sb;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            da += __shfl_xor(da, o);
            db += __shfl_xor(db, o);
        }
        if (lane == 0) {
            l1.part[2 * tile] = da;
            l1.part[2 * tile + 1] = db;
        }
    }
}

// Work distribution: one workgroup per tile.  Without a schedule, in the super-tile order of map_tile.  With a
// schedule (qg_schedule_tiles), each XCD keeps the same tiles, taken heaviest first: workgroup b runs on XCD
// x = b mod 8 and takes the (b div 8)-th tile of x's segment of the order.  Workgroups start in index order,
// so on every XCD the longest tile lists start first and spread over its SIMDs, and the short ones fill in
// behind them, while neighbouring tiles still share the XCD's L2.
struct Sched {
    const uint32_t* seg;    // [16]: start and length of each XCD's segment of the order, or nullptr
    const uint32_t* order;  // [total_tiles]
};

__device__ __forceinline__ int64_t sched_tile(const Sched& sc, const TileMap& tm, const ViewTable& vt) {
    if (!sc.seg) return map_tile(tm, vt, blockIdx.x);
    const uint32_t x = blockIdx.x & 7, k = blockIdx.x >> 3;
    return k < sc.seg[8 + x] ? (int64_t)sc.order[sc.seg[x] + k] : -1;
}

template <int TW, int TH, int BD, bool kL1>
__global__ __launch_bounds__(64) void k_render_fwd(ViewTable vt, const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ ranges, float bg0, float bg1,
                                                   float bg2, ViewPtrsF image, ViewPtrsF tfinal, ViewPtrsU lastp,
                                                   FwdL1 l1, TileMap tm, Sched sc) {
    __shared__ float4 s_a[BD];  // x, y, o, A'
    __shared__ float4 s_b[BD];  // 2B', C', r, g
    __shared__ float s_c[BD];   // b
    __shared__ uint32_t s_pos[BD];  // position of the entry in vals
    const int64_t tile = sched_tile(sc, tm, vt);
    if (tile >= 0)
        fwd_tile<TW, TH, BD, kL1>(vt, vals, ranges, bg0, bg1, bg2, image, tfinal, lastp, l1, tile, s_a, s_b, s_c,
                                  s_pos);
}

// ---- wave64 sums of K values at once: DPP inclusive scans inside each 8-lane half row (row_shr 1, 2, 4,
// interleaved over the K values so consecutive DPP operations never depend on each other), then the eight
// half-row totals go through LDS and are added by the lanes that issue the atomics.  (A fourth DPP step
// would cost the whole wave two instructions per value; the extra four adds run on those few lanes.)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_term(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

// Scans with shifts 1, 2, 4 inside each 16-lane row (zeros shifted in at the row start): afterwards lane l
// holds the sum of the 8 lanes l - 7 .. l of its row that exist, so lane 8h + 7 holds exactly the sum of
// lanes 8h .. 8h + 7.
template <int K>
__device__ __forceinline__ void row_sums(float (&v)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp_term<0x111, 0xf>(v[k]);  // row_shr:1
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp_term<0x112, 0xf>(v[k]);  // row_shr:2
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp_term<0x114, 0xf>(v[k]);  // row_shr:4
}

// Pixel slots of the blend adjoint's second pass that run branch-free (bit k: slot k).  With slot 0 masked
// instead of skipped, the per-entry sums start from registers that always hold slot 0's terms, so the compiler
// needs no copies to zero them for the path that would skip it.
constexpr int kBwdMaskedSlots = 0x1;

template <int TW, int TH, int BD>
__device__ __forceinline__ void bwd_tile(const ViewTable& vt, const uint32_t* __restrict__ vals,
                                         const uint32_t* __restrict__ ranges, float bg0, float bg1, float bg2,
                                         const ViewPtrsCF& tfinal, const ViewPtrsCU& lastp, const ViewPtrsCF& gimage,
                                         float* __restrict__ grad2d, int64_t g2d_view_stride, PairPart pp,
                                         int64_t tile, float4* s_a, float4* s_b, float4* s_c, uint32_t* s_gid,
                                         uint32_t* s_pos, float (*s_red)[12]) {
    constexpr int PPL = TileGeom<TW, TH>::PPL;
    constexpr int RPK = TileGeom<TW, TH>::ROWS_PER_K;
    const int v = view_of_tile(vt, (uint32_t)tile);
    const CamDev& cam = vt.cam[v];
    const int local = (int)(tile - cam.tile_off);
    const int tx = local % cam.grid_w, ty = local / cam.grid_w;
    const int lane = threadIdx.x;
    const int px = tx * TW + (lane % TW);
    const int py0 = ty * TH + lane / TW;
    const float fx = (float)px + 0.5f;
    const float gscale = geom_scale(lane);
    const uint32_t s = ranges[2 * tile];
    const int W = cam.width, H = cam.height;
    const size_t plane = (size_t)W * H;
    // Per pixel: T (walked backwards from T_final), the image gradient G, and SG = sum_ch S_ch G_ch where S is
    // the colour of everything behind the current entry (background included): dL/dalpha_i only needs
    // T_i (c_i . G - SG_{i+1}), and SG_i = SG_{i+1} + alpha_i (c_i . G - SG_{i+1}).
    float T[PPL], SG[PPL], G0[PPL], G1[PPL], G2[PPL], fy[PPL];
    uint32_t last[PPL];
    uint32_t maxlast = s;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = py0 + k * RPK;
        fy[k] = (float)py + 0.5f;
        const bool in = px < W && py < H;
        const size_t o = (size_t)(in ? py : 0) * W + (in ? px : 0);
        T[k] = in ? tfinal.p[v][o] : 1.f;
        last[k] = in ? lastp.p[v][o] : s;
        G0[k] = in ? gimage.p[v][o] : 0.f;
        G1[k] = in ? gimage.p[v][plane + o] : 0.f;
        G2[k] = in ? gimage.p[v][2 * plane + o] : 0.f;
        SG[k] = bg0 * G0[k] + bg1 * G1[k] + bg2 * G2[k];
        maxlast = max(maxlast, last[k]);
    }
    // wave max of last
    for (int o = 32; o >= 1; o >>= 1) maxlast = max(maxlast, (uint32_t)__shfl_xor((int)maxlast, o));
    const float* __restrict__ splat = vt.proj[v].splat;
    float* __restrict__ g2 = grad2d + (int64_t)v * g2d_view_stride;
    // pixel centres of this tile inside the image (the forward's culling test, repeated exactly)
    const float bx0 = (float)(tx * TW) + 0.5f, bx1 = (float)min(tx * TW + TW, W) - 0.5f;
    const float by0 = (float)(ty * TH) + 0.5f, by1 = (float)min(ty * TH + TH, H) - 0.5f;
    for (uint32_t hi = maxlast; hi > s;) {
        const uint32_t lo = hi - s > (uint32_t)BD ? hi - (uint32_t)BD : s;
        int cnt = 0;
#pragma unroll
        for (int q = 0; q < (BD + 63) / 64; ++q) {
            const int slot = q * 64 + lane;
            const uint32_t j = lo + (uint32_t)slot;
            bool hit = false;
            float4 r0, r1, r2;
            uint32_t gid = 0;
            if (slot < BD && j < hi) {
                gid = vals[j];
                const float4* r = reinterpret_cast<const float4*>(splat) + 3 * (size_t)gid;
                r0 = r[0];
                r1 = r[1];
                r2 = r[2];
                hit = tile_hit(r0.x, r0.y, r0.z, r1.x, r1.y, r1.z, bx0, bx1, by0, by1);
            }
            const uint64_t m = __ballot(hit);
            if (hit) {
                const int dst = cnt + (int)__popcll(m & ((1ull << lane) - 1ull));
                s_a[dst] = make_float4(r0.x, r0.y, r0.z, kFold * r1.x);
                s_b[dst] = make_float4(2.f * kFold * r1.y, kFold * r1.z, r2.x, r2.y);
                s_c[dst] = make_float4(r2.z, r1.x, r1.y, r1.z);
                s_gid[dst] = gid;
                s_pos[dst] = j;
            }
            cnt += (int)__popcll(m);
        }
        __syncthreads();
        for (int jj = cnt - 1; jj >= 0; --jj) {
            const uint32_t pos = s_pos[jj];
            const float4 a = s_a[jj];
            const float4 bb = s_b[jj];
            const float4 cc = s_c[jj];
            const float dx = fx - a.x;
            // acc: gx, gy, gA, gB, gC, go, gr, gg, gb
            float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            // the lane's moments sum m, sum m dy, sum m dy^2 over its pixels (dx is the same for all of them)
            float M0 = 0.f, M1 = 0.f, M2 = 0.f;
            // pass 1: alpha and T_i of every pixel; branch-free, and the decisions (entry reached, alpha >= 1/255,
            // clamp) repeat the forward's exactly
            float ekv[PPL], rawv[PPL], alv[PPL], dyv[PPL];
            bool onv[PPL];
            bool hit = false;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                const float dy = fy[k] - a.y;
                const float ek = blend_e(a.w, bb.x, bb.y, dx, dy);
                const float raw = a.z * ek;
                const float al = fminf(kAlphaMax, raw);
                const bool on = pos < last[k] && al >= kAlphaMin;
                hit |= on;
                T[k] = on ? T[k] * __builtin_amdgcn_rcpf(1.f - al) : T[k];
                ekv[k] = ek;
                rawv[k] = raw;
                alv[k] = al;
                dyv[k] = dy;
                onv[k] = on;
            }
            if (__ballot(hit) == 0) continue;
            // pass 2: gradients and the suffix colour, only in the lanes whose pixel is on (an off pixel adds exact
            // zeros).  Slots in kBwdMaskedSlots run in every lane with alpha taken as 0 where the pixel is off; the
            // others branch on the exec mask, so a slot that no lane reaches costs nothing.
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                const bool masked = (kBwdMaskedSlots >> k) & 1;
                if (!masked && !onv[k]) continue;
                const float al = (masked && !onv[k]) ? 0.f : alv[k], dy = dyv[k], Ti = T[k];
                const float w = al * Ti;
                acc[6] = __builtin_fmaf(w, G0[k], acc[6]);
                acc[7] = __builtin_fmaf(w, G1[k], acc[7]);
                acc[8] = __builtin_fmaf(w, G2[k], acc[8]);
                const float cG = __builtin_fmaf(cc.x, G2[k], __builtin_fmaf(bb.w, G1[k], bb.z * G0[k]));
                const float d = cG - SG[k];
                SG[k] = __builtin_fmaf(al, d, SG[k]);
                // geometric part: zero where the 0.99 clamp is active.  With m = alpha dL/dalpha,
                // dL/dq = -m/2 (q = A dx^2 + 2 B dx dy + C dy^2); the constant factors -1/2 and -1 of the
                // conic terms are applied once per entry after the wave sum (kGeomScale).
                const float dLda = (rawv[k] <= kAlphaMax && (!masked || onv[k])) ? Ti * d : 0.f;
                acc[5] = __builtin_fmaf(dLda, ekv[k], acc[5]);
                const float m = al * dLda;
                const float mdy = m * dy;
                M0 += m;
                M1 += mdy;
                M2 = __builtin_fmaf(mdy, dy, M2);
            }
            // the lane's sums of m (A dx + B dy), m (B dx + C dy), m dx^2, m dx dy, m dy^2 (cc.y, cc.z, cc.w = A, B,
            // C of the unfolded conic)
            acc[0] = __builtin_fmaf(cc.z, M1, cc.y * dx * M0);
            acc[1] = __builtin_fmaf(cc.w, M1, cc.z * dx * M0);
            acc[2] = dx * dx * M0;
            acc[3] = dx * M1;
            acc[4] = M2;
            row_sums<9>(acc);
            // the sums are formed here, in all lanes, so that each step is one DPP add (left to itself the
            // compiler moves the last step's adds into the branch below, as a DPP move plus an add)
#pragma unroll
            for (int k = 0; k < 9; ++k) asm volatile("" : "+v"(acc[k]));
            if ((lane & 7) == 7) {
#pragma unroll
                for (int k = 0; k < 9; ++k) s_red[lane >> 3][k] = acc[k];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane < 9) {
                const float val =
                    gscale * (((s_red[0][lane] + s_red[1][lane]) + (s_red[2][lane] + s_red[3][lane])) +
                              ((s_red[4][lane] + s_red[5][lane]) + (s_red[6][lane] + s_red[7][lane])));
                if (pp.part == nullptr) {
                    atomicAdd(g2 + (size_t)s_gid[jj] * QG_GRAD2D_STRIDE + lane, val);
                } else {  // deterministic mode: this (tile, entry)'s sums in its slot, added up later in order
                    const uint32_t gid = s_gid[jj];
                    const int4 r = reinterpret_cast<const int4*>(vt.proj[v].rect)[gid];
                    const uint32_t slot = pp.base[(size_t)v * pp.n + gid] + (uint32_t)((ty - r.y) * (r.z - r.x) + (tx - r.x));
                    if (slot < pp.cap) pp.part[(size_t)slot * kPairPart + lane] = val;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __syncthreads();
        hi = lo;
    }
}

// At most 96 VGPRs, for five waves per SIMD: the kernel is VALU-issue-bound and the extra wave hides the latency
// of its LDS reads and transcendentals better than the registers it costs.
template <int TW, int TH, int BD>
__global__ __launch_bounds__(64, 5) void k_render_bwd(ViewTable vt, const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ ranges, float bg0, float bg1,
                                                   float bg2, ViewPtrsCF tfinal, ViewPtrsCU lastp, ViewPtrsCF gimage,
                                                   float* __restrict__ grad2d, int64_t g2d_view_stride,
                                                   PairPart pp, TileMap tm, Sched sc) {
    __shared__ float4 s_a[BD];  // x, y, o, A'
    __shared__ float4 s_b[BD];  // 2B', C', r, g
    __shared__ float4 s_c[BD];  // b, A, B, C
    __shared__ uint32_t s_gid[BD];
    __shared__ uint32_t s_pos[BD];  // position of the entry in vals
    __shared__ float s_red[8][12];  // half-row totals of the 9 gradient components
    const int64_t tile = sched_tile(sc, tm, vt);
    if (tile >= 0)
        bwd_tile<TW, TH, BD>(vt, vals, ranges, bg0, bg1, bg2, tfinal, lastp, gimage, grad2d, g2d_view_stride, pp, tile,
                             s_a, s_b, s_c, s_gid, s_pos, s_red);
}

// The plain grid's tile order (super-tiles of 4 x 4 tiles) and its size, a multiple of 8 * 16 workgroups.
constexpr int kSuperTile = 4;

TileMap make_tile_map(const ViewTable& vt, int64_t* grid, int64_t* xcd_max = nullptr) {
    TileMap m{};
    m.S = kSuperTile;
    m.V = vt.V;
    int64_t j = 0;
    int64_t per_xcd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int v = 0; v < vt.V; ++v) {
        m.sup_off[v] = (int32_t)j;
        const int gw = vt.cam[v].grid_w, gh = vt.cam[v].grid_h;
        m.sw[v] = (int32_t)ceil_div(gw, kSuperTile);
        const int64_t sh = ceil_div(gh, kSuperTile);
        if (xcd_max) {  // tiles of each XCD: whole super-tiles, plus the clipped ones of the last row and column
            for (int64_t sy = 0; sy < sh; ++sy)
                for (int64_t sx = 0; sx < m.sw[v]; ++sx)
                    per_xcd[(j + sy * m.sw[v] + sx) & 7] += std::min<int64_t>(kSuperTile, gw - sx * kSuperTile) *
                                                             std::min<int64_t>(kSuperTile, gh - sy * kSuperTile);
        }
        j += (int64_t)m.sw[v] * sh;
    }
    m.sup_off[vt.V] = (int32_t)j;
    m.supers = j;
    *grid = ceil_div(j, 8) * 8 * kSuperTile * kSuperTile;
    if (xcd_max) *xcd_max = *std::max_element(per_xcd, per_xcd + 8);
    return m;
}

inline Sched make_sched(const qg_tiling& t) {
    Sched sc = {nullptr, nullptr};
    if (t.schedule) {
        sc.seg = t.schedule;
        sc.order = t.schedule + QG_SCHEDULE_HEADER_WORDS;
    }
    return sc;
}

template <int TW, int TH, int BD>
qg_status launch_fwd_t(const ViewTable& vt, const qg_tiling& tiling, const uint32_t* vals, const uint32_t* ranges,
                       const float* bg, const ViewPtrsF& img, const ViewPtrsF& tf, const ViewPtrsU& lp,
                       const FwdL1* l1, hipStream_t s) {
    int64_t grid = 0, xcd_max = 0;
    const TileMap tm = make_tile_map(vt, &grid, tiling.schedule ? &xcd_max : nullptr);
    const Sched sc = make_sched(tiling);
    if (sc.seg) grid = 8 * xcd_max;
    if (l1) {
        QG_TIMED("render_fwd_l1", s);
        k_render_fwd<TW, TH, BD, true><<<(unsigned)grid, 64, 0, s>>>(vt, vals, ranges, bg[0], bg[1], bg[2], img, tf,
                                                                      lp, *l1, tm, sc);
    } else {
        QG_TIMED("render_fwd", s);
        k_render_fwd<TW, TH, BD, false><<<(unsigned)grid, 64, 0, s>>>(vt, vals, ranges, bg[0], bg[1], bg[2], img, tf,
                                                                       lp, FwdL1{}, tm, sc);
    }
    QG_LAUNCH_CHECK("qg_render_fwd");
    return QG_OK;
}

template <int TW, int TH, int BD>
qg_status launch_bwd_t(const ViewTable& vt, const qg_tiling& tiling, const uint32_t* vals, const uint32_t* ranges,
                       const float* bg, const ViewPtrsCF& tf, const ViewPtrsCU& lp, const ViewPtrsCF& gi,
                       float* grad2d, int64_t stride, PairPart pp, hipStream_t s) {
    int64_t grid = 0, xcd_max = 0;
    const TileMap tm = make_tile_map(vt, &grid, tiling.schedule ? &xcd_max : nullptr);
    const Sched sc = make_sched(tiling);
    if (sc.seg) grid = 8 * xcd_max;
    {
        QG_TIMED("blend_bwd", s);
        k_render_bwd<TW, TH, BD><<<(unsigned)grid, 64, 0, s>>>(vt, vals, ranges, bg[0], bg[1], bg[2], tf, lp, gi,
                                                                grad2d, stride, pp, tm, sc);
    }
    QG_LAUNCH_CHECK("qg_render_bwd");
    return QG_OK;
}

template <int TW, int TH>
qg_status launch_fwd_b(const ViewTable& vt, const qg_tiling& t, const uint32_t* vals, const uint32_t* ranges,
                       const float* bg, const ViewPtrsF& img, const ViewPtrsF& tf, const ViewPtrsU& lp,
                       const FwdL1* l1, hipStream_t s) {
    if (t.batch == 32) return launch_fwd_t<TW, TH, 32>(vt, t, vals, ranges, bg, img, tf, lp, l1, s);
    if (t.batch == 128) return launch_fwd_t<TW, TH, 128>(vt, t, vals, ranges, bg, img, tf, lp, l1, s);
    if (t.batch == 256) return launch_fwd_t<TW, TH, 256>(vt, t, vals, ranges, bg, img, tf, lp, l1, s);
    return launch_fwd_t<TW, TH, 64>(vt, t, vals, ranges, bg, img, tf, lp, l1, s);
}

template <int TW, int TH>
qg_status launch_bwd_b(const ViewTable& vt, const qg_tiling& t, const uint32_t* vals, const uint32_t* ranges,
                       const float* bg, const ViewPtrsCF& tf, const ViewPtrsCU& lp, const ViewPtrsCF& gi,
                       float* grad2d, int64_t stride, PairPart pp, hipStream_t s) {
    if (t.batch == 32) return launch_bwd_t<TW, TH, 32>(vt, t, vals, ranges, bg, tf, lp, gi, grad2d, stride, pp, s);
    if (t.batch == 128) return launch_bwd_t<TW, TH, 128>(vt, t, vals, ranges, bg, tf, lp, gi, grad2d, stride, pp, s);
    if (t.batch == 256) return launch_bwd_t<TW, TH, 256>(vt, t, vals, ranges, bg, tf, lp, gi, grad2d, stride, pp, s);
    return launch_bwd_t<TW, TH, 64>(vt, t, vals, ranges, bg, tf, lp, gi, grad2d, stride, pp, s);
}

qg_status launch_fwd(const ViewTable& vt, const qg_tiling& t, const uint32_t* vals, const uint32_t* ranges,
                     const float* bg, const ViewPtrsF& img, const ViewPtrsF& tf, const ViewPtrsU& lp, const FwdL1* l1,
                     hipStream_t s) {
    if (t.tile_w == 16) return launch_fwd_b<16, 16>(vt, t, vals, ranges, bg, img, tf, lp, l1, s);
    if (t.tile_w == 8) return launch_fwd_b<8, 8>(vt, t, vals, ranges, bg, img, tf, lp, l1, s);
    return launch_fwd_b<32, 8>(vt, t, vals, ranges, bg, img, tf, lp, l1, s);
}

qg_status launch_bwd_tiles(const ViewTable& vt, const qg_tiling& t, const uint32_t* vals, const uint32_t* ranges,
                           const float* bg, const ViewPtrsCF& tf, const ViewPtrsCU& lp, const ViewPtrsCF& gi,
                           float* grad2d, int64_t stride, PairPart pp, hipStream_t s) {
    if (t.tile_w == 16) return launch_bwd_b<16, 16>(vt, t, vals, ranges, bg, tf, lp, gi, grad2d, stride, pp, s);
    if (t.tile_w == 8) return launch_bwd_b<8, 8>(vt, t, vals, ranges, bg, tf, lp, gi, grad2d, stride, pp, s);
    return launch_bwd_b<32, 8>(vt, t, vals, ranges, bg, tf, lp, gi, grad2d, stride, pp, s);
}

// Deterministic mode.  Slot bases: the exclusive scan of the tile counts of the (view, Gaussian) items, in three
// steps (block sums, one-block scan of the block sums, block-local scans).
constexpr int kDetScanBlock = 1024;

__global__ __launch_bounds__(kDetScanBlock) void k_det_base_sums(int64_t items, int64_t n, ViewTable vt,
                                                                 uint32_t* __restrict__ bsum) {
    __shared__ uint32_t s_w[kDetScanBlock / 64];
    const int64_t item = (int64_t)blockIdx.x * kDetScanBlock + threadIdx.x;
    uint32_t c = 0;
    if (item < items) {
        const int v = (int)(item / n);
        c = (uint32_t)max(vt.proj[v].ntiles[item - (int64_t)v * n], 0);
    }
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
    if (__lane_id() == 0) s_w[threadIdx.x / 64] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kDetScanBlock / 64; ++k) t += s_w[k];
        bsum[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kDetScanBlock) void k_det_base_scan(int64_t nb, uint32_t* __restrict__ bsum) {
    __shared__ uint32_t s[kDetScanBlock];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kDetScanBlock) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t x = b < nb ? bsum[b] : 0u;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < kDetScanBlock; o <<= 1) {
            const uint32_t add = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (b < nb) bsum[b] = carry + s[threadIdx.x] - x;
        carry += s[kDetScanBlock - 1];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kDetScanBlock) void k_det_base(int64_t items, int64_t n, ViewTable vt,
                                                            const uint32_t* __restrict__ bsum,
                                                            uint32_t* __restrict__ base) {
    __shared__ uint32_t s[kDetScanBlock];
    const int64_t item = (int64_t)blockIdx.x * kDetScanBlock + threadIdx.x;
    uint32_t c = 0;
    if (item < items) {
        const int v = (int)(item / n);
        c = (uint32_t)max(vt.proj[v].ntiles[item - (int64_t)v * n], 0);
    }
    s[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < kDetScanBlock; o <<= 1) {
        const uint32_t add = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    if (item < items) base[item] = bsum[blockIdx.x] + s[threadIdx.x] - c;
}

// Second pass: the 2D gradient record of (view v, Gaussian i) is the sum of its slots in order (the tiles of its
// rectangle, row-major): the same bits on every run.
__global__ __launch_bounds__(256) void k_det_gather(int64_t n, ViewTable vt, PairPart pp, float* __restrict__ grad2d,
                                                    int64_t stride) {
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= n * vt.V) return;
    const int v = (int)(item / n);
    const int64_t i = item - (int64_t)v * n;
    const int32_t k = vt.proj[v].ntiles[i];
    if (k <= 0) return;
    float acc[kPairPart];
#pragma unroll
    for (int c = 0; c < kPairPart; ++c) acc[c] = 0.f;
    const uint32_t b = pp.base[item];
    const uint32_t e = (uint32_t)min<uint64_t>((uint64_t)b + (uint64_t)k, pp.cap);
    for (uint32_t sl = b; sl < e; ++sl) {
#pragma unroll
        for (int c = 0; c < kPairPart; ++c) acc[c] += pp.part[(size_t)sl * kPairPart + c];
    }
    float* rec = grad2d + (int64_t)v * stride + (size_t)i * QG_GRAD2D_STRIDE;
#pragma unroll
    for (int c = 0; c < kPairPart; ++c) rec[c] = acc[c];
}

// The blend adjoint into the zeroed 2D gradient records: float atomics across tiles, or, with a pair-partial
// buffer (deterministic mode), per-(tile, entry) sums and then a fixed-order gather.
qg_status launch_bwd(const ViewTable& vt, const qg_tiling& t, const uint32_t* vals, const uint32_t* ranges,
                     const float* bg, const ViewPtrsCF& tf, const ViewPtrsCU& lp, const ViewPtrsCF& gi, float* grad2d,
                     int64_t stride, int64_t n, PairPart pp, hipStream_t s) {
    if (pp.part && n > 0) {
        qg_status st = qg_zero(pp.part, (int64_t)pp.cap * kPairPart * 4, s);
        if (st != QG_OK) return st;
        const int64_t items = n * vt.V, nb = ceil_div(items, kDetScanBlock);
        uint32_t* bsum = pp.base + align_up((size_t)items * 4) / 4;
        QG_TIMED("blend_bwd_slots", s);
        k_det_base_sums<<<(unsigned)nb, kDetScanBlock, 0, s>>>(items, n, vt, bsum);
        k_det_base_scan<<<1, kDetScanBlock, 0, s>>>(nb, bsum);
        k_det_base<<<(unsigned)nb, kDetScanBlock, 0, s>>>(items, n, vt, bsum, pp.base);
    }
    qg_status st = launch_bwd_tiles(vt, t, vals, ranges, bg, tf, lp, gi, grad2d, stride, pp, s);
    if (st != QG_OK || !pp.part || n == 0) return st;
    {
        QG_TIMED("blend_bwd_gather", s);
        k_det_gather<<<(unsigned)ceil_div(n * vt.V, 256), 256, 0, s>>>(n, vt, pp, grad2d, stride);
    }
    QG_LAUNCH_CHECK("deterministic gather");
    return QG_OK;
}

// ---- heaviest-first tile order, per XCD ----------------------------------------------------------------
// Every tile keeps the XCD that the super-tile order gives it.  Within each XCD the tiles are ordered by the
// length of their entry list, heaviest first, on a log scale (float exponent and the top three mantissa bits, 8
// buckets per octave; order inside a bucket is arbitrary: every tile is blended by exactly one wave either way).
// The sort key is (XCD, bucket).  Schedule layout: 8 segment starts, 8 segment lengths, kSchedKeys key words,
// then the order.  Up to kSchedOneBlock tiles one workgroup builds it in LDS; above, a histogram, a scan and a
// scatter kernel go through the key words.
constexpr int kSchedBuckets = 512;
constexpr int kSchedKeys = 8 * kSchedBuckets;
constexpr int64_t kSchedOneBlock = 1 << 18;
static_assert(QG_SCHEDULE_HEADER_WORDS == 16 + kSchedKeys, "schedule header: 8 starts, 8 lengths, the key words");

__device__ __forceinline__ uint32_t sched_bucket(uint32_t len) {
    if (len == 0) return kSchedBuckets - 1;
    const uint32_t key = (__float_as_uint((float)len) >> 20) - (127u << 3);  // 8 * log2(len), >= 0
    return (uint32_t)(kSchedBuckets - 2) - min(key, (uint32_t)(kSchedBuckets - 2));
}

__device__ __forceinline__ uint32_t sched_key(const TileMap& m, const ViewTable& vt, const uint32_t* __restrict__ ranges,
                                              int64_t t) {
    const int v = view_of_tile(vt, (uint32_t)t);
    const CamDev& c = vt.cam[v];
    const int local = (int)((uint32_t)t - c.tile_off);
    return xcd_of_tile(m, vt, v, local % c.grid_w, local / c.grid_w) * kSchedBuckets +
           sched_bucket(ranges[2 * t + 1] - ranges[2 * t]);
}

// In-place exclusive scan of kSchedKeys counts by a workgroup of 1024 threads (four consecutive keys each), and
// the 8 XCD segments' starts and lengths into seg[0..15].  `total` is the sum of the counts.
__device__ __forceinline__ void sched_scan_keys(uint32_t* h, uint32_t* s_w, uint32_t* seg, uint32_t total) {
    const int k = threadIdx.x, w = k / 64, lane = __lane_id();
    uint32_t c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = h[4 * k + i];
    const uint32_t sum = c[0] + c[1] + c[2] + c[3];
    uint32_t x = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t run = x - sum;
    for (int j = 0; j < w; ++j) run += s_w[j];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h[4 * k + i] = run;
        run += c[i];
    }
    __syncthreads();
    if (k < 8) {
        const uint32_t st = h[k * kSchedBuckets];
        seg[k] = st;
        seg[8 + k] = (k < 7 ? h[(k + 1) * kSchedBuckets] : total) - st;
    }
    __syncthreads();
}

// The whole schedule in one workgroup of 1024 threads: key histogram, scan and scatter in LDS.  Up to
// kSchedKeep keys per thread (8192 tiles) are kept in registers between the histogram and the scatter;
// beyond, the scatter computes them again.
constexpr int kSchedKeep = 8;

__global__ __launch_bounds__(1024) void k_sched_one(int64_t total, ViewTable vt, TileMap tm,
                                                    const uint32_t* __restrict__ ranges, uint32_t* __restrict__ sched) {
    __shared__ uint32_t s_h[kSchedKeys];
    __shared__ uint32_t s_w[1024 / 64];
    for (int k = threadIdx.x; k < kSchedKeys; k += blockDim.x) s_h[k] = 0;
    __syncthreads();
    uint32_t key[kSchedKeep];
#pragma unroll
    for (int r = 0; r < kSchedKeep; ++r) {
        const int64_t t = threadIdx.x + (int64_t)r * blockDim.x;
        key[r] = t < total ? sched_key(tm, vt, ranges, t) : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSchedKeep; ++r) {
        const int64_t t = threadIdx.x + (int64_t)r * blockDim.x;
        if (t < total) atomicAdd(&s_h[key[r]], 1u);
    }
    for (int64_t t = threadIdx.x + (int64_t)kSchedKeep * blockDim.x; t < total; t += blockDim.x)
        atomicAdd(&s_h[sched_key(tm, vt, ranges, t)], 1u);
    __syncthreads();
    sched_scan_keys(s_h, s_w, sched, (uint32_t)total);
    uint32_t* order = sched + QG_SCHEDULE_HEADER_WORDS;
#pragma unroll
    for (int r = 0; r < kSchedKeep; ++r) {
        const int64_t t = threadIdx.x + (int64_t)r * blockDim.x;
        if (t < total) order[atomicAdd(&s_h[key[r]], 1u)] = (uint32_t)t;
    }
    for (int64_t t = threadIdx.x + (int64_t)kSchedKeep * blockDim.x; t < total; t += blockDim.x)
        order[atomicAdd(&s_h[sched_key(tm, vt, ranges, t)], 1u)] = (uint32_t)t;
}

__global__ void k_sched_clear(uint32_t* __restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < QG_SCHEDULE_HEADER_WORDS) w[i] = 0u;
}

__global__ __launch_bounds__(256) void k_sched_hist(int64_t total, ViewTable vt, TileMap tm,
                                                    const uint32_t* __restrict__ ranges, uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_h[kSchedKeys];
    for (int k = threadIdx.x; k < kSchedKeys; k += blockDim.x) s_h[k] = 0;
    __syncthreads();
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&s_h[sched_key(tm, vt, ranges, t)], 1u);
    __syncthreads();
    for (int k = threadIdx.x; k < kSchedKeys; k += blockDim.x)
        if (s_h[k]) atomicAdd(&hist[k], s_h[k]);
}

__global__ __launch_bounds__(1024) void k_sched_scan(int64_t total, uint32_t* __restrict__ sched) {
    __shared__ uint32_t s_w[1024 / 64];
    sched_scan_keys(sched + 16, s_w, sched, (uint32_t)total);
}

__global__ void k_sched_scatter(int64_t total, ViewTable vt, TileMap tm, const uint32_t* __restrict__ ranges,
                                uint32_t* __restrict__ sched) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const uint32_t pos = atomicAdd(&sched[16 + sched_key(tm, vt, ranges, t)], 1u);
    sched[QG_SCHEDULE_HEADER_WORDS + pos] = (uint32_t)t;
}

// ---- adaptive masked training (Sec. 3.3, "Adaptive Masked Training") -------------------------------
struct ViewPtrsB8 {
    uint8_t* p[QG_MAX_VIEWS];
};
struct ViewPtrsCB8 {
    const uint8_t* p[QG_MAX_VIEWS];
};

// Gaussians whose score ||(sx d_x, sy d_y)|| exceeds t_d are dynamic; decided in double precision.
__global__ void k_dyn_flags(int64_t n, const float* __restrict__ d, double sx, double sy, double t_d,
                            uint8_t* __restrict__ dyn) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = (double)d[i] * sx, y = (double)d[n + i] * sy;
    dyn[i] = sqrt(x * x + y * y) > t_d ? 1 : 0;
}

// Image mask of each view: the pixels that a render of the dynamic Gaussians alone reaches.  In such a
// render the first splat with alpha >= 1/255 at a pixel always contributes (T' >= 0.01 > 1e-4 after it), so
// the mask is the union over the tile's dynamic entries of the blend forward's own alpha test, evaluated
// with the same operands.  Entries are staged 64 at a time; only the dynamic ones are kept.
template <int TW, int TH>
__global__ __launch_bounds__(64) void k_dyn_mask(ViewTable vt, const uint32_t* __restrict__ vals,
                                                 const uint32_t* __restrict__ ranges, const uint8_t* __restrict__ dyn,
                                                 ViewPtrsB8 mask, int64_t per_xcd) {
    constexpr int PPL = TileGeom<TW, TH>::PPL;
    constexpr int RPK = TileGeom<TW, TH>::ROWS_PER_K;
    __shared__ float4 s_a[64];   // x, y, opacity, A'
    __shared__ float2 s_b[64];   // 2B', C'
    const int64_t tile = xcd_tile(blockIdx.x, per_xcd);
    if (tile >= vt.total_tiles) return;
    const int v = view_of_tile(vt, (uint32_t)tile);
    const CamDev& cam = vt.cam[v];
    const int local = (int)(tile - cam.tile_off);
    const int tx = local % cam.grid_w, ty = local / cam.grid_w;
    const int lane = threadIdx.x;
    const int px = tx * TW + (lane % TW);
    const int py0 = ty * TH + lane / TW;
    const float fx = (float)px + 0.5f;
    float fy[PPL];
    bool hit[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        fy[k] = (float)(py0 + k * RPK) + 0.5f;
        hit[k] = false;
    }
    const uint32_t b0 = ranges[2 * tile], e = ranges[2 * tile + 1];
    const float* __restrict__ splat = vt.proj[v].splat;
    for (uint32_t b = b0; b < e; b += 64) {
        const uint32_t j = b + (uint32_t)lane;
        bool keep = false;
        float4 r0, r1;
        if (j < e) {
            const uint32_t gid = vals[j];
            if (dyn[gid]) {
                const float4* r = reinterpret_cast<const float4*>(splat) + 3 * (size_t)gid;
                r0 = r[0];
                r1 = r[1];
                keep = true;
            }
        }
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int dst = (int)__popcll(m & ((1ull << lane) - 1ull));
            s_a[dst] = make_float4(r0.x, r0.y, r0.z, kFold * r1.x);
            s_b[dst] = make_float2(2.f * kFold * r1.y, kFold * r1.z);
        }
        __syncthreads();
        const int cnt = (int)__popcll(m);
        for (int jj = 0; jj < cnt; ++jj) {
            const float4 a = s_a[jj];
            const float2 bb = s_b[jj];
            const float dx = fx - a.x;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                const float dy = fy[k] - a.y;
                const float raw = a.z * blend_e(a.w, bb.x, bb.y, dx, dy);
                hit[k] = hit[k] || fminf(kAlphaMax, raw) >= kAlphaMin;
            }
        }
        __syncthreads();
        bool all = true;
#pragma unroll
        for (int k = 0; k < PPL; ++k) all = all && hit[k];
        if (__ballot(!all) == 0) break;
    }
    uint8_t* out = mask.p[v];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = py0 + k * RPK;
        if (px < cam.width && py < cam.height) out[(size_t)py * cam.width + px] = hit[k] ? 1 : 0;
    }
}

// Box dilation, separable: out[y][x] = 1 if in has a set pixel at x + [lo, hi] (rows) or y + [lo, hi]
// (columns), clipped to the image.
__global__ void k_dilate_rows(const uint8_t* __restrict__ in, uint8_t* __restrict__ out, int W, int H, int lo,
                              int hi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)W * H) return;
    const int x = (int)(i % W);
    const uint8_t* row = in + (i - x);
    const int x0 = max(0, x + lo), x1 = min(W - 1, x + hi);
    uint8_t any = 0;
    for (int xx = x0; xx <= x1; ++xx) any |= row[xx];
    out[i] = any ? 1 : 0;
}

__global__ void k_dilate_cols(const uint8_t* __restrict__ in, uint8_t* __restrict__ out, int W, int H, int lo,
                              int hi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)W * H) return;
    const int x = (int)(i % W), y = (int)(i / W);
    const int y0 = max(0, y + lo), y1 = min(H - 1, y + hi);
    uint8_t any = 0;
    for (int yy = y0; yy <= y1; ++yy) any |= in[(size_t)yy * W + x];
    out[i] = any ? 1 : 0;
}

// Tile t is rendered in a masked iteration if its pixels (inside the image) include a set dilated pixel.
__global__ __launch_bounds__(64) void k_tile_flags(ViewTable vt, ViewPtrsCB8 dil, int TW, int TH,
                                                   uint8_t* __restrict__ flags) {
    const int64_t tile = blockIdx.x;
    if (tile >= vt.total_tiles) return;
    const int v = view_of_tile(vt, (uint32_t)tile);
    const CamDev& cam = vt.cam[v];
    const int local = (int)(tile - cam.tile_off);
    const int tx = local % cam.grid_w, ty = local / cam.grid_w;
    bool any = false;
    for (int q = threadIdx.x; q < TW * TH; q += 64) {
        const int x = tx * TW + q % TW, y = ty * TH + q / TW;
        if (x < cam.width && y < cam.height && dil.p[v][(size_t)y * cam.width + x]) any = true;
    }
    const uint64_t m = __ballot(any);
    if (threadIdx.x == 0) flags[tile] = m ? 1 : 0;
}

// A tile that is not rendered gets an empty range [start, start): the blend forward then writes the
// background there and the adjoint adds nothing.
__global__ void k_mask_ranges(int64_t total, uint32_t* __restrict__ ranges, const uint8_t* __restrict__ flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < total && !flags[t]) ranges[2 * t + 1] = ranges[2 * t];
}

template <int TW, int TH>
qg_status launch_dyn_mask(const ViewTable& vt, const uint32_t* vals, const uint32_t* ranges, const uint8_t* dyn,
                          const ViewPtrsB8& mask, hipStream_t s) {
    const int64_t per = ceil_div(vt.total_tiles, 8);
    {
        QG_TIMED("dynamic_mask", s);
        k_dyn_mask<TW, TH><<<(unsigned)(per * 8), 64, 0, s>>>(vt, vals, ranges, dyn, mask, per);
    }
    QG_LAUNCH_CHECK("qg_dynamic_mask");
    return QG_OK;
}

}  // namespace

qg_status blend_bwd_launch(const ViewTable& vt, qg_tiling tiling, const uint32_t* vals, const uint32_t* ranges,
                           const float* bg, const float* const* T_final, const uint32_t* const* last,
                           const float* const* grad_image, float* grad2d, int64_t stride, int64_t n, PairPart pp,
                           hipStream_t s) {
    ViewPtrsCF tf = {}, gi = {};
    ViewPtrsCU lp = {};
    for (int v = 0; v < vt.V; ++v) {
        tf.p[v] = T_final[v];
        lp.p[v] = last[v];
        gi.p[v] = grad_image[v];
    }
    return launch_bwd(vt, tiling, vals, ranges, bg, tf, lp, gi, grad2d, stride, n, pp, s);
}

}  // namespace qg

using namespace qg;

extern "C" qg_status qg_render_fwd(const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                                   const uint32_t* vals, const uint32_t* tile_ranges, const float* bg,
                                   float* const* image, float* const* T_final, uint32_t* const* last,
                                   qg_stream stream) {
    clear_error();
    ViewTable vt;
    if (!make_view_table(cams, proj, V, tiling, true, &vt)) return QG_ERR_ARG;
    QG_REQUIRE(tile_ranges && bg && image && T_final && last, "a required pointer is NULL");
    ViewPtrsF img = {}, tf = {};
    ViewPtrsU lp = {};
    for (int v = 0; v < V; ++v) {
        QG_REQUIRE(image[v] && T_final[v] && last[v], "view %d: an output pointer is NULL", v);
        img.p[v] = image[v];
        tf.p[v] = T_final[v];
        lp.p[v] = last[v];
    }
    return launch_fwd(vt, tiling, vals, tile_ranges, bg, img, tf, lp, nullptr, (hipStream_t)stream);
}

extern "C" qg_status qg_render_fwd_l1(const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                                      const uint32_t* vals, const uint32_t* tile_ranges, const float* bg,
                                      float* const* image, float* const* T_final, uint32_t* const* last,
                                      const float* const* gt, const float* scale, float* const* grad_image,
                                      double* partials, qg_stream stream) {
    clear_error();
    ViewTable vt;
    if (!make_view_table(cams, proj, V, tiling, true, &vt)) return QG_ERR_ARG;
    QG_REQUIRE(tile_ranges && bg && image && T_final && last && gt && scale && grad_image && partials,
               "a required pointer is NULL");
    ViewPtrsF img = {}, tf = {};
    ViewPtrsU lp = {};
    FwdL1 l1 = {};
    for (int v = 0; v < V; ++v) {
        QG_REQUIRE(image[v] && T_final[v] && last[v] && gt[v] && grad_image[v], "view %d: a pointer is NULL", v);
        QG_REQUIRE(std::isfinite(scale[v]), "view %d: scale is not finite", v);
        img.p[v] = image[v];
        tf.p[v] = T_final[v];
        lp.p[v] = last[v];
        l1.gt[v] = gt[v];
        l1.grad[v] = grad_image[v];
        const int64_t count = 3ll * cams[v].width * cams[v].height;
        l1.gscale[v] = scale[v] / (float)count;  // as qg_l1_loss over the view's 3 H W values
    }
    l1.part = partials;
    return launch_fwd(vt, tiling, vals, tile_ranges, bg, img, tf, lp, &l1, (hipStream_t)stream);
}

extern "C" size_t qg_render_bwd_workspace_size(int64_t n, int32_t V) {
    if (n < 0 || V < 1) return 0;
    return align_up((size_t)V * (size_t)(n > 0 ? n : 1) * QG_GRAD2D_STRIDE * sizeof(float));
}

extern "C" qg_status qg_render_bwd(int64_t n, int64_t ld, const float* attrs, int32_t sh_degree,
                                   const qg_camera* cams, int32_t V, qg_tiling tiling, float dilation,
                                   const qg_projected* proj, const uint32_t* vals, const uint32_t* tile_ranges,
                                   const float* bg, const float* const* T_final, const uint32_t* const* last,
                                   const float* const* grad_image, float* grad_attrs, float* grad_xy_abs,
                                   float* const* grad_xy, void* ws, size_t ws_bytes, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n && n < (1ll << 31), "n=%lld ld=%lld invalid", (long long)n, (long long)ld);
    QG_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "sh_degree=%d outside [0, 3]", sh_degree);
    QG_REQUIRE(dilation >= 0.f, "dilation < 0");
    ViewTable vt;
    if (!make_view_table(cams, proj, V, tiling, true, &vt)) return QG_ERR_ARG;
    QG_REQUIRE(tile_ranges && bg && T_final && last && grad_image, "a required pointer is NULL");
    QG_REQUIRE(n == 0 || (attrs && grad_attrs), "attrs/grad_attrs NULL");
    const size_t need = qg_render_bwd_workspace_size(n, V);
    QG_REQUIRE(ws && ws_bytes >= need, "workspace too small: %zu < %zu", ws_bytes, need);
    PairPart pp{nullptr, 0, nullptr, n};
    if (deterministic_mode()) {
        qg_status st = det_layout((char*)ws + need, ws_bytes - need, n, V, nullptr, &pp);
        if (st != QG_OK) return st;
    }
    ViewPtrsCF tf = {}, gi = {};
    ViewPtrsCU lp = {};
    for (int v = 0; v < V; ++v) {
        QG_REQUIRE(T_final[v] && last[v] && grad_image[v], "view %d: an input pointer is NULL", v);
        tf.p[v] = T_final[v];
        lp.p[v] = last[v];
        gi.p[v] = grad_image[v];
    }
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    float* grad2d = (float*)ws;
    const int64_t stride = n * QG_GRAD2D_STRIDE;
    qg_status st = qg_zero(grad2d, (int64_t)V * stride * 4, stream);
    if (st != QG_OK) return st;
    st = launch_bwd(vt, tiling, vals, tile_ranges, bg, tf, lp, gi, grad2d, stride, n, pp, s);
    if (st != QG_OK) return st;
    return project_bwd_launch(n, ld, attrs, sh_degree, vt, dilation, grad2d, stride, grad_attrs, grad_xy_abs,
                              grad_xy, s);
}

extern "C" int64_t qg_schedule_words(int64_t total_tiles) {
    if (total_tiles < 0) return -1;
    return QG_SCHEDULE_HEADER_WORDS + total_tiles;
}

extern "C" qg_status qg_schedule_tiles(const qg_camera* cams, int32_t V, qg_tiling tiling, const uint32_t* tile_ranges,
                                       uint32_t* schedule, int64_t schedule_words, qg_stream stream) {
    clear_error();
    ViewTable vt;
    if (!make_view_table(cams, nullptr, V, tiling, false, &vt)) return QG_ERR_ARG;
    const int64_t total_tiles = vt.total_tiles;
    QG_REQUIRE(total_tiles >= 1, "no tiles");
    QG_REQUIRE(tile_ranges && schedule, "a pointer is NULL");
    QG_REQUIRE(schedule_words >= qg_schedule_words(total_tiles), "schedule buffer too small: %lld < %lld words",
               (long long)schedule_words, (long long)qg_schedule_words(total_tiles));
    int64_t grid_unused = 0;
    const TileMap tm = make_tile_map(vt, &grid_unused);
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("schedule", s);
        if (total_tiles <= kSchedOneBlock) {
            k_sched_one<<<1, 1024, 0, s>>>(total_tiles, vt, tm, tile_ranges, schedule);
        } else {
            const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total_tiles, 256), 1024);
            k_sched_clear<<<(unsigned)ceil_div(QG_SCHEDULE_HEADER_WORDS, 256), 256, 0, s>>>(schedule);
            k_sched_hist<<<grid, 256, 0, s>>>(total_tiles, vt, tm, tile_ranges, schedule + 16);
            k_sched_scan<<<1, 1024, 0, s>>>(total_tiles, schedule);
            k_sched_scatter<<<(unsigned)ceil_div(total_tiles, 256), 256, 0, s>>>(total_tiles, vt, tm, tile_ranges,
                                                                                 schedule);
        }
    }
    QG_LAUNCH_CHECK("qg_schedule_tiles");
    return QG_OK;
}

extern "C" qg_status qg_dynamic_flags(int64_t n, const float* d, double sx, double sy, double t_d, uint8_t* dynamic,
                                      qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0, "n < 0");
    QG_REQUIRE(sx > 0.0 && sy > 0.0 && t_d >= 0.0, "need sx, sy > 0 and t_d >= 0");
    if (n == 0) return QG_OK;
    QG_REQUIRE(d && dynamic, "a pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    k_dyn_flags<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, d, sx, sy, t_d, dynamic);
    QG_LAUNCH_CHECK("qg_dynamic_flags");
    return QG_OK;
}

extern "C" qg_status qg_dynamic_mask(const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                                     const uint32_t* vals, const uint32_t* tile_ranges, const uint8_t* dynamic,
                                     uint8_t* const* mask, qg_stream stream) {
    clear_error();
    ViewTable vt;
    if (!make_view_table(cams, proj, V, tiling, true, &vt)) return QG_ERR_ARG;
    QG_REQUIRE(tile_ranges && dynamic && mask, "a required pointer is NULL");
    ViewPtrsB8 mp = {};
    for (int v = 0; v < V; ++v) {
        QG_REQUIRE(mask[v], "view %d: mask is NULL", v);
        mp.p[v] = mask[v];
    }
    hipStream_t s = (hipStream_t)stream;
    if (tiling.tile_w == 16) return launch_dyn_mask<16, 16>(vt, vals, tile_ranges, dynamic, mp, s);
    if (tiling.tile_w == 8) return launch_dyn_mask<8, 8>(vt, vals, tile_ranges, dynamic, mp, s);
    return launch_dyn_mask<32, 8>(vt, vals, tile_ranges, dynamic, mp, s);
}

extern "C" qg_status qg_dilate_mask(const qg_camera* cams, int32_t V, qg_tiling tiling, int32_t k,
                                    const uint8_t* const* mask, uint8_t* const* tmp, uint8_t* const* dilated,
                                    uint8_t* tile_flags, qg_stream stream) {
    clear_error();
    ViewTable vt;
    if (!make_view_table(cams, nullptr, V, tiling, false, &vt)) return QG_ERR_ARG;
    QG_REQUIRE(k >= 1 && k <= 1024, "k=%d outside [1, 1024]", k);
    QG_REQUIRE(mask && tmp && dilated && tile_flags, "a required pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int lo = -(k / 2), hi = k - 1 - k / 2;
    ViewPtrsCB8 dp = {};
    for (int v = 0; v < V; ++v) {
        QG_REQUIRE(mask[v] && tmp[v] && dilated[v], "view %d: a buffer is NULL", v);
        QG_REQUIRE(mask[v] != tmp[v] && tmp[v] != dilated[v], "view %d: tmp must differ from mask and dilated", v);
        const int W = cams[v].width, H = cams[v].height;
        const unsigned grid = (unsigned)ceil_div((int64_t)W * H, 256);
        k_dilate_rows<<<grid, 256, 0, s>>>(mask[v], tmp[v], W, H, lo, hi);
        k_dilate_cols<<<grid, 256, 0, s>>>(tmp[v], dilated[v], W, H, lo, hi);
        dp.p[v] = dilated[v];
    }
    k_tile_flags<<<(unsigned)vt.total_tiles, 64, 0, s>>>(vt, dp, tiling.tile_w, tiling.tile_h, tile_flags);
    QG_LAUNCH_CHECK("qg_dilate_mask");
    return QG_OK;
}

extern "C" qg_status qg_mask_tile_ranges(int64_t total_tiles, uint32_t* tile_ranges, const uint8_t* tile_flags,
                                         qg_stream stream) {
    clear_error();
    QG_REQUIRE(total_tiles >= 1 && total_tiles < (1ll << 32), "total_tiles=%lld outside [1, 2^32)",
               (long long)total_tiles);
    QG_REQUIRE(tile_ranges && tile_flags, "a pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("mask_ranges", s);
        k_mask_ranges<<<(unsigned)ceil_div(total_tiles, 256), 256, 0, s>>>(total_tiles, tile_ranges, tile_flags);
    }
    QG_LAUNCH_CHECK("qg_mask_tile_ranges");
    return QG_OK;
}
