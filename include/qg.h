/*
 * qg.h -- C ABI of the MI355X (gfx950) hot path of QUEEN's per-frame residual fitting
 * (differentiable 3D Gaussian splatting with a quantised-latent residual decoder and gated
 * position residuals).  Paper: QUEEN: QUantized Efficient ENcoding of Dynamic Gaussians for
 * Streaming Free-viewpoint Videos (NeurIPS 2024, arXiv 2412.04469).
 *
 * General rules
 *   - Pointers are DEVICE pointers unless marked [host].  Every call only enqueues work on
 *     `stream` (a hipStream_t; NULL is the null stream): no host synchronisation, no device
 *     allocation, no device free.  The caller owns every buffer; the library keeps no pointer
 *     after a call returns.  Host arrays ([host]) are read during the call only.
 *   - Validation happens before anything is enqueued.  On a bad argument the call returns
 *     QG_ERR_ARG and enqueues nothing; a failed launch returns QG_ERR_HIP.  qg_last_error()
 *     returns a thread-local message for the last non-OK status.  Nothing throws across the ABI.
 *   - Gradient outputs are accumulated (+=): the caller zeroes them once per step.
 *   - Float data are IEEE float32.  Results of the forward calls are bit-reproducible run to run;
 *     backward calls accumulate with float32 atomics (run-to-run differences ~1e-6 relative) unless
 *     deterministic mode is on (qg_set_deterministic below).
 *
 * Attribute layout (the Gaussian attribute set A = {p, q, s, o, h} of Sec. 3.1): 59 float32
 * planes of length n with plane stride ld >= n ("[59][ld]"):
 *     0-2    mean x, y, z
 *     3-6    quaternion w, x, y, z (stored unnormalised; normalised before use)
 *     7-9    log-scale x, y, z (scale = exp)
 *     10     opacity logit (opacity = sigmoid)
 *     11+3k+ch  SH coefficient of real basis function k (0..15, l-major, m = -l..l, Condon-Shortley
 *               phase), colour channel ch
 */
#ifndef QG_H_
#define QG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qg_status;
#define QG_OK 0
#define QG_ERR_ARG (-1)
#define QG_ERR_HIP (-2)
#define QG_ERR_UNSUPPORTED (-3)

#define QG_N_PLANES 59
#define QG_MAX_VIEWS 16
#define QG_SPLAT_STRIDE 12 /* floats per projected splat record */
#define QG_GRAD2D_STRIDE 12 /* floats per 2D gradient record */

typedef void* qg_stream; /* hipStream_t */

/* Thread-local message describing the last non-OK status of this thread ("" if none). */
const char* qg_last_error(void);
/* ABI version (incremented on incompatible change). */
int32_t qg_version(void);

/*
 * Deterministic mode of the adjoints (qg_render_bwd, qg_render_decode_bwd).  Off by default; QG_DETERMINISTIC=1 in
 * the environment turns it on when the library first reads the setting, and qg_set_deterministic(on) overrides
 * that.  In this mode the blend adjoint writes the wave-reduced partial derivatives of each (tile, entry) pair to
 * its own slot (slots of a (view, Gaussian) are consecutive, one per tile of its rectangle in row-major order)
 * instead of adding them into the Gaussian's record with float atomics; a second kernel then adds each
 * (view, Gaussian)'s slots in order, and the fused adjoint keeps one decoder weight-gradient row per 64
 * Gaussians, summed in a fixed order.  Gradients are then the same bits on every run (and differ from the
 * default mode only in rounding order).
 * Workspace: while the mode is on, both adjoint calls need qg_deterministic_workspace_size(n, V, capacity) bytes
 * appended to their usual workspace, where capacity is the one passed to the qg_bin call whose tile lists are
 * differentiated (one slot per pair).  The calls return QG_ERR_ARG if the workspace has no room for them;
 * slots beyond the room they find are dropped, so size it with the bin capacity.
 * The setting is process-wide; change it only while no adjoint call is being enqueued.
 */
qg_status qg_set_deterministic(int32_t on);
int32_t qg_get_deterministic(void);
size_t qg_deterministic_workspace_size(int64_t n, int32_t V, int64_t capacity);

/*
 * Pinhole camera (Sec. 3.1: intrinsics K and viewing transform W), OpenCV axes (x right, y down,
 * z forward), world->camera u = R p + t with R row-major.  p' = (fx ux/uz + cx, fy uy/uz + cy);
 * pixel (row i, column j) has its centre at (j + 0.5, i + 0.5).  Gaussians with uz <= z_near are culled.
 */
typedef struct {
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    int32_t width, height;
    float z_near;
} qg_camera;

/*
 * How the image plane is cut into tiles and how the blend kernels walk them.
 *   tile_w x tile_h  one of 8x8, 16x16, 32x8.
 *   batch            tile-list entries staged per LDS batch in the blend kernels: 32, 64, 128 or 256 (0 = 64).
 *                    Results do not depend on it.
 *   reserved         must be 0.
 *   schedule         optional device buffer written by qg_schedule_tiles for the current binning.  NULL =
 *                    tiles in groups of 4x4 dealt round-robin to the 8 XCDs; with a schedule each XCD keeps
 *                    the same tiles and takes them heaviest first.  One workgroup per tile either way; results
 *                    do not depend on it, except for the order of the float atomics of the blend adjoint.  The
 *                    blend calls only read the buffer.
 * qg_project and qg_bin read only the tile shape.
 */
typedef struct {
    int32_t tile_w, tile_h;
    int32_t batch;
    int32_t reserved;
    uint32_t* schedule;
} qg_tiling;

/*
 * Per-view output of qg_project / input of the later calls (all device, length n):
 *   splat     [n][12] float: x, y, opacity, 0 | A, B, C, 0 | r, g, b, 0
 *             where (x, y) = p' (Eq. 1), (A, B, C) = Sigma'^{-1} in q = A dx^2 + 2B dx dy + C dy^2,
 *             opacity = sigmoid(logit), (r, g, b) = max(0, SH colour + 0.5).
 *   depth     [n] float camera-space z (the order of Eq. 2's depth sort).
 *   rect      [n][4] int32 half-open tile rectangle tx0, ty0, tx1, ty1 of the tiles that hold a
 *             pixel centre with alpha >= 1/255 (axis-aligned bound of that ellipse, clipped to the
 *             image); all zero if none.
 *   ntiles    [n] int32 number of tiles in rect (0 for culled Gaussians).
 *   flags     [n] uint8: bit ch (0..2) = colour channel ch clamped at 0; bit 7 = culled.
 */
typedef struct {
    float* splat;
    float* depth;
    int32_t* rect;
    int32_t* ntiles;
    uint8_t* flags;
} qg_projected;

/* ---------------------------------------------------------------------------------------------- */
/* Decode and gate (Eq. 4-8).                                                                      */
/* ---------------------------------------------------------------------------------------------- */
/*
 * attrs_out = prev_attrs + [g * l_p ; W2 SiLU(W1 rint(latents))]          (Eq. 4, 5, Sec. 3.2.2)
 *   latent rounding is round-half-to-even, used straight-through in the backward (Eq. 5);
 *   the decoder is a shared bias-free MLP (L -> Hd -> M) with SiLU; M = 56 maps onto planes 3..58
 *   (rotation 4, log-scale 3, opacity logit 1, SH 48).  Built shape: L = 8, Hd = 32, M = 56; other
 *   shapes return QG_ERR_UNSUPPORTED.
 *   g = min(1, max(0, sigmoid((a + e) / tau) (gamma1 - gamma0) + gamma0))      (Eq. 6-7)
 *   with e = gate_noise[i] if gate_noise is given (the stochastic hard concrete gate Eq. 6 cites: e is a
 *   logistic sample log u - log(1 - u), e.g. from qg_gate_noise), else e = 0 (the gate as Eq. 6 is written).
 *   The backward and the fused calls take the same gate_noise; Eq. 8's regulariser does not depend on it.
 *   lreg_partial receives one float per 256-Gaussian block: the block's sum of
 *   sigmoid(a - tau ln(-gamma0/gamma1)) (Eq. 8); the caller reduces (qg_decode_lreg_blocks()).
 * Sizes: n >= 0, ld >= n; latents [L][ld]; W1 [Hd][L], W2 [M][Hd]; pos_pre (l_p) [3][ld]; gate_logit (a) [n];
 *   attrs_out [59][ld] (may not alias prev_attrs); gate_out [n] (may be NULL); lreg_partial
 *   [qg_decode_lreg_blocks(n)] (may be NULL).  gamma0 < 0 < 1 < gamma1, tau > 0.
 */
qg_status qg_decode_residuals(int64_t n, int64_t ld, const float* prev_attrs, const float* latents, int32_t L,
                              const float* W1, const float* W2, int32_t Hd, int32_t M, const float* pos_pre,
                              const float* gate_logit, const float* gate_noise, float gamma0, float gamma1,
                              float tau, float* attrs_out,
                              float* gate_out, float* lreg_partial, qg_stream stream);

int64_t qg_decode_lreg_blocks(int64_t n);

/*
 * Eq. 8's regulariser as the mean over the n Gaussians (the reading under which lambda_reg = 0.01 is comparable
 * with an image loss): out[0] = (sum of the nblocks block sums lreg_partial) / n, summed in a fixed order on the
 * device (0 for n = 0).  nblocks = qg_decode_lreg_blocks(n) after qg_decode_residuals, or
 * qg_decode_project_lreg_blocks(n) after qg_decode_project.  out: device float [1].
 */
qg_status qg_decode_lreg_mean(int64_t n, const float* lreg_partial, int64_t nblocks, float* out, qg_stream stream);

/*
 * Adjoint of qg_decode_lreg_mean with respect to the gate logits a (Eq. 8):
 *   grad_gate_logit[i] (+=) weight[0] * s_i (1 - s_i) / n,  s_i = sigmoid(a_i - tau ln(-gamma0 / gamma1)),
 * with weight a DEVICE float [1] (dLoss/dL_reg, e.g. lambda_reg as produced by autograd), so the caller does not
 * read it back to the host.  Same gate hyper-parameter rules as qg_decode_residuals.
 */
qg_status qg_decode_lreg_bwd(int64_t n, const float* gate_logit, float gamma0, float gamma1, float tau,
                             const float* weight, float* grad_gate_logit, qg_stream stream);

/*
 * Backward of qg_decode_residuals for loss = f(attrs_out) + lambda_reg * mean_i sigmoid(a_i - tau ln(-g0/g1)):
 *   grad_latents (+=) [L][ld]: straight-through: d/d latents = d/d rint(latents)
 *   grad_W1 (+=) [Hd][L], grad_W2 (+=) [M][Hd]: summed over Gaussians (block partials in `ws`,
 *     then a deterministic fixed-order sum)
 *   grad_pos_pre (+=) [3][ld] = g * dL/d(mean residual)
 *   grad_gate_logit (+=) [n] = (dL/d dp . l_p) (gamma1-gamma0) ghat (1-ghat)/tau [0 < g~ < 1]
 *                              + lambda_reg sigmoid'(a - tau ln(-g0/g1)) / n
 * grad_attrs [59][ld] is dL/d attrs_out.  ws must hold qg_decode_bwd_workspace_size(n, L, Hd, M) bytes.
 */
size_t qg_decode_bwd_workspace_size(int64_t n, int32_t L, int32_t Hd, int32_t M);
qg_status qg_decode_residuals_bwd(int64_t n, int64_t ld, const float* latents, int32_t L, const float* W1,
                                  const float* W2, int32_t Hd, int32_t M, const float* pos_pre,
                                  const float* gate_logit, const float* gate_noise, float gamma0, float gamma1,
                                  float tau,
                                  const float* grad_attrs, float lambda_reg, float* grad_latents, float* grad_W1,
                                  float* grad_W2, float* grad_pos_pre, float* grad_gate_logit, void* ws,
                                  size_t ws_bytes, qg_stream stream);

/*
 * Paper-mode decode (Eq. 5 as written, Sec. 3.2.1): one shared linear decoder per attribute category,
 * r_c = D_c rint(l_c), for the categories rotation (4 planes from plane 3), scaling (3 from 7), opacity (1 from
 * 10), colour base (SH degree 0, 3 from 11) and colour frequencies (higher SH, 45 from 14), with latent dimensions
 * dims[0..4] ([host]; each in [1, 16]; the paper's quantisation table gives 6, 8, 3, 8, 4 on N3DV and 6, 8, 3, 8,
 * 12 on Immersive).  latents [sum(dims)][ld] (category by category); D packed category by category, each D_c
 * row-major [M_c][L_c] (qg_linear_decoder_params(dims) floats).  Everything else (gate, positions, Eq. 8
 * partials in qg_decode_linear_blocks(n) blocks, gate_noise) as in qg_decode_residuals.
 */
int64_t qg_linear_decoder_params(const int32_t* dims);
int64_t qg_decode_linear_blocks(int64_t n);
qg_status qg_decode_linear(int64_t n, int64_t ld, const float* prev_attrs, const float* latents, const int32_t* dims,
                           const float* D, const float* pos_pre, const float* gate_logit, const float* gate_noise,
                           float gamma0, float gamma1, float tau, float* attrs_out, float* gate_out,
                           float* lreg_partial, qg_stream stream);

/*
 * Backward of qg_decode_linear (as qg_decode_residuals_bwd): grad_latents (+=) = D_c^T dL/dr_c (straight-through),
 * grad_D (+=) = sum over Gaussians of dL/dr_c rint(l_c)^T (block partials in ws, then a fixed-order sum:
 * deterministic), grad_pos_pre and grad_gate_logit (+=).  ws: qg_decode_linear_bwd_workspace_size(n, dims).
 */
size_t qg_decode_linear_bwd_workspace_size(int64_t n, const int32_t* dims);
qg_status qg_decode_linear_bwd(int64_t n, int64_t ld, const float* latents, const int32_t* dims, const float* D,
                               const float* pos_pre, const float* gate_logit, const float* gate_noise, float gamma0,
                               float gamma1, float tau, const float* grad_attrs, float lambda_reg,
                               float* grad_latents, float* grad_D, float* grad_pos_pre, float* grad_gate_logit,
                               void* ws, size_t ws_bytes, qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* Projection (Eq. 1) with SH colour.                                                              */
/* ---------------------------------------------------------------------------------------------- */
/*
 * For every Gaussian and each of the V cameras (attributes read once for all views):
 *   Sigma = R(q) diag(exp(2 s)) R(q)^T; u = R_v p + t_v; cull if uz <= z_near, non-finite input,
 *   non-positive-definite Sigma' or opacity < 1/255;
 *   Sigma' = J R_v Sigma R_v^T J^T + dilation I, J = [[fx/uz, 0, -fx ux/uz^2], [0, fy/uz, -fy uy/uz^2]];
 *   conic = Sigma'^{-1}; opacity = sigmoid(logit); colour from degree-`sh_degree` SH at the direction
 *   from the camera centre to the mean; tile rectangle from k^2 = 2 ln(255 opacity).
 * 1 <= V <= QG_MAX_VIEWS; 0 <= sh_degree <= 3; dilation >= 0; cams [host] V; out [host] V.
 */
qg_status qg_project(int64_t n, int64_t ld, const float* attrs, int32_t sh_degree, const qg_camera* cams, int32_t V,
                     qg_tiling tiling, float dilation, const qg_projected* out, qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* Tile binning: (tile, depth) keys and a device radix sort.                                       */
/* ---------------------------------------------------------------------------------------------- */
/*
 * Every (view, Gaussian) pair whose rectangle covers a tile yields one entry.  Entries are ordered by
 * the 64-bit key (global tile id << 32) | float32 bits of depth, ties by Gaussian index -- the
 * per-tile depth order of Eq. 2.  Global tile id of view v = sum of the earlier views' tile counts +
 * ty * grid_w(v) + tx.  The per-(view, Gaussian) tile counts are scanned by a reduce and an apply kernel, the
 * pairs are emitted, and they are sorted by their tile bits with stable 8-bit LSD radix passes (count, scan
 * and scatter kernels).  The depth order comes from one of two routes with the same result: when capacity
 * <= 512 * total_tiles (short tile lists) the pairs are emitted in (view, Gaussian) order and each tile's list
 * is then sorted by (depth bits, Gaussian index): one wavefront per tile for lists of up to 1024 entries, a
 * 512-thread workgroup per longer list (merge sort in LDS); otherwise the 32 depth bits are sorted
 * once per (view, Gaussian) by four radix passes before the pairs are emitted in that order.  No workgroup
 * ever waits for another.
 *   vals        [capacity] uint32 sorted Gaussian indices (within their view).
 *   keys        [capacity] uint64 sorted keys (optional, NULL to skip).
 *   tile_ranges [total_tiles][2] uint32 half-open spans into vals ([0,0) for an empty tile).
 *   num_pairs   [1] int64: the pair count P.  If P > capacity nothing is emitted, tile_ranges are all
 *               empty, and the caller must not render this step; re-run with capacity >= P.  Never
 *               negative (a reader may treat a negative value as a corrupt count).
 *   ws          qg_bin_workspace_size(n, V, capacity, total_tiles) bytes.
 * capacity <= 2^32 - 1.  total_tiles = sum over views of ceil(W/tile_w) * ceil(H/tile_h).
 */
size_t qg_bin_workspace_size(int64_t n, int32_t V, int64_t capacity, int64_t total_tiles);
int64_t qg_total_tiles(const qg_camera* cams, int32_t V, qg_tiling tiling);
qg_status qg_bin(int64_t n, const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                 int64_t capacity, uint32_t* vals, uint64_t* keys, uint32_t* tile_ranges, int64_t* num_pairs,
                 void* ws, size_t ws_bytes, qg_stream stream);

/*
 * qg_bin without a workspace argument, for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation).  Arguments, results and errors are those
 * of qg_bin; the caller still passes and owns vals, keys, tile_ranges and num_pairs.  The workspace is a
 * device array of QG_BIN_NOALLOC_SCRATCH_BYTES bytes held by the library: one copy per device, kept until the
 * process ends, its address looked up on the first call on each device (make that first call outside stream
 * capture).  The call allocates and frees nothing.
 *   Limit: a call whose qg_bin_workspace_size(n, V, capacity, .) exceeds QG_BIN_NOALLOC_SCRATCH_BYTES returns
 *   QG_ERR_ARG with nothing enqueued (64 MiB holds e.g. 300k Gaussians, one view, capacity 3.5M pairs).
 *   Sharing: every call on a device uses that device's one array, which keeps the last call's contents (each
 *   call clears what it needs zeroed itself).  Calls that overlap in time on one device -- on different
 *   streams or from different host threads -- race on it and give wrong results: serialise them.
 */
#define QG_BIN_NOALLOC_SCRATCH_BYTES (64u << 20)
size_t qg_bin_noalloc_max_bytes(void);
qg_status qg_bin_noalloc(int64_t n, const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                         int64_t capacity, uint32_t* vals, uint64_t* keys, uint32_t* tile_ranges,
                         int64_t* num_pairs, qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* Front-to-back alpha compositing (Eq. 2).                                                        */
/* ---------------------------------------------------------------------------------------------- */
/*
 * Per pixel centre x, over its tile's depth-ordered entries:
 *   alpha = min(0.99, o exp(-q/2)); skip if alpha < 1/255; T' = T (1 - alpha); stop before an entry
 *   with T' < 1e-4 (that entry is not added); C += c alpha T; T = T'.   Output C + T bg.
 * image [V] -> [3][H][W] float (planar), T_final [V] -> [H][W] float, last [V] -> [H][W] uint32: the
 * exclusive end position (in vals) of the pixel's contributors (= its tile start if none).
 * bg [host] 3 floats.  image, T_final, last are [host] arrays of V device pointers.  If qg_bin reported
 * num_pairs > capacity, every tile range is empty and the image is the background: do not use it.
 */
qg_status qg_render_fwd(const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                        const uint32_t* vals, const uint32_t* tile_ranges, const float* bg, float* const* image,
                        float* const* T_final, uint32_t* const* last, qg_stream stream);

/*
 * qg_render_fwd followed, in the same kernel, by the L1 term of Eq. 3 against gt: for each view v, as
 * qg_l1_loss(3 W_v H_v, image[v], gt[v], scale[v], grad_image[v], ...) would write it, grad_image[v] =
 * scale[v] * sign(image - gt) / (3 W_v H_v) (bit-identical values).  partials [2 * total_tiles] doubles: per
 * tile, sum |image - gt| and sum (clamp(image, 0, 1) - gt)^2 over its pixels' three channels (the sums of
 * qg_l1_loss, grouped by tile, so their rounding differs in the last bits); a view's tiles are the consecutive
 * global tile ids of that view, and qg_loss_reduce_parts(view tiles, 3 W_v H_v, partials + 2 * first tile,
 * out) gives that view's L1 and MSE.  gt, grad_image: [host] arrays of V device pointers, planar [3][H][W]
 * float; scale: [host] V floats.  Errors: QG_ERR_ARG for a NULL pointer or a non-finite scale.
 */
qg_status qg_render_fwd_l1(const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                           const uint32_t* vals, const uint32_t* tile_ranges, const float* bg, float* const* image,
                           float* const* T_final, uint32_t* const* last, const float* const* gt,
                           const float* scale, float* const* grad_image, double* partials, qg_stream stream);

/*
 * Heaviest-first tile order for the blend kernels (a scheduling aid; no arithmetic of the method).  Each tile
 * keeps the XCD that the 4x4 super-tile order gives it (neighbouring tiles share an L2); within each XCD the
 * tiles are ordered by decreasing entry count (on a log scale, 8 steps per octave; order within a step is
 * arbitrary), so that on every XCD the longest tile lists start first.
 * cams [host] V, tiling: the cameras and tiling of the binning (tile shape only is read).
 * schedule [device] qg_schedule_words(total_tiles) words: the 8 XCD segments' starts and lengths, 8 * 512
 * working words, then the order.  Build it after each qg_bin and pass it as qg_tiling.schedule to
 * qg_render_fwd / qg_render_bwd / qg_render_decode_bwd.  Up to 2^18 tiles one workgroup builds it in LDS.
 * Stream-ordered, no allocation, safe under graph capture.  QG_ERR_ARG for bad cameras, NULL pointers or a
 * short buffer.
 */
#define QG_SCHEDULE_HEADER_WORDS (16 + 8 * 512)
int64_t qg_schedule_words(int64_t total_tiles);
qg_status qg_schedule_tiles(const qg_camera* cams, int32_t V, qg_tiling tiling, const uint32_t* tile_ranges,
                            uint32_t* schedule, int64_t schedule_words, qg_stream stream);

/*
 * Adjoint of qg_render_fwd followed by the adjoint of qg_project (Eq. 1-2), for the loss gradient
 * grad_image [V] -> [3][H][W].  The blend adjoint walks each pixel's entries in reverse from `last`,
 * recomputing T_i = T_{i+1} / (1 - alpha_i) from T_final (no per-pixel lists are stored).
 *   grad_attrs   (+=) [59][ld] gradient with respect to the attribute planes, summed over views.
 *   grad_xy_abs  (+=) [n] sum over views of |dL/dp'| (optional, NULL to skip).
 *   grad_xy      [host] V pointers (optional, NULL to skip; entries may be NULL) -> (+=) [2][n] dL/dp'
 *                per view (the viewspace gradient of Eq. 9).
 *   ws           qg_render_bwd_workspace_size(n, V) bytes (per-view 2D gradient records).
 * The other arguments must be those of the qg_project / qg_bin / qg_render_fwd calls of this step.
 */
size_t qg_render_bwd_workspace_size(int64_t n, int32_t V);
qg_status qg_render_bwd(int64_t n, int64_t ld, const float* attrs, int32_t sh_degree, const qg_camera* cams,
                        int32_t V, qg_tiling tiling, float dilation, const qg_projected* proj, const uint32_t* vals,
                        const uint32_t* tile_ranges, const float* bg, const float* const* T_final, const uint32_t* const* last, const float* const* grad_image,
                        float* grad_attrs, float* grad_xy_abs, float* const* grad_xy, void* ws, size_t ws_bytes,
                        qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* Fused per-Gaussian passes.                                                                      */
/* ---------------------------------------------------------------------------------------------- */
/*
 * qg_decode_project: qg_decode_residuals followed by qg_project in one pass (Eq. 4-8 then Eq. 1).  The
 * decoded attributes stay on chip unless attrs_out ([59][ld], may be NULL) is given.  Arguments as in
 * those two calls; lreg_partial has qg_decode_project_lreg_blocks(n) entries (block sums of Eq. 8's
 * probabilities).  The projected records are bit-identical to the two-call path.
 */
int64_t qg_decode_project_lreg_blocks(int64_t n);
qg_status qg_decode_project(int64_t n, int64_t ld, const float* prev_attrs, const float* latents, int32_t L,
                            const float* W1, const float* W2, int32_t Hd, int32_t M, const float* pos_pre,
                            const float* gate_logit, const float* gate_noise, float gamma0, float gamma1, float tau,
                            int32_t sh_degree,
                            const qg_camera* cams, int32_t V, qg_tiling tiling, float dilation,
                            const qg_projected* out, float* attrs_out, float* gate_out, float* lreg_partial,
                            qg_stream stream);

/*
 * qg_render_decode_bwd: qg_render_bwd followed by qg_decode_residuals_bwd without materialising
 * dL/d attrs: the blend adjoint (Eq. 2), then per Gaussian the decoded attributes, the projection adjoint
 * (Eq. 1) and the decoder / gate backward (Eq. 5-8).  Gradient outputs as in qg_decode_residuals_bwd (+=),
 * plus grad_xy_abs / grad_xy as in qg_render_bwd.  The other arguments must be those of the
 * qg_decode_project / qg_bin / qg_render_fwd calls of this step.
 *   attrs: [59][ld] the attributes qg_decode_project wrote to attrs_out in this step (read instead of
 *          decoding the residuals again; prev_attrs may then be NULL), or NULL: the residuals are decoded
 *          again from prev_attrs on the matrix cores.  Either way the results are the same.
 * ws: qg_render_decode_bwd_workspace_size(n, V) bytes (about 48 V + 32 bytes per Gaussian).  Results equal
 * the two-call path's up to the summation order of float atomics and of the weight-gradient partials.
 */
size_t qg_render_decode_bwd_workspace_size(int64_t n, int32_t V);
qg_status qg_render_decode_bwd(int64_t n, int64_t ld, const float* prev_attrs, const float* attrs,
                               const float* latents, int32_t L, const float* W1, const float* W2, int32_t Hd,
                               int32_t M, const float* pos_pre,
                               const float* gate_logit, const float* gate_noise, float gamma0, float gamma1,
                               float tau, float lambda_reg,
                               int32_t sh_degree, const qg_camera* cams, int32_t V, qg_tiling tiling,
                               float dilation, const qg_projected* proj, const uint32_t* vals,
                               const uint32_t* tile_ranges, const float* bg, const float* const* T_final,
                               const uint32_t* const* last, const float* const* grad_image, float* grad_latents,
                               float* grad_W1, float* grad_W2, float* grad_pos_pre, float* grad_gate_logit,
                               float* grad_xy_abs, float* const* grad_xy, void* ws, size_t ws_bytes,
                               qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* Viewspace-gradient difference (Eq. 9) and gate initialisation (Eq. 10).                          */
/* ---------------------------------------------------------------------------------------------- */
/*
 * out[i] = scale * (a[i] - b[i]) for i < count.  With a = I_{t-1}, b = I_t and scale = 2 / (3 H W) this
 * is dMSE_t/dI - dMSE_{t-1}/dI at any render I, so qg_render_bwd with this image gradient and grad_xy
 * set yields one view's term of Eq. 9 (both gradients of Eq. 9 are taken at the same render, and the
 * adjoint is linear in the image gradient).
 */
qg_status qg_scaled_diff(int64_t count, const float* a, const float* b, float scale, float* out, qg_stream stream);

/*
 * Gate initialisation (Eq. 10): with |d_i| the L2 norm of d[:, i] (d is [2][n], e.g. the view sum of
 * Eq. 9's viewspace gradients; the result does not depend on its scale) and m the lower median of the
 * norms (element (n-1)/2 after sorting, found exactly by radix select), p_i = |d_i| / (|d_i| + m)
 * clamped to [1e-6, 1 - 1e-6] (0/0 gives 1e-6), and a_out[i] = logit(p_i) + tau ln(-gamma0/gamma1),
 * the gate logit whose Eq. 8 probability is p_i.  p_out [n] and median_out [1] are optional.
 * ws: qg_gate_init_workspace_size(n) bytes.
 */
size_t qg_gate_init_workspace_size(int64_t n);
qg_status qg_gate_init(int64_t n, const float* d, float gamma0, float gamma1, float tau, float* a_out, float* p_out,
                       float* median_out, void* ws, size_t ws_bytes, qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* Adaptive masked training (Sec. 3.3 "Adaptive Masked Training"; implementation details in the     */
/* appendix: t_d = 0.001, a 48 x 48 dilation, masking for a fraction of a frame's iterations).       */
/* ---------------------------------------------------------------------------------------------- */
/*
 * Static/dynamic split: dynamic[i] = 1 if sqrt((sx d[i])^2 + (sy d[n + i])^2) > t_d, evaluated in double
 * precision from the float d, else 0.  d is [2][n], e.g. the view sum of Eq. 9's viewspace gradients in
 * pixels; sx = W / (2V), sy = H / (2V) turn it into Eq. 9's mean in normalised device coordinates, the
 * units of the 3D-GS viewspace gradient the threshold t_d = 0.001 refers to.  Errors: QG_ERR_ARG for n < 0,
 * sx or sy <= 0, t_d < 0 or a NULL pointer with n > 0.
 */
qg_status qg_dynamic_flags(int64_t n, const float* d, double sx, double sy, double t_d, uint8_t* dynamic,
                           qg_stream stream);

/*
 * Image mask of each view: mask[v][y*W + x] = 1 if the render of the dynamic Gaussians alone reaches pixel
 * (x, y), i.e. some entry of the pixel's tile list (vals, tile_ranges of a qg_bin of all Gaussians) with
 * dynamic[gid] = 1 has blend alpha min(0.99, o exp(-q/2)) >= 1/255 there, evaluated exactly as in
 * qg_render_fwd (in a dynamic-only render the first such splat always contributes).  proj, cams, V,
 * tiling: as for qg_render_fwd.  mask[v]: device buffer of W_v * H_v bytes, fully written.
 */
qg_status qg_dynamic_mask(const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                          const uint32_t* vals, const uint32_t* tile_ranges, const uint8_t* dynamic,
                          uint8_t* const* mask, qg_stream stream);

/*
 * Box dilation by a k x k kernel (k = 48 in the paper): dilated[v][y*W + x] = 1 if mask[v] has a set pixel in
 * [x - k/2, x + k - 1 - k/2] x [y - k/2, y + k - 1 - k/2] (clipped to the image; integer division), else 0.
 * tmp[v] (W_v * H_v bytes, distinct from mask[v] and dilated[v]) holds the row pass.  tile_flags
 * [total tiles of the view set, global tile index as in qg_bin] = 1 if the tile contains a set dilated
 * pixel inside the image, else 0: the tiles a masked iteration renders.  Errors: QG_ERR_ARG for k outside
 * [1, 1024], a bad view set or a NULL / aliased buffer.
 */
qg_status qg_dilate_mask(const qg_camera* cams, int32_t V, qg_tiling tiling, int32_t k, const uint8_t* const* mask,
                         uint8_t* const* tmp, uint8_t* const* dilated, uint8_t* tile_flags, qg_stream stream);

/*
 * Masked iteration: every tile t with tile_flags[t] = 0 gets the empty range [start, start) in tile_ranges
 * (call after qg_bin, before the blend kernels).  qg_render_fwd then writes the background there
 * (T_final = 1) and the blend adjoint adds nothing for it, which is exact when the image gradient is zero on
 * those tiles (qg_l1_loss_masked with the dilated mask).
 */
qg_status qg_mask_tile_ranges(int64_t total_tiles, uint32_t* tile_ranges, const uint8_t* tile_flags,
                              qg_stream stream);

/*
 * qg_l1_loss restricted to the pixels set in mask [plane bytes; element i of the image, [C][plane] planar,
 * uses mask[i % plane]]: elements of unset pixels get grad_image = 0 and add nothing to the partial sums.
 * The gradient scale stays scale / count (the full image's normalisation, the masked-iteration reading), so
 * qg_loss_reduce(count, ...) gives sum over masked elements of |image - gt| / count.  count must be a
 * multiple of plane.
 */
qg_status qg_l1_loss_masked(int64_t count, int64_t plane, const float* image, const float* gt, const uint8_t* mask,
                            float scale, float* grad_image, double* partials, qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* The stochastic hard concrete gate (Eq. 6 cites it) and per-frame densification (the 3D-GS stage the */
/* paper runs at every time step: Sec. 3.4; implementation details: epochs 6 to 80%, every 2 epochs, */
/* gradient threshold 0.00125).                                                                     */
/* ---------------------------------------------------------------------------------------------- */
/*
 * Random draws come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) with key (seed low word, seed high
 * word); a uniform is u = ((w >> 9) + 1/2) / 2^23 of a 32-bit output word w, in (0, 1).
 *
 * qg_gate_noise: noise[i] = log u_i - log(1 - u_i), u_i from word 0 of Philox(counter (i, s, 0x67617465, 0)),
 * with s = step_state[0] if step_state (device int32, e.g. qg_adam_multi's step counter, so a replayed graph draws
 * afresh) is given, else s = step.  Pass the result as gate_noise to the decode calls of that step.
 */
qg_status qg_gate_noise(int64_t n, uint64_t seed, int32_t step, const int32_t* step_state, float* noise,
                        qg_stream stream);

/*
 * One iteration's densification statistic for one view: for every Gaussian with ntiles[i] > 0 (visible in the
 * view), accum[i] += |(sx grad_xy[0][i], sy grad_xy[1][i])| and count[i] += 1.  grad_xy [2][n] is dL/dp' of the
 * view in pixels (qg_render_bwd / qg_render_decode_bwd's grad_xy); sx = W/2, sy = H/2 turn it into normalised
 * device coordinates, the units of 3D-GS's gradient threshold.
 */
qg_status qg_densify_accumulate(int64_t n, const float* grad_xy, const int32_t* ntiles, float sx, float sy,
                                float* accum, float* count, qg_stream stream);

/*
 * The densification plan from the statistic and the current (decoded) attributes attrs [59][ld], decided in
 * double precision: action[i] = 3 (prune) if sigmoid(logit) < min_opacity; else, with score accum/count (0 if
 * count = 0), 0 (keep) if score < threshold, 1 (clone) if exp(max log-scale) <= max_scale, 2 (split) otherwise.
 * offsets [n + 1] (device int64): the exclusive scan of the child counts (0 prune, 1 keep, 2 clone or split),
 * offsets[n] = the new count n'.  The new set keeps each Gaussian's children in place, in parent order.
 * ws: qg_densify_plan_workspace_size(n) bytes.
 */
size_t qg_densify_plan_workspace_size(int64_t n);
qg_status qg_densify_plan(int64_t n, const float* accum, const float* count, const float* attrs, int64_t ld,
                          double threshold, double max_scale, double min_opacity, uint8_t* action, int64_t* offsets,
                          void* ws, size_t ws_bytes, qg_stream stream);

/*
 * Expands nplanes planes src [nplanes][ld_src] of n Gaussians into dst [nplanes][ld_dst] (ld_dst >= n') through the
 * plan: every child gets its parent's value (mode 0), or, for optimiser moments (mode 1), only the first child of a
 * kept or cloned Gaussian keeps it and new Gaussians start at 0.  dst may not alias src.
 */
qg_status qg_densify_expand(int64_t n, const uint8_t* action, const int64_t* offsets, int32_t nplanes,
                            const float* src, int64_t ld_src, float* dst, int64_t ld_dst, int32_t mode,
                            qg_stream stream);

/*
 * Clone and split children, after the expansion of the stored attributes into prev_out [59][ld_out], from the
 * parents' decoded attributes (decoded [59][ld]):
 *   clone: both children's opacity logit += logit(o') - logit(o), o the parent's decoded opacity and
 *          o' = 1 - sqrt(1 - o), so the two coincident copies composite like the parent where its Gaussian factor
 *          is 1 (the N-copy rule 1 - (1 - o)^(1/N) of Kheradmand et al., 3D Gaussian Splatting as Markov Chain
 *          Monte Carlo);
 *   split: child c (0, 1) gets mean += R(q) (s * z_c) and log-scale -= ln 1.6, with q, s the parent's decoded
 *          rotation (normalised) and scale and z_0, z_1 standard normal 3-vectors by Box-Muller
 *          (r = sqrt(-2 ln u_even), angle 2 pi u_odd) on the words of Philox(counter (i, round, 0x73706C74, 0))
 *          and Philox(counter (i, round, 0x73706C74, 1)).
 */
qg_status qg_densify_children(int64_t n, const uint8_t* action, const int64_t* offsets, const float* decoded,
                              int64_t ld, uint64_t seed, int32_t round, float* prev_out, int64_t ld_out,
                              qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* Storage of a frame's residuals (the compression back end after the fit): the quantised latents   */
/* (Sec. 3.2; the decoder reads rint(l_hat)) entropy coded with one model per latent dimension.     */
/* ---------------------------------------------------------------------------------------------- */
/*
 * symbols[i*L + k] = rint(latents[k*ld + i]) as int8 (device, [n*L], Gaussian-major); hist[k*256 + s + 128]
 * (device, uint32 [L][256], cleared here) counts symbol s of dimension k; *overflow (device) counts values
 * outside [-128, 127], which are stored as 0 (the caller treats a non-zero count as an error).  L <= 16.
 */
qg_status qg_latent_symbols(int64_t n, int64_t ld, const float* latents, int32_t L, int8_t* symbols, uint32_t* hist,
                            uint32_t* overflow, qg_stream stream);

/*
 * Host-side byte-wise rANS (Duda's asymmetric numeral systems, range variant; 32-bit state in [2^23, 2^31),
 * byte renormalisation) over count = n*L int8 symbols, symbol i coded with model i mod L.  Each model's
 * probabilities are its histogram row (hist, host, uint32 [L][256]) quantised to 2^16: every present symbol
 * at least 1, the rest in proportion with the remainder given to (or taken from) the most frequent symbols,
 * a deterministic function of the counts, so the decoder rebuilds it from the same histogram.  All pointers
 * are host memory.  encode: out holds at most qg_rans_bound(count) bytes; *out_bytes receives the length.
 * decode: reads exactly in_bytes and writes count symbols.  Errors: QG_ERR_ARG for bad sizes, a symbol with
 * a zero count, a short buffer, or (decode) a stream that does not end exactly.
 */
size_t qg_rans_bound(int64_t count);
qg_status qg_rans_encode(int64_t count, int32_t L, const int8_t* symbols, const uint32_t* hist, uint8_t* out,
                         size_t capacity, size_t* out_bytes);
qg_status qg_rans_decode(int64_t count, int32_t L, const uint8_t* in, size_t in_bytes, const uint32_t* hist,
                         int8_t* symbols);

/* ---------------------------------------------------------------------------------------------- */
/* Learned residual proposal (not a method of the paper: a learned replacement for zero-initialised  */
/* residual parameters of frame t, Sec. 3.2 / Eq. 5-8; its analogue in the paper is Eq. 10).         */
/* ---------------------------------------------------------------------------------------------- */
/*
 * Features [24][ld_out] of n Gaussians from the reconstructions A1 = A_{t-1}, A2 = A_{t-2}, A3 = A_{t-3}
 * ([59][ld] planes, only planes 0..9 are read: mean, quaternion, log-scale) and p [n] (the Eq. 10 gate
 * probability of frame t):  [ mean of A1 (3) | A1 - A2 on planes 0..9 (10) | A2 - A3 on planes 0..9 (10) | p ].
 */
qg_status qg_proposal_features(int64_t n, int64_t ld, const float* A1, const float* A2, const float* A3,
                               const float* p, float* out, int64_t ld_out, qg_stream stream);

/*
 * The network: y = (W3 h2 + b3) * out_std + out_mean, h2 = SiLU(W2 h1 + b2), h1 = SiLU(W1 x_s + b1),
 * x_s = (x - in_mean) * in_rstd.  Outputs (12) = [ l_p (3) | gate logit a (1) | latents l_hat (8) ].
 * Products on BF16 matrix cores with FP32 accumulation: the weights, x_s, h1, h2 (and in the backward the
 * output gradient and both dL/d pre-activation tiles) are rounded to bfloat16, round to nearest even,
 * from their float32 values; biases and pre-activations stay float32.
 * params [device] QG_PROPOSAL_PARAMS float32: W1 [64][24] | b1 [64] | W2 [64][64] | b2 [64] | W3 [12][64] | b3 [12].
 * stats  [device] 72 float32: in_mean [24] | in_rstd [24] | out_mean [12] | out_std [12].
 */
#define QG_PROPOSAL_PARAMS 6540
qg_status qg_proposal_fwd(int64_t n, int64_t ld_in, const float* features, const float* params,
                          const float* stats, float* out, int64_t ld_out, qg_stream stream);

/*
 * Gradient of the training loss L = (1/m) sum over m samples and 12 outputs of (y_s - t_s)^2, with
 * standardised outputs y_s and targets t_s = (t - out_mean) / out_std, for samples idx[0..m) (device
 * uint32 columns of features [24][ld] and targets [12][ld], or columns 0..m-1 when idx is NULL; an index
 * >= n is skipped).
 * grad (+=) [QG_PROPOSAL_PARAMS] in the params layout; loss_out [device, optional] receives L.
 * Per-wave partials are summed in a fixed order (deterministic).  ws: qg_proposal_bwd_workspace_size() bytes.
 */
size_t qg_proposal_bwd_workspace_size(void);
qg_status qg_proposal_bwd(int64_t m, const uint32_t* idx, int64_t n, int64_t ld, const float* features,
                          const float* targets, const float* params, const float* stats, float* grad,
                          float* loss_out, void* ws, size_t ws_bytes, qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* Loss (L1 term of Eq. 3), PSNR, Adam.                                                            */
/* ---------------------------------------------------------------------------------------------- */
/*
 * L1 = mean |image - gt| over count values; grad_image = scale * sign(image - gt) / count (sign(0) = 0;
 * written, not accumulated; may be NULL).  partials receives 2 doubles per block of
 * qg_loss_block_elems() values: sum |d| and sum (clamp(image,0,1) - gt)^2; qg_loss_reduce sums
 * them in a fixed order into out[0] = L1, out[1] = MSE of the clamped image (PSNR = -10 log10 MSE).
 */
int64_t qg_loss_blocks(int64_t count);

/*
 * D-SSIM term of Eq. 3 for an image [C][H][W] (planar float32) against gt: SSIM per pixel and channel under an
 * 11 x 11 Gaussian window (sigma 1.5, taps normalised to sum 1, zero padding outside the image), C1 = 0.01^2,
 * C2 = 0.03^2; D-SSIM = 1 - mean SSIM.  dssim_out (device, 1 double, may be NULL) receives D-SSIM, summed in
 * a fixed order.  grad_image (may be NULL) is incremented (+=) by weight * dD-SSIM/dimage, so an L1
 * gradient written first with scale (1 - weight) yields Eq. 3's (1 - lambda) L1 + lambda D-SSIM (the
 * paper does not give lambda; 3D-GS uses 0.2).  ws: qg_ssim_workspace_size(C, H, W) bytes.
 * Errors: QG_ERR_ARG for bad sizes (H * W must be below 2^31), NULL image/gt, both outputs NULL or a short
 * workspace.
 */
size_t qg_ssim_workspace_size(int32_t C, int32_t H, int32_t W);
qg_status qg_ssim_loss(int32_t C, int32_t H, int32_t W, const float* image, const float* gt, float weight,
                       float* grad_image, double* dssim_out, void* ws, size_t ws_bytes, qg_stream stream);
qg_status qg_l1_loss(int64_t count, const float* image, const float* gt, float scale, float* grad_image,
                     double* partials, qg_stream stream);
qg_status qg_loss_reduce(int64_t count, const double* partials, double* out, qg_stream stream);
/* As qg_loss_reduce over nparts pairs of partial sums (e.g. the per-tile partials of qg_render_fwd_l1),
 * divided by count. */
qg_status qg_loss_reduce_parts(int64_t nparts, int64_t count, const double* partials, double* out,
                               qg_stream stream);

/*
 * One bias-corrected Adam step on `count` parameters (beta = (b1, b2), eps) at 1-based step `t`:
 *   m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 */
qg_status qg_adam(int64_t count, float* param, const float* grad, float* m, float* v, float lr, float b1,
                  float b2, float eps, int32_t t, qg_stream stream);

/*
 * Several parameter groups in one launch (up to 8 segments), same update as qg_adam with a learning rate
 * per segment.  If zero_grad is non-zero each gradient is set to 0 after it is read, so the next backward
 * can accumulate (+=) into it without a separate zeroing pass.  segs [host].
 * step_state: NULL to use the host step count t (>= 1); otherwise a device buffer of 3 words {int32 step,
 * float 1 - b1^step, float 1 - b2^step}: the call increments the step on the device and uses it (t is
 * ignored), so a captured graph can replay the update.  Start it at {0, 0, 0}.
 */
typedef struct {
    float* param;
    float* grad;
    float* m;
    float* v;
    int64_t count;
    float lr;
} qg_adam_segment;
qg_status qg_adam_multi(int32_t nseg, const qg_adam_segment* segs, float b1, float b2, float eps, int32_t t,
                        int32_t* step_state, int32_t zero_grad, qg_stream stream);

/* Zero `bytes` bytes at dst with a fill kernel (no memset node, so it is safe to capture). */
qg_status qg_zero(void* dst, int64_t bytes, qg_stream stream);

/*
 * Measurement helper for the FP32 vector roofline (not part of the method): `blocks` workgroups of 256 threads,
 * each thread advancing 16 independent FP32 multiply-add chains `iters` times in registers (single FMAs, the
 * instruction the library's kernels are built with), then writing one float to out[blocks * 256] (device).
 * Work: blocks * 256 * iters * 16 * 2 flop.  QG_ERR_ARG if blocks < 1, iters < 1 or out is NULL.
 */
qg_status qg_probe_fma(int32_t blocks, int32_t iters, float* out, qg_stream stream);

/* ---------------------------------------------------------------------------------------------- */
/* Diagnostics: per-kernel timing with HIP events.                                                 */
/* ---------------------------------------------------------------------------------------------- */
/*
 * While enabled, every kernel the library launches (or, if `only` is not NULL, every kernel of that
 * name) is bracketed by two HIP events recorded on the stream it is launched on.  qg_timing_report()
 * waits for the recorded events, writes one line "name count total_ms" per kernel name into buf
 * (NUL-terminated, truncated to len bytes), clears the record and returns the number of names.
 * Off by default; not for use under stream capture.  `only` [host] is copied.
 */
qg_status qg_timing_enable(int32_t on, const char* only);
int64_t qg_timing_report(char* buf, int64_t len);

#ifdef __cplusplus
}
#endif

#endif /* QG_H_ */
