// Projection of 3D Gaussians to 2D splats (Eq. 1) with SH colour, and its adjoint.
//
// One thread per Gaussian; the thread walks all V views so the 59 attribute planes (coalesced SoA
// loads, 236 B per Gaussian) are read once per call whatever V is.  The forward writes, per view,
// a 48-byte splat record (gathered later by the blend kernels), the depth used by the sort, the
// integer tile rectangle and tile count.  The adjoint re-derives the same forward quantities and
// applies the chain rule by hand; gradients that do not depend on the view (covariance, opacity)
// are summed over views first and pushed through the quaternion/scale chain once.
#include <cmath>

#include "gauss_math.h"

namespace qg {

namespace {

__global__ __launch_bounds__(256) void k_project(int64_t n, int64_t ld, const float* __restrict__ A, int sh_deg,
                                                 ViewTable vt, float dilation, int tile_w, int tile_h) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    auto get = [&](int k) { return A[(int64_t)k * ld + i]; };
    project_gauss(i, get, sh_deg, vt, dilation, tile_w, tile_h);
}

__global__ __launch_bounds__(256) void k_project_bwd(int64_t n, int64_t ld, const float* __restrict__ A, int sh_deg,
                                                     ViewTable vt, float dilation,
                                                     const float* __restrict__ grad2d, int64_t g2d_view_stride,
                                                     float* __restrict__ G, float* __restrict__ gxy_abs,
                                                     ViewPtrs gxyv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    auto get = [&](int k) { return A[(int64_t)k * ld + i]; };
    auto put = [&](int k, float v) { G[(int64_t)k * ld + i] += v; };
    project_bwd_gauss(n, i, get, put, sh_deg, vt, dilation, grad2d, g2d_view_stride, gxy_abs, gxyv);
}

}  // namespace

qg_status project_bwd_launch(int64_t n, int64_t ld, const float* attrs, int sh_degree, const ViewTable& vt,
                             float dilation, const float* grad2d, int64_t g2d_view_stride, float* grad_attrs,
                             float* grad_xy_abs, float* const* grad_xy, hipStream_t s) {
    if (n == 0) return QG_OK;
    ViewPtrs gv = {};
    if (grad_xy)
        for (int v = 0; v < vt.V; ++v) gv.p[v] = grad_xy[v];
    {
        QG_TIMED("project_bwd", s);
        k_project_bwd<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, ld, attrs, sh_degree, vt, dilation, grad2d,
                                                                 g2d_view_stride, grad_attrs, grad_xy_abs, gv);
    }
    QG_LAUNCH_CHECK("project_bwd");
    return QG_OK;
}

}  // namespace qg

using namespace qg;

extern "C" qg_status qg_project(int64_t n, int64_t ld, const float* attrs, int32_t sh_degree, const qg_camera* cams,
                                int32_t V, qg_tiling tiling, float dilation, const qg_projected* out,
                                qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n, "n=%lld ld=%lld: need 0 <= n <= ld", (long long)n, (long long)ld);
    QG_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "sh_degree=%d outside [0, 3]", sh_degree);
    QG_REQUIRE(dilation >= 0.f && std::isfinite(dilation), "dilation must be finite and >= 0");
    QG_REQUIRE(n == 0 || attrs, "attrs is NULL");
    QG_REQUIRE(n < (1ll << 31), "n too large");
    ViewTable vt;
    if (!make_view_table(cams, out, V, tiling, true, &vt)) return QG_ERR_ARG;
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("project", s);
        k_project<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, ld, attrs, sh_degree, vt, dilation, tiling.tile_w,
                                                             tiling.tile_h);
    }
    QG_LAUNCH_CHECK("qg_project");
    return QG_OK;
}
