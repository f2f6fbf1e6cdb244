// Device math of the projection (Eq. 1) with SH colour and of its adjoint, shared by the standalone
// projection kernels and the fused decode+projection kernels.  Internal to libqg.
#pragma once

#include <cmath>

#include "qg_internal.h"

namespace qg {

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Real SH basis (l-major, m = -l..l, Condon-Shortley phase) written as polynomials of the unit
// direction, and the constants as closed forms of sqrt((2l+1)/4pi (l-m)!/(l+m)!) times the
// Legendre-derivative coefficients.
__device__ __forceinline__ void sh_consts(float* c) {
    // c0 = 1/(2 sqrt(pi)), c1 = sqrt(3/(4 pi))
    c[0] = 0.28209479177387814f;
    c[1] = 0.48860251190291992f;
    // degree 2: 1/2 sqrt(15/pi), 1/4 sqrt(5/pi), 1/4 sqrt(15/pi)
    c[2] = 1.0925484305920792f;
    c[3] = 0.31539156525252005f;
    c[4] = 0.54627421529603959f;
    // degree 3: 1/4 sqrt(35/(2pi)), 1/2 sqrt(105/pi), 1/4 sqrt(21/(2pi)), 1/4 sqrt(7/pi), 1/4 sqrt(105/pi)
    c[5] = 0.59004358992664352f;
    c[6] = 2.8906114426405538f;
    c[7] = 0.45704579946446572f;
    c[8] = 0.37317633259011546f;
    c[9] = 1.4453057213202769f;
}

// Y[k] for k < (deg+1)^2, zero above.
__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y) {
#pragma clang fp contract(off)
    float c[10];
    sh_consts(c);
#pragma unroll
    for (int k = 0; k < 16; ++k) Y[k] = 0.f;
    Y[0] = c[0];
    if (deg < 1) return;
    Y[1] = -c[1] * y;
    Y[2] = c[1] * z;
    Y[3] = -c[1] * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c[2] * x * y;
    Y[5] = -c[2] * y * z;
    Y[6] = c[3] * (3.f * zz - 1.f);
    Y[7] = -c[2] * x * z;
    Y[8] = c[4] * (xx - yy);
    if (deg < 3) return;
    Y[9] = -c[5] * y * (3.f * xx - yy);
    Y[10] = c[6] * x * y * z;
    Y[11] = -c[7] * y * (5.f * zz - 1.f);
    Y[12] = c[8] * z * (5.f * zz - 3.f);
    Y[13] = -c[7] * x * (5.f * zz - 1.f);
    Y[14] = c[9] * z * (xx - yy);
    Y[15] = -c[5] * x * (xx - 3.f * yy);
}

// g = sum_k w[k] grad Y_k (gradient in R^3 of the polynomial forms above).
__device__ __forceinline__ void sh_grad(int deg, float x, float y, float z, const float* w, float* g) {
    float c[10];
    sh_consts(c);
    g[0] = g[1] = g[2] = 0.f;
    if (deg < 1) return;
    g[1] += -c[1] * w[1];
    g[2] += c[1] * w[2];
    g[0] += -c[1] * w[3];
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    g[0] += c[2] * y * w[4];
    g[1] += c[2] * x * w[4];
    g[1] += -c[2] * z * w[5];
    g[2] += -c[2] * y * w[5];
    g[2] += 6.f * c[3] * z * w[6];
    g[0] += -c[2] * z * w[7];
    g[2] += -c[2] * x * w[7];
    g[0] += 2.f * c[4] * x * w[8];
    g[1] += -2.f * c[4] * y * w[8];
    if (deg < 3) return;
    g[0] += -c[5] * 6.f * x * y * w[9];
    g[1] += -c[5] * (3.f * xx - 3.f * yy) * w[9];
    g[0] += c[6] * y * z * w[10];
    g[1] += c[6] * x * z * w[10];
    g[2] += c[6] * x * y * w[10];
    g[1] += -c[7] * (5.f * zz - 1.f) * w[11];
    g[2] += -c[7] * 10.f * y * z * w[11];
    g[2] += c[8] * (15.f * zz - 3.f) * w[12];
    g[0] += -c[7] * (5.f * zz - 1.f) * w[13];
    g[2] += -c[7] * 10.f * x * z * w[13];
    g[0] += c[9] * 2.f * x * z * w[14];
    g[1] += -c[9] * 2.f * y * z * w[14];
    g[2] += c[9] * (xx - yy) * w[14];
    g[0] += -c[5] * (3.f * xx - 3.f * yy) * w[15];
    g[1] += c[5] * 6.f * x * y * w[15];
}

// Rotation matrix (row-major) of a unit quaternion (w, x, y, z).
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float* R) {
#pragma clang fp contract(off)
    R[0] = 1.f - 2.f * (y * y + z * z);
    R[1] = 2.f * (x * y - w * z);
    R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);
    R[4] = 1.f - 2.f * (x * x + z * z);
    R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);
    R[7] = 2.f * (y * z + w * x);
    R[8] = 1.f - 2.f * (x * x + y * y);
}

struct Gauss {
    float p[3];
    float q[4];      // normalised
    float qnorm;
    float s[3];      // exp(log-scale)
    float Sig[6];    // xx, xy, xz, yy, yz, zz
    float M[9];      // R(q) diag(s)
    float Rq[9];
    float opacity;
    bool finite;
};

template <class Get>
__device__ __forceinline__ void load_gauss(const Get& get, Gauss& g) {
#pragma clang fp contract(off)
    float raw[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) raw[k] = get(k);
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 11; ++k) fin = fin && isfinite(raw[k]);
    g.p[0] = raw[0];
    g.p[1] = raw[1];
    g.p[2] = raw[2];
    float qn = sqrtf(raw[3] * raw[3] + raw[4] * raw[4] + raw[5] * raw[5] + raw[6] * raw[6]);
    fin = fin && qn > 0.f;
    float inv = qn > 0.f ? rcp(qn) : 0.f;
    g.qnorm = qn;
    g.q[0] = raw[3] * inv;
    g.q[1] = raw[4] * inv;
    g.q[2] = raw[5] * inv;
    g.q[3] = raw[6] * inv;
    g.s[0] = expf(raw[7]);
    g.s[1] = expf(raw[8]);
    g.s[2] = expf(raw[9]);
    g.opacity = rcp(1.f + expf(-raw[10]));
    quat_rot(g.q[0], g.q[1], g.q[2], g.q[3], g.Rq);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) g.M[r * 3 + c] = g.Rq[r * 3 + c] * g.s[c];
    const float* M = g.M;
    g.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    g.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    g.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    g.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    g.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    g.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
    g.finite = fin;
}

// Per-view forward quantities.
// The 2D part of the projection -- J R_v, Sigma' = (J R_v) Sigma (J R_v)^T + h I, its inverse -- is computed
// in double precision: near the camera and far off-axis J grows large and Sigma' gets ill-conditioned
// (det(Sigma') is a small difference of two large products), which float32 resolves poorly.  On this chip
// unpacked FP64 vector arithmetic issues at the same rate as unpacked FP32.  Stored records are float32.
struct ViewProj {
    float u[3];
    double T0[3], T1[3];  // rows of J R_v
    double a, b, c, det;  // Sigma' (dilated) and its determinant
    float x, y;
    bool ok;
};

__device__ __forceinline__ void sym_mul(const float* S, const double* v, double* o) {
#pragma clang fp contract(off)
    o[0] = (double)S[0] * v[0] + (double)S[1] * v[1] + (double)S[2] * v[2];
    o[1] = (double)S[1] * v[0] + (double)S[3] * v[1] + (double)S[4] * v[2];
    o[2] = (double)S[2] * v[0] + (double)S[4] * v[1] + (double)S[5] * v[2];
}

__device__ __forceinline__ void view_project(const Gauss& g, const CamDev& cam, float dilation, ViewProj& vp) {
    // no multiply-add contraction: every kernel that inlines this must produce the same bits
#pragma clang fp contract(off)
    const float* R = cam.R;
    vp.u[0] = R[0] * g.p[0] + R[1] * g.p[1] + R[2] * g.p[2] + cam.t[0];
    vp.u[1] = R[3] * g.p[0] + R[4] * g.p[1] + R[5] * g.p[2] + cam.t[1];
    vp.u[2] = R[6] * g.p[0] + R[7] * g.p[1] + R[8] * g.p[2] + cam.t[2];
    const float uz = vp.u[2];
    vp.ok = g.finite && (uz > cam.z_near);
    const double iz = vp.ok ? 1.0 / (double)uz : 1.0;
    const double j00 = (double)cam.fx * iz, j02 = -(double)cam.fx * (double)vp.u[0] * iz * iz;
    const double j11 = (double)cam.fy * iz, j12 = -(double)cam.fy * (double)vp.u[1] * iz * iz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        vp.T0[k] = j00 * (double)R[k] + j02 * (double)R[6 + k];
        vp.T1[k] = j11 * (double)R[3 + k] + j12 * (double)R[6 + k];
    }
    double s0[3], s1[3];
    sym_mul(g.Sig, vp.T0, s0);
    sym_mul(g.Sig, vp.T1, s1);
    vp.a = vp.T0[0] * s0[0] + vp.T0[1] * s0[1] + vp.T0[2] * s0[2] + (double)dilation;
    vp.b = vp.T0[0] * s1[0] + vp.T0[1] * s1[1] + vp.T0[2] * s1[2];
    vp.c = vp.T1[0] * s1[0] + vp.T1[1] * s1[1] + vp.T1[2] * s1[2] + (double)dilation;
    vp.det = vp.a * vp.c - vp.b * vp.b;
    vp.ok = vp.ok && vp.det > 0.0 && vp.a > 0.0;
    vp.x = (float)((double)cam.fx * (double)vp.u[0] * iz + (double)cam.cx);
    vp.y = (float)((double)cam.fy * (double)vp.u[1] * iz + (double)cam.cy);
}

// Projects one Gaussian (attribute plane k read by get(k)) into every view of vt and writes its records.
template <class Get>
__device__ __forceinline__ void project_gauss(int64_t i, const Get& get, int sh_deg, const ViewTable& vt, float dilation,
                                              int tile_w, int tile_h) {
    // the forward projection rounds identically in every kernel that inlines it (no contraction)
#pragma clang fp contract(off)
    Gauss g;
    load_gauss(get, g);
    const int nb = (sh_deg + 1) * (sh_deg + 1);
    float h[48];
#pragma unroll
    for (int k = 0; k < 48; ++k) h[k] = (k < 3 * nb) ? get(11 + k) : 0.f;
    bool shfin = true;
#pragma unroll
    for (int k = 0; k < 48; ++k) shfin = shfin && isfinite(h[k]);
    g.finite = g.finite && shfin;
    const float op = g.opacity;
#pragma unroll 1
    for (int v = 0; v < vt.V; ++v) {
        const CamDev& cam = vt.cam[v];
        const ProjDev& pd = vt.proj[v];
        ViewProj vp;
        view_project(g, cam, dilation, vp);
        bool ok = vp.ok && op >= (1.f / 255.f);
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
        int4 rect = make_int4(0, 0, 0, 0);
        int nt = 0;
        uint8_t flags = 0x80;
        if (ok) {
            flags = 0;
            const double id = 1.0 / vp.det;
            r0 = make_float4(vp.x, vp.y, op, 0.f);
            r1 = make_float4((float)(vp.c * id), (float)(-vp.b * id), (float)(vp.a * id), 0.f);
            // colour
            float dx = g.p[0] - cam.cpos[0], dy = g.p[1] - cam.cpos[1], dz = g.p[2] - cam.cpos[2];
            float inv = rsq(dx * dx + dy * dy + dz * dz);
            float Y[16];
            sh_basis(sh_deg, dx * inv, dy * inv, dz * inv, Y);
            float col[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.5f;
#pragma unroll
                for (int k = 0; k < 16; ++k) acc += h[3 * k + ch] * Y[k];
                if (acc < 0.f) {
                    flags |= (uint8_t)(1u << ch);
                    acc = 0.f;
                }
                col[ch] = acc;
            }
            r2 = make_float4(col[0], col[1], col[2], 0.f);
            // support: alpha >= 1/255 <=> q <= k^2 = 2 ln(255 o); half extents k sqrt(Sigma'_xx), k sqrt(Sigma'_yy)
            const float k2 = 2.f * logf(255.f * op);
            const float rx = sqrtf(k2 * (float)vp.a), ry = sqrtf(k2 * (float)vp.c);
            float j0 = ceilf(vp.x - rx - 0.5f), j1 = floorf(vp.x + rx - 0.5f);
            float i0 = ceilf(vp.y - ry - 0.5f), i1 = floorf(vp.y + ry - 0.5f);
            j0 = fmaxf(j0, 0.f);
            i0 = fmaxf(i0, 0.f);
            j1 = fminf(j1, (float)(cam.width - 1));
            i1 = fminf(i1, (float)(cam.height - 1));
            if (j0 <= j1 && i0 <= i1) {
                const int J0 = (int)j0, J1 = (int)j1, I0 = (int)i0, I1 = (int)i1;
                rect = make_int4(J0 / tile_w, I0 / tile_h, J1 / tile_w + 1, I1 / tile_h + 1);
                nt = (rect.z - rect.x) * (rect.w - rect.y);
            }
        }
        float4* rec = reinterpret_cast<float4*>(pd.splat) + 3 * i;
        rec[0] = r0;
        rec[1] = r1;
        rec[2] = r2;
        pd.depth[i] = vp.u[2];
        reinterpret_cast<int4*>(pd.rect)[i] = rect;
        pd.ntiles[i] = nt;
        pd.flags[i] = flags;
    }
}

struct ViewPtrs {
    float* p[QG_MAX_VIEWS];
};

// One view's 2D gradient record of a Gaussian (12 floats, see project_bwd_gauss) and its projection flags.
struct GradRec {
    float4 g0, g1, g2;
    uint32_t flags;
};

__device__ __forceinline__ GradRec load_grad_rec(const ViewTable& vt, const float* __restrict__ grad2d,
                                                 int64_t g2d_view_stride, int v, int64_t i) {
    const float4* gr = reinterpret_cast<const float4*>(grad2d + (int64_t)v * g2d_view_stride) + 3 * i;
    GradRec r;
    r.g0 = gr[0];
    r.g1 = gr[1];
    r.g2 = gr[2];
    r.flags = vt.proj[v].flags[i];
    return r;
}

// What project_bwd_gauss<.., kPre> takes from its caller instead of loading it: the record of view 0 and the
// old value of gxy_abs[i].  A caller that issues these loads together with its other loads waits for HBM
// once, where the passes over the views would otherwise wait once per pass.
struct BwdPre {
    GradRec r0;
    float gabs;
};

__device__ __forceinline__ BwdPre load_bwd_pre(const ViewTable& vt, const float* __restrict__ grad2d,
                                               int64_t g2d_view_stride, const float* __restrict__ gxy_abs,
                                               int64_t i) {
    BwdPre p;
    p.r0 = load_grad_rec(vt, grad2d, g2d_view_stride, 0, i);
    p.gabs = gxy_abs ? gxy_abs[i] : 0.f;
    return p;
}

// Adjoint of project_gauss for one Gaussian.  grad2d[v] holds per Gaussian: dx, dy, dA, dB, dC, dopacity,
// dr, dg, db (stride 12).  Attribute plane k is read by get(k); the gradient of plane k is handed to
// put(k, value) exactly once for planes 0..10 and the planes 11 .. 11+3(deg+1)^2-1, after every get of
// that plane.
// kShSlots: get and put address one storage slot per plane (put overwrites what get returns).  The SH
// coefficient gradients are then summed over the views in those slots, after a first sweep over the views
// that has read the coefficients for the view-direction gradient, instead of in 48 registers; the sums are
// formed in the same order, so the results are the same.
// kPre: view 0's record and the old gxy_abs[i] come from pre (load_bwd_pre) instead of memory.
template <bool kShSlots = false, bool kPre = false, class Get, class Put>
__device__ __forceinline__ void project_bwd_gauss(int64_t n, int64_t i, const Get& get, const Put& put, int sh_deg,
                                                  const ViewTable& vt, float dilation,
                                                  const float* __restrict__ grad2d, int64_t g2d_view_stride,
                                                  float* __restrict__ gxy_abs, const ViewPtrs& gxyv,
                                                  BwdPre pre = BwdPre{}) {
    // Each pass over the views carries the next view's record: it is loaded at the top of the previous
    // iteration (before anything can skip the rest of it), so its wait overlaps that view's work.
    auto first_rec = [&]() {
        GradRec r{};
        if (kPre)
            r = pre.r0;
        else if (vt.V > 0)
            r = load_grad_rec(vt, grad2d, g2d_view_stride, 0, i);
        return r;
    };
    Gauss g;
    load_gauss(get, g);
    const int nb = (sh_deg + 1) * (sh_deg + 1);
    double dPd[3] = {0.0, 0.0, 0.0};
    double dSigd[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // symmetric gradient: xx, xy, xz, yy, yz, zz
    float dop = 0.f;
    float abs_acc = 0.f;
    bool any_col = false;
    // pass 1: geometry (position, covariance, opacity) over all views
    GradRec nxt = first_rec();
#pragma unroll 1
    for (int v = 0; v < vt.V; ++v) {
        const GradRec r = nxt;
        if (v + 1 < vt.V) nxt = load_grad_rec(vt, grad2d, g2d_view_stride, v + 1, i);
        const float4 g0 = r.g0, g1 = r.g1;
        const uint32_t flags = r.flags;
        if (flags & 0x80) continue;
        const float gx = g0.x, gy = g0.y, gA = g0.z, gB = g0.w, gC = g1.x, go = g1.y;
        any_col = true;
        const CamDev& cam = vt.cam[v];
        ViewProj vp;
        view_project(g, cam, dilation, vp);
        abs_acc += sqrtf(gx * gx + gy * gy);
        if (gxyv.p[v]) {
            gxyv.p[v][i] += gx;
            gxyv.p[v][n + i] += gy;
        }
        dop += go;
        // conic -> Sigma' (a, b, c), in double precision (see ViewProj)
        const double a = vp.a, b = vp.b, c = vp.c;
        const double id = 1.0 / vp.det, id2 = id * id;
        const double dA = gA, dB = gB, dC = gC;
        const double ga = (-c * c * dA + b * c * dB - b * b * dC) * id2;
        const double gb = (2.0 * b * c * dA - (a * c + b * b) * dB + 2.0 * a * b * dC) * id2;
        const double gc = (-b * b * dA + a * b * dB - a * a * dC) * id2;
        // Sigma' = T Sigma T^T: symmetric gradient on Sigma and gradient on T rows
        const double* T0 = vp.T0;
        const double* T1 = vp.T1;
        dSigd[0] += ga * T0[0] * T0[0] + gb * T0[0] * T1[0] + gc * T1[0] * T1[0];
        dSigd[3] += ga * T0[1] * T0[1] + gb * T0[1] * T1[1] + gc * T1[1] * T1[1];
        dSigd[5] += ga * T0[2] * T0[2] + gb * T0[2] * T1[2] + gc * T1[2] * T1[2];
        dSigd[1] += ga * T0[0] * T0[1] + 0.5 * gb * (T0[0] * T1[1] + T1[0] * T0[1]) + gc * T1[0] * T1[1];
        dSigd[2] += ga * T0[0] * T0[2] + 0.5 * gb * (T0[0] * T1[2] + T1[0] * T0[2]) + gc * T1[0] * T1[2];
        dSigd[4] += ga * T0[1] * T0[2] + 0.5 * gb * (T0[1] * T1[2] + T1[1] * T0[2]) + gc * T1[1] * T1[2];
        double s0[3], s1[3];
        sym_mul(g.Sig, T0, s0);
        sym_mul(g.Sig, T1, s1);
        double dT0[3], dT1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dT0[k] = 2.0 * ga * s0[k] + gb * s1[k];
            dT1[k] = gb * s0[k] + 2.0 * gc * s1[k];
        }
        const float* R = cam.R;
        const double dJ00 = dT0[0] * R[0] + dT0[1] * R[1] + dT0[2] * R[2];
        const double dJ02 = dT0[0] * R[6] + dT0[1] * R[7] + dT0[2] * R[8];
        const double dJ11 = dT1[0] * R[3] + dT1[1] * R[4] + dT1[2] * R[5];
        const double dJ12 = dT1[0] * R[6] + dT1[1] * R[7] + dT1[2] * R[8];
        const double ux = vp.u[0], uy = vp.u[1], uz = vp.u[2];
        const double fx = cam.fx, fy = cam.fy, gxd = gx, gyd = gy;
        const double iz = 1.0 / uz, iz2 = iz * iz, iz3 = iz2 * iz;
        double du[3];
        du[0] = -fx * iz2 * dJ02 + gxd * fx * iz;
        du[1] = -fy * iz2 * dJ12 + gyd * fy * iz;
        du[2] = -fx * iz2 * dJ00 + 2.0 * fx * ux * iz3 * dJ02 - fy * iz2 * dJ11 + 2.0 * fy * uy * iz3 * dJ12 -
                gxd * fx * ux * iz2 - gyd * fy * uy * iz2;
#pragma unroll
        for (int k = 0; k < 3; ++k) dPd[k] += R[k] * du[0] + R[3 + k] * du[1] + R[6 + k] * du[2];
    }
    float dP[3] = {(float)dPd[0], (float)dPd[1], (float)dPd[2]};
    const float dSig[6] = {(float)dSigd[0], (float)dSigd[1], (float)dSigd[2],
                           (float)dSigd[3], (float)dSigd[4], (float)dSigd[5]};
    // pass 2: SH colour -> coefficients and view direction (only if some view had a record)
    if (kShSlots && any_col) {
        // sweep 1: view-direction gradient, reading the coefficients
        nxt = first_rec();
#pragma unroll 1
        for (int v = 0; v < vt.V; ++v) {
            const GradRec r = nxt;
            if (v + 1 < vt.V) nxt = load_grad_rec(vt, grad2d, g2d_view_stride, v + 1, i);
            const float4 g1 = r.g1, g2 = r.g2;
            const uint32_t flags = r.flags;
            if (flags & 0x80) continue;
            float gcol[3] = {g1.z, g1.w, g2.x};
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                if (flags & (1u << ch)) gcol[ch] = 0.f;
            if (gcol[0] == 0.f && gcol[1] == 0.f && gcol[2] == 0.f) continue;
            const CamDev& cam = vt.cam[v];
            float vx = g.p[0] - cam.cpos[0], vy = g.p[1] - cam.cpos[1], vz = g.p[2] - cam.cpos[2];
            float inv = rsq(vx * vx + vy * vy + vz * vz);
            float d[3] = {vx * inv, vy * inv, vz * inv};
            float w[16];
#pragma unroll
            for (int k = 0; k < 16; ++k)
                w[k] = k < nb ? gcol[0] * get(11 + 3 * k) + gcol[1] * get(12 + 3 * k) + gcol[2] * get(13 + 3 * k)
                              : 0.f;
            float gd[3];
            sh_grad(sh_deg, d[0], d[1], d[2], w, gd);
            const float dotp = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
#pragma unroll
            for (int k = 0; k < 3; ++k) dP[k] += (gd[k] - d[k] * dotp) * inv;
        }
        // sweep 2: the coefficients are dead; their slots sum gcol * Y over the views
#pragma unroll
        for (int k = 0; k < 48; ++k)
            if (k < 3 * nb) put(11 + k, 0.f);
        nxt = first_rec();
#pragma unroll 1
        for (int v = 0; v < vt.V; ++v) {
            const GradRec r = nxt;
            if (v + 1 < vt.V) nxt = load_grad_rec(vt, grad2d, g2d_view_stride, v + 1, i);
            const float4 g1 = r.g1, g2 = r.g2;
            const uint32_t flags = r.flags;
            if (flags & 0x80) continue;
            float gcol[3] = {g1.z, g1.w, g2.x};
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                if (flags & (1u << ch)) gcol[ch] = 0.f;
            if (gcol[0] == 0.f && gcol[1] == 0.f && gcol[2] == 0.f) continue;
            const CamDev& cam = vt.cam[v];
            float vx = g.p[0] - cam.cpos[0], vy = g.p[1] - cam.cpos[1], vz = g.p[2] - cam.cpos[2];
            float inv = rsq(vx * vx + vy * vy + vz * vz);
            float Y[16];
            sh_basis(sh_deg, vx * inv, vy * inv, vz * inv, Y);
            // four coefficients (12 slots) at a time: all reads of a group before its writes, so the group
            // waits for storage once
#pragma unroll
            for (int k0 = 0; k0 < 16; k0 += 4) {
                if (k0 >= nb) break;
                if (k0 + 4 <= nb) {
                    float cur[12];
#pragma unroll
                    for (int j = 0; j < 12; ++j) cur[j] = get(11 + 3 * k0 + j);
#pragma unroll
                    for (int j = 0; j < 12; ++j) put(11 + 3 * k0 + j, cur[j] + gcol[j % 3] * Y[k0 + j / 3]);
                } else {
                    // a partial last group (degree 0 or 2)
#pragma unroll
                    for (int k = k0; k < k0 + 4; ++k)
                        if (k < nb) {
#pragma unroll
                            for (int ch = 0; ch < 3; ++ch)
                                put(11 + 3 * k + ch, get(11 + 3 * k + ch) + gcol[ch] * Y[k]);
                        }
                }
            }
        }
    } else if (any_col) {
        // the coefficients are read where they live (get) when needed, so only their gradients occupy registers
        float dH[48];
#pragma unroll
        for (int k = 0; k < 48; ++k) dH[k] = 0.f;
        nxt = first_rec();
#pragma unroll 1
        for (int v = 0; v < vt.V; ++v) {
            const GradRec r = nxt;
            if (v + 1 < vt.V) nxt = load_grad_rec(vt, grad2d, g2d_view_stride, v + 1, i);
            const float4 g1 = r.g1, g2 = r.g2;
            const uint32_t flags = r.flags;
            if (flags & 0x80) continue;
            float gcol[3] = {g1.z, g1.w, g2.x};
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                if (flags & (1u << ch)) gcol[ch] = 0.f;
            if (gcol[0] == 0.f && gcol[1] == 0.f && gcol[2] == 0.f) continue;
            const CamDev& cam = vt.cam[v];
            float vx = g.p[0] - cam.cpos[0], vy = g.p[1] - cam.cpos[1], vz = g.p[2] - cam.cpos[2];
            float inv = rsq(vx * vx + vy * vy + vz * vz);
            float d[3] = {vx * inv, vy * inv, vz * inv};
            float Y[16];
            sh_basis(sh_deg, d[0], d[1], d[2], Y);
            float w[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                dH[3 * k + 0] += gcol[0] * Y[k];
                dH[3 * k + 1] += gcol[1] * Y[k];
                dH[3 * k + 2] += gcol[2] * Y[k];
                w[k] = k < nb ? gcol[0] * get(11 + 3 * k) + gcol[1] * get(12 + 3 * k) + gcol[2] * get(13 + 3 * k)
                              : 0.f;
            }
            float gd[3];
            sh_grad(sh_deg, d[0], d[1], d[2], w, gd);
            const float dotp = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
#pragma unroll
            for (int k = 0; k < 3; ++k) dP[k] += (gd[k] - d[k] * dotp) * inv;
        }
#pragma unroll
        for (int k = 0; k < 48; ++k)
            if (k < 3 * nb) put(11 + k, dH[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 48; ++k)
            if (k < 3 * nb) put(11 + k, 0.f);
    }
    if (gxy_abs) gxy_abs[i] = (kPre ? pre.gabs : gxy_abs[i]) + abs_acc;
    // Sigma = M M^T -> dM = 2 dSig M (dSig symmetric)
    const float S[9] = {dSig[0], dSig[1], dSig[2], dSig[1], dSig[3], dSig[4], dSig[2], dSig[4], dSig[5]};
    float dM[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            dM[r * 3 + cc] = 2.f * (S[r * 3 + 0] * g.M[0 + cc] + S[r * 3 + 1] * g.M[3 + cc] + S[r * 3 + 2] * g.M[6 + cc]);
    // M = Rq diag(s)
    float dls[3], dR[9];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        float ds = dM[cc] * g.Rq[cc] + dM[3 + cc] * g.Rq[3 + cc] + dM[6 + cc] * g.Rq[6 + cc];
        dls[cc] = ds * g.s[cc];
#pragma unroll
        for (int r = 0; r < 3; ++r) dR[r * 3 + cc] = dM[r * 3 + cc] * g.s[cc];
    }
    const float w = g.q[0], x = g.q[1], y = g.q[2], z = g.q[3];
    float dq[4];
    dq[0] = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                   2.f * x * dR[8]);
    dq[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                   2.f * y * dR[8]);
    dq[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] +
                   x * dR[6] + y * dR[7]);
    const float qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
    const float iq = g.qnorm > 0.f ? rcp(g.qnorm) : 0.f;
    const float dlogit = dop * g.opacity * (1.f - g.opacity);
    put(0, dP[0]);
    put(1, dP[1]);
    put(2, dP[2]);
    put(3, (dq[0] - w * qd) * iq);
    put(4, (dq[1] - x * qd) * iq);
    put(5, (dq[2] - y * qd) * iq);
    put(6, (dq[3] - z * qd) * iq);
    put(7, dls[0]);
    put(8, dls[1]);
    put(9, dls[2]);
    put(10, dlogit);
}

}  // namespace qg
