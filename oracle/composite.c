/*
 * CPU FP64 oracle: per-pixel front-to-back alpha compositing (Eq. 2) and its exact adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this file; only the
 * tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Plain definition, no tiles, no sort keys: for every requested pixel centre x the oracle scans
 * ALL splats, keeps those whose blend alpha
 *     a_i(x) = min(alpha_max, o_i * exp(-q_i / 2)),   q_i = A dx^2 + 2 B dx dy + C dy^2,  d = x - p'_i
 * is >= alpha_min, orders them by (depth, index), and blends front to back (Eq. 2):
 *     T = 1, C = 0;  for each kept splat: T' = T (1 - a);  stop if T' < t_min (splat not added);
 *                    C += c a T;  T = T'.
 *     output C + T bg,  T_final = T,  last = index of the last added splat.
 * (alpha_max = 0.99, alpha_min = 1/255, t_min = 1e-4 in standard mode; the "smooth" mode used for
 * finite differences sets alpha_max = +inf, alpha_min = 0, t_min = 0.)
 *
 * Adjoint (exact reverse-mode derivative of the above for fixed decisions), written from Eq. 2:
 *     dC/dc_k = a_k T_k
 *     dC/da_k = T_k c_k - R_k / (1 - a_k),   R_k = sum_{j>k} c_j a_j T_j + T_final bg
 * with T_k either stored from the forward sweep or recomputed from T_final by T_k = T_{k+1}/(1-a_k)
 * (both are offered so the two can be compared), then chained through a = o e^{-q/2} (zero where
 * the 0.99 clamp is active) and q(d, conic).
 *
 * Decision margins: for each pixel the oracle reports the smallest relative distance of any
 * alpha/transmittance decision taken on its path to its threshold (1/255 skip, 0.99 clamp,
 * termination) and, separately, the smallest relative gap between two adjacent depths on the path
 * (an order decision, which can only differ when the two sides compute depths independently).
 * Pixels with a tiny margin may legitimately decide differently in float32 and are excluded from
 * parity comparisons by the tests.  The distance of an alpha decision is reduced by an estimate of the
 * relative error of a float32 evaluation of alpha, (1/2) eps (|A| dx^2 + 2 |B dx dy| + |C| dy^2) with
 * eps = 8 * 2^-24: q is a sum whose terms can be far larger than q itself (a large splat far from the
 * pixel), and float32 resolves q only to a few units in the last place of its largest term.  The
 * distance of a termination decision is reduced by the propagated relative error of T.  For ordinary
 * splats the reduction is negligible.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double depth;
    int64_t idx;
    double alpha;   /* clamped/unclamped alpha as used */
    double gexp;    /* exp(-q/2) */
    double raw;     /* o * exp(-q/2) before the clamp */
    double err;     /* estimated relative error of a float32 evaluation of raw */
} cand_t;

#define F32_EVAL_EPS (8.0 / 16777216.0)

static int cmp_cand(const void* a, const void* b) {
    const cand_t* x = (const cand_t*)a;
    const cand_t* y = (const cand_t*)b;
    if (x->depth < y->depth) return -1;
    if (x->depth > y->depth) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

static double rel(double v, double thr) {
    double d = fabs(v - thr);
    return thr != 0.0 ? d / fabs(thr) : d;
}

int oracle_composite(int64_t n, const double* xy, const double* conic, const double* opacity,
                     const double* rgb, const double* depth, const uint8_t* valid,
                     int64_t m, const double* px, const double* py, const double* bg,
                     double alpha_min, double alpha_max, double t_min, int reverse_t,
                     const double* grad_color,
                     double* color, double* t_final, int64_t* last_id, int32_t* n_contrib,
                     double* margin, double* order_margin,
                     double* g_xy, double* g_conic, double* g_opacity, double* g_rgb,
                     int nthreads) {
    if (n < 0 || m < 0) return -1;
    int do_grad = grad_color != NULL && g_xy != NULL && g_conic != NULL && g_opacity != NULL &&
                  g_rgb != NULL;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    /* per-thread gradient accumulators (9 doubles per splat), summed at the end */
    double* acc = NULL;
    if (do_grad) {
        acc = (double*)calloc((size_t)nthreads * (size_t)(n > 0 ? n : 1) * 9, sizeof(double));
        if (!acc) return -2;
    }
    int err = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cand_t* cand = (cand_t*)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
        double* Tk = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n + 1 : 2));
        double* my = do_grad ? acc + (size_t)tid * (size_t)(n > 0 ? n : 1) * 9 : NULL;
        if (!cand || !Tk) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < m; ++p) {
            if (!cand || !Tk) continue;
            const double x = px[p], y = py[p];
            double mg = INFINITY, og = INFINITY;
            int64_t nc = 0;
            /* 1. all splats with alpha close to or above alpha_min */
            for (int64_t i = 0; i < n; ++i) {
                if (valid && !valid[i]) continue;
                const double dx = x - xy[2 * i], dy = y - xy[2 * i + 1];
                const double q = conic[3 * i] * dx * dx + 2.0 * conic[3 * i + 1] * dx * dy +
                                 conic[3 * i + 2] * dy * dy;
                const double qabs = fabs(conic[3 * i]) * dx * dx + 2.0 * fabs(conic[3 * i + 1] * dx * dy) +
                                    fabs(conic[3 * i + 2]) * dy * dy;
                const double ge = exp(-0.5 * q);
                const double raw = opacity[i] * ge;
                const double a = raw < alpha_max ? raw : alpha_max;
                /* keep near-threshold splats too so their margin is seen */
                if (a < alpha_min * (1.0 - 1e-3)) continue;
                cand[nc].depth = depth[i];
                cand[nc].idx = i;
                cand[nc].alpha = a;
                cand[nc].gexp = ge;
                cand[nc].raw = raw;
                cand[nc].err = 0.5 * F32_EVAL_EPS * qabs + F32_EVAL_EPS;
                ++nc;
            }
            qsort(cand, (size_t)nc, sizeof(cand_t), cmp_cand);
            /* 2. front-to-back blend */
            double T = 1.0, C[3] = {0.0, 0.0, 0.0};
            int64_t k = 0, nk = 0; /* nk: number of entries of cand[] that were considered */
            int64_t last = -1;
            int32_t cnt = 0;
            double prev_depth = NAN;
            double terr = 0.0; /* estimated relative error of T in float32 */
            for (k = 0; k < nc; ++k) {
                const cand_t* c = &cand[k];
                if (!isnan(prev_depth) && c->depth != 0.0)
                    og = fmin(og, fabs(c->depth - prev_depth) / fabs(c->depth));
                prev_depth = c->depth;
                if (alpha_min > 0.0) mg = fmin(mg, rel(c->raw, alpha_min) - c->err);
                if (isfinite(alpha_max)) mg = fmin(mg, rel(c->raw, alpha_max) - c->err);
                nk = k + 1;
                if (c->alpha < alpha_min) { cand[k].alpha = -1.0; continue; } /* skipped */
                const double Tn = T * (1.0 - c->alpha);
                const double tn_err = terr + c->err * c->alpha / fmax(1.0 - c->alpha, 1e-300) + F32_EVAL_EPS;
                if (t_min > 0.0) mg = fmin(mg, rel(Tn, t_min) - tn_err);
                if (Tn < t_min) { nk = k; break; }
                Tk[k] = T;
                const double* col = rgb + 3 * c->idx;
                for (int ch = 0; ch < 3; ++ch) C[ch] += col[ch] * c->alpha * T;
                T = Tn;
                terr = tn_err;
                last = c->idx;
                ++cnt;
            }
            for (int ch = 0; ch < 3; ++ch) color[3 * p + ch] = C[ch] + T * bg[ch];
            t_final[p] = T;
            last_id[p] = last;
            n_contrib[p] = cnt;
            if (margin) margin[p] = mg;
            if (order_margin) order_margin[p] = og;
            /* 3. adjoint */
            if (do_grad) {
                const double* G = grad_color + 3 * p;
                if (G[0] == 0.0 && G[1] == 0.0 && G[2] == 0.0) continue;
                double R[3] = {T * bg[0], T * bg[1], T * bg[2]}; /* suffix sum R_k */
                double Tnext = T;                                 /* T_{k+1} for reverse-T */
                for (int64_t j = nk - 1; j >= 0; --j) {
                    const cand_t* c = &cand[j];
                    if (c->alpha < 0.0) continue; /* skipped */
                    const int64_t i = c->idx;
                    const double a = c->alpha;
                    const double Tcur = reverse_t ? Tnext / (1.0 - a) : Tk[j];
                    const double* col = rgb + 3 * i;
                    double dLda = 0.0;
                    for (int ch = 0; ch < 3; ++ch) {
                        my[9 * i + 6 + ch] += G[ch] * a * Tcur; /* d rgb */
                        dLda += G[ch] * (Tcur * col[ch] - R[ch] / (1.0 - a));
                    }
                    for (int ch = 0; ch < 3; ++ch) R[ch] += col[ch] * a * Tcur;
                    Tnext = Tcur;
                    const int clamped = c->raw > alpha_max;
                    if (clamped) continue;
                    const double dx = x - xy[2 * i], dy = y - xy[2 * i + 1];
                    const double dLdq = dLda * (-0.5 * a);
                    my[9 * i + 5] += dLda * c->gexp; /* d opacity */
                    /* q = A dx^2 + 2 B dx dy + C dy^2 with d = x - p' */
                    my[9 * i + 0] += dLdq * (-(2.0 * conic[3 * i] * dx + 2.0 * conic[3 * i + 1] * dy));
                    my[9 * i + 1] += dLdq * (-(2.0 * conic[3 * i + 1] * dx + 2.0 * conic[3 * i + 2] * dy));
                    my[9 * i + 2] += dLdq * dx * dx;
                    my[9 * i + 3] += dLdq * 2.0 * dx * dy;
                    my[9 * i + 4] += dLdq * dy * dy;
                }
            }
        }
        free(cand);
        free(Tk);
    }
    if (do_grad) {
        for (int64_t i = 0; i < n; ++i) {
            double s[9] = {0};
            for (int t = 0; t < nthreads; ++t) {
                const double* a = acc + ((size_t)t * (size_t)n + (size_t)i) * 9;
                for (int k = 0; k < 9; ++k) s[k] += a[k];
            }
            g_xy[2 * i] += s[0];
            g_xy[2 * i + 1] += s[1];
            g_conic[3 * i] += s[2];
            g_conic[3 * i + 1] += s[3];
            g_conic[3 * i + 2] += s[4];
            g_opacity[i] += s[5];
            g_rgb[3 * i] += s[6];
            g_rgb[3 * i + 1] += s[7];
            g_rgb[3 * i + 2] += s[8];
        }
        free(acc);
    }
    return err;
}
