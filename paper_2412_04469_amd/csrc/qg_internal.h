// Internal helpers shared by the HIP translation units of libqg (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>

#include "qg.h"

namespace qg {

// Thread-local error message behind qg_last_error().
void set_error(const char* fmt, ...);
void clear_error();

#define QG_REQUIRE(cond, ...)              \
    do {                                   \
        if (!(cond)) {                     \
            ::qg::set_error(__VA_ARGS__);  \
            return QG_ERR_ARG;             \
        }                                  \
    } while (0)

#define QG_LAUNCH_CHECK(what)                                                              \
    do {                                                                                   \
        hipError_t e_ = hipGetLastError();                                                 \
        if (e_ != hipSuccess) {                                                            \
            ::qg::set_error("%s: launch failed: %s", what, hipGetErrorString(e_));         \
            return QG_ERR_HIP;                                                             \
        }                                                                                  \
    } while (0)

constexpr int kWave = 64;

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Camera in the form the kernels use (float32, by value in kernel arguments).
struct CamDev {
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float cpos[3];  // camera centre -R^T t
    int32_t width, height;
    float z_near;
    int32_t grid_w, grid_h;  // tiles
    uint32_t tile_off;       // first global tile id of this view
};

// Projected per-view buffers in kernel-argument form.
struct ProjDev {
    float* splat;
    float* depth;
    int32_t* rect;
    int32_t* ntiles;
    uint8_t* flags;
};

struct ViewTable {
    CamDev cam[QG_MAX_VIEWS];
    ProjDev proj[QG_MAX_VIEWS];
    int32_t V;
    uint32_t total_tiles;
};

// Fill a view table from host arrays; returns false (with the error set) on a bad argument.
bool make_view_table(const qg_camera* cams, const qg_projected* proj, int32_t V, qg_tiling tiling,
                     bool need_proj, ViewTable* out);
bool tiling_ok(qg_tiling t);

// Deterministic mode of the adjoints (QG_DETERMINISTIC=1 in the environment, or qg_set_deterministic).
bool deterministic_mode();

// Per-(tile, entry) partial sums of the blend adjoint in deterministic mode: kPairPart floats per pair slot.  The
// slots of (view v, Gaussian i) are base[v * n + i] + j for the tiles j = 0 .. ntiles-1 of its rectangle in
// row-major order (base: exclusive scan of the tile counts, view-major), for slots below cap.
constexpr int kPairPart = 9;
struct PairPart {
    float* part;
    uint32_t cap;
    uint32_t* base;  // [n * V]
    int64_t n;
};

// Bytes of the per-chunk decoder weight-gradient rows that deterministic mode appends to the adjoint workspaces
// (ahead of the pair partials).
size_t det_weight_part_bytes(int64_t n);
// Carves the deterministic-mode buffers out of the workspace bytes past an adjoint call's own.
qg_status det_layout(char* base, size_t bytes, int64_t n, int32_t V, float** wdet, PairPart* pp);

// Event timing around launches (no-ops unless qg_timing_enable(1)).
void timing_begin(const char* name, hipStream_t s);
void timing_end(hipStream_t s);

struct TimedScope {
    hipStream_t s;
    TimedScope(const char* name, hipStream_t st) : s(st) { timing_begin(name, st); }
    ~TimedScope() { timing_end(s); }
};
#define QG_CAT2_(a, b) a##b
#define QG_CAT_(a, b) QG_CAT2_(a, b)
#define QG_TIMED(name, stream) ::qg::TimedScope QG_CAT_(qg_timed_scope_, __LINE__)(name, stream)

}  // namespace qg
