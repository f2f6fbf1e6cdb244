// Error state, argument tables and small utilities of libqg.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "qg_internal.h"

namespace qg {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// ---- event timing -------------------------------------------------------------------------------
namespace {
struct TimedLaunch {
    const char* name;
    hipEvent_t start, stop;
};
std::mutex g_tmu;
bool g_timing = false;
std::string g_only;
std::vector<TimedLaunch> g_launches;
std::vector<hipEvent_t> g_pool;
thread_local const char* t_name = nullptr;
thread_local hipEvent_t t_start = nullptr;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

void timing_begin(const char* name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing) return;
    if (!g_only.empty() && g_only != name) return;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;  // not in graphs
    t_name = name;
    t_start = get_event();
    if (t_start) hipEventRecord(t_start, s);
}

void timing_end(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing || !t_start) return;
    hipEvent_t stop = get_event();
    if (!stop) return;
    hipEventRecord(stop, s);
    g_launches.push_back({t_name, t_start, stop});
    t_start = nullptr;
}

// ---- deterministic mode ---------------------------------------------------------------------------------
namespace {
std::once_flag g_det_once;
std::atomic<int> g_det{0};
}  // namespace

bool deterministic_mode() {
    std::call_once(g_det_once, [] {
        const char* e = std::getenv("QG_DETERMINISTIC");
        if (e && std::strcmp(e, "1") == 0) g_det.store(1);
    });
    return g_det.load() != 0;
}

bool tiling_ok(qg_tiling t) {
    const bool shape = (t.tile_w == 8 && t.tile_h == 8) || (t.tile_w == 16 && t.tile_h == 16) ||
                       (t.tile_w == 32 && t.tile_h == 8);
    const bool batch = t.batch == 0 || t.batch == 32 || t.batch == 64 || t.batch == 128 || t.batch == 256;
    return shape && batch && t.reserved == 0;
}

bool make_view_table(const qg_camera* cams, const qg_projected* proj, int32_t V, qg_tiling tiling,
                     bool need_proj, ViewTable* out) {
    if (V < 1 || V > QG_MAX_VIEWS) {
        set_error("V=%d outside [1, %d]", V, QG_MAX_VIEWS);
        return false;
    }
    if (!cams) {
        set_error("cams is NULL");
        return false;
    }
    if (!tiling_ok(tiling)) {
        set_error("unsupported tiling %dx%d batch %d (8x8, 16x16, 32x8; batch 0, 32, 64, 128, 256; reserved 0)",
                  tiling.tile_w, tiling.tile_h, tiling.batch);
        return false;
    }
    if (need_proj && !proj) {
        set_error("proj is NULL");
        return false;
    }
    std::memset(out, 0, sizeof(*out));
    out->V = V;
    uint64_t off = 0;
    for (int v = 0; v < V; ++v) {
        const qg_camera& c = cams[v];
        if (c.width < 1 || c.width > 16384 || c.height < 1 || c.height > 16384) {
            set_error("view %d: size %dx%d outside [1, 16384]", v, c.width, c.height);
            return false;
        }
        if (!(c.z_near > 0.f) || !std::isfinite(c.fx) || !std::isfinite(c.fy)) {
            set_error("view %d: z_near must be > 0 and focal lengths finite", v);
            return false;
        }
        CamDev& d = out->cam[v];
        d.fx = c.fx;
        d.fy = c.fy;
        d.cx = c.cx;
        d.cy = c.cy;
        for (int k = 0; k < 9; ++k) d.R[k] = c.R[k];
        for (int k = 0; k < 3; ++k) d.t[k] = c.t[k];
        for (int k = 0; k < 3; ++k)  // centre = -R^T t, in double then rounded
            d.cpos[k] = (float)(-((double)c.R[0 + k] * c.t[0] + (double)c.R[3 + k] * c.t[1] +
                                  (double)c.R[6 + k] * c.t[2]));
        d.width = c.width;
        d.height = c.height;
        d.z_near = c.z_near;
        d.grid_w = (c.width + tiling.tile_w - 1) / tiling.tile_w;
        d.grid_h = (c.height + tiling.tile_h - 1) / tiling.tile_h;
        d.tile_off = (uint32_t)off;
        off += (uint64_t)d.grid_w * d.grid_h;
        if (need_proj) {
            const qg_projected& p = proj[v];
            if (!p.splat || !p.depth || !p.rect || !p.ntiles || !p.flags) {
                set_error("view %d: a projected buffer is NULL", v);
                return false;
            }
            out->proj[v] = ProjDev{p.splat, p.depth, p.rect, p.ntiles, p.flags};
        }
    }
    if (off >= (1ull << 31)) {
        set_error("total tile count %llu too large", (unsigned long long)off);
        return false;
    }
    out->total_tiles = (uint32_t)off;
    return true;
}

__global__ void k_zero(uint32_t* __restrict__ p, int64_t words) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) p[i] = 0u;
}

// 16-byte stores, grid-stride over a capped grid (every lane writes whole uint4s).
__global__ __launch_bounds__(256) void k_zero16(uint4* __restrict__ p, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_zero_bytes(uint8_t* __restrict__ p, int64_t bytes) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < bytes) p[i] = 0;
}

}  // namespace qg

using namespace qg;

extern "C" const char* qg_last_error(void) { return g_err; }

extern "C" int32_t qg_version(void) { return 2; }

extern "C" qg_status qg_set_deterministic(int32_t on) {
    clear_error();
    deterministic_mode();  // the environment's setting is read first, so this call overrides it
    g_det.store(on ? 1 : 0);
    return QG_OK;
}

extern "C" int32_t qg_get_deterministic(void) { return deterministic_mode() ? 1 : 0; }

extern "C" qg_status qg_timing_enable(int32_t on, const char* only) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    g_only = only ? only : "";
    return QG_OK;
}

extern "C" int64_t qg_timing_report(char* buf, int64_t len) {
    std::lock_guard<std::mutex> lk(g_tmu);
    std::map<std::string, std::pair<int64_t, double>> agg;
    for (auto& l : g_launches) {
        float ms = 0.f;
        if (hipEventSynchronize(l.stop) == hipSuccess && hipEventElapsedTime(&ms, l.start, l.stop) == hipSuccess) {
            auto& a = agg[l.name];
            a.first += 1;
            a.second += ms;
        }
        g_pool.push_back(l.start);
        g_pool.push_back(l.stop);
    }
    g_launches.clear();
    std::string out;
    for (auto& kv : agg) {
        char line[256];
        snprintf(line, sizeof(line), "%s %lld %.6f\n", kv.first.c_str(), (long long)kv.second.first, kv.second.second);
        out += line;
    }
    if (buf && len > 0) {
        const size_t n = std::min<size_t>(out.size(), (size_t)len - 1);
        std::memcpy(buf, out.data(), n);
        buf[n] = 0;
    }
    return (int64_t)agg.size();
}

extern "C" int64_t qg_total_tiles(const qg_camera* cams, int32_t V, qg_tiling tiling) {
    ViewTable t;
    if (!make_view_table(cams, nullptr, V, tiling, false, &t)) return -1;
    return t.total_tiles;
}

namespace {

// FP32 FMA issue probe: kProbeChains independent multiply-add chains per thread, held in registers, each
// advanced `iters` times; one float per thread is written so that the work is kept.
constexpr int kProbeChains = 16;

__global__ __launch_bounds__(256) void k_fma_probe(int32_t iters, float x, float y, float* __restrict__ out) {
    float a[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kProbeChains; ++k) a[k] = __builtin_fmaf(a[k], x, y);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += a[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" qg_status qg_probe_fma(int32_t blocks, int32_t iters, float* out, qg_stream stream) {
    clear_error();
    QG_REQUIRE(blocks >= 1 && iters >= 1, "blocks and iters must be >= 1");
    QG_REQUIRE(out != nullptr, "out is NULL");
    hipStream_t s = (hipStream_t)stream;
    k_fma_probe<<<(unsigned)blocks, 256, 0, s>>>(iters, 0.999f, 1e-4f, out);
    QG_LAUNCH_CHECK("qg_probe_fma");
    return QG_OK;
}

extern "C" qg_status qg_zero(void* dst, int64_t bytes, qg_stream stream) {
    clear_error();
    QG_REQUIRE(bytes >= 0, "bytes < 0");
    if (bytes == 0) return QG_OK;
    QG_REQUIRE(dst != nullptr, "dst is NULL");
    hipStream_t s = (hipStream_t)stream;
    uintptr_t a = (uintptr_t)dst;
    if (a % 16 == 0 && bytes % 16 == 0) {
        const int64_t n16 = bytes / 16;
        const int64_t blocks = std::min<int64_t>(ceil_div(n16, 256), 16384);
        {
            QG_TIMED("zero", s);
            k_zero16<<<(unsigned)blocks, 256, 0, s>>>((uint4*)dst, n16);
        }
    } else if (a % 4 == 0 && bytes % 4 == 0) {
        int64_t words = bytes / 4;
        int64_t blocks = std::min<int64_t>(ceil_div(words, 256), 65536);
        {
            QG_TIMED("zero", s);
            k_zero<<<(unsigned)blocks, 256, 0, s>>>((uint32_t*)dst, words);
        }
    } else {
        k_zero_bytes<<<(unsigned)ceil_div(bytes, 256), 256, 0, s>>>((uint8_t*)dst, bytes);
    }
    QG_LAUNCH_CHECK("qg_zero");
    return QG_OK;
}
