// Tile binning by (tile, depth) keys with a device LSD radix sort.
//
// The blend of Eq. 2 visits, per pixel, the Gaussians in depth order; tiling restricts each pixel to the
// Gaussians whose tile rectangle covers its tile.  The order wanted is that of the 64-bit key
// (global tile << 32 | depth bits), ties by Gaussian index.  An LSD radix sort on that key first sorts
// by the 32 depth bits, then by the tile bits.  All pairs of one (view, Gaussian) share the depth
// digits, so the depth passes are run once per (view, Gaussian) before pairs are emitted (4 passes
// over V*n items instead of 4 passes over P pairs), and only the tile bits are sorted over the pairs
// (2 passes for up to 65,536 tiles).  Both sorts use the same stable 8-bit-digit pass:
//   histogram per block -> exclusive scan of the digit-major histogram -> stable scatter, where the
//   rank of an item inside its block is found with wave64 ballot matching on the digit bits and
//   per-wave digit counters in LDS.
#include <algorithm>

#include "qg_internal.h"

namespace qg {

qg_status bin_launch_checks();

namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// Lanes of this wave holding the same digit (among active, valid lanes).
__device__ __forceinline__ uint64_t match8(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

// Item r of lane l in wave w of block b sits at b*TILE + w*(IPT*64) + r*64 + l (wave-contiguous,
// so within a wave the rounds are in element order and waves are in element order).
template <int IPT>
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* __restrict__ keys, const uint32_t* count_ptr,
                                                        uint32_t count_fixed, int shift, uint32_t* __restrict__ hist,
                                                        int nblocks) {
    __shared__ uint32_t s_hist[kRadix];
    const uint32_t count = count_ptr ? *count_ptr : count_fixed;
    const int tid = threadIdx.x, w = tid / kWave, lane = __lane_id();
    s_hist[tid] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * (IPT * kBlock) + (uint64_t)w * (IPT * kWave);
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t idx = base + (uint64_t)r * kWave + lane;
        const bool valid = idx < count;
        const uint32_t d = valid ? (keys[idx] >> shift) & (kRadix - 1) : 0u;
        const uint64_t m = match8(d, valid);
        if (valid && (m & lanemask_lt()) == 0) atomicAdd(&s_hist[d], (uint32_t)__popcll(m));
    }
    __syncthreads();
    hist[(size_t)tid * nblocks + blockIdx.x] = s_hist[tid];
}

template <int IPT>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                           const uint32_t* count_ptr, uint32_t count_fixed, int shift,
                                                           const uint32_t* __restrict__ offsets, int nblocks) {
    __shared__ uint32_t s_cnt[kWaves][kRadix];
    const uint32_t count = count_ptr ? *count_ptr : count_fixed;
    const uint64_t blk0 = (uint64_t)blockIdx.x * (IPT * kBlock);
    if (blk0 >= count) return;  // whole block empty (uniform)
    const int tid = threadIdx.x, w = tid / kWave, lane = __lane_id();
#pragma unroll
    for (int k = 0; k < kWaves; ++k) s_cnt[k][tid] = 0;
    __syncthreads();
    const uint64_t base = blk0 + (uint64_t)w * (IPT * kWave);
    uint32_t key[IPT], val[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t idx = base + (uint64_t)r * kWave + lane;
        const bool valid = idx < count;
        key[r] = valid ? kin[idx] : 0u;
        val[r] = valid ? vin[idx] : 0u;
    }
    // phase 1: per-wave digit counts
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t idx = base + (uint64_t)r * kWave + lane;
        const bool valid = idx < count;
        const uint32_t d = (key[r] >> shift) & (kRadix - 1);
        const uint64_t m = match8(d, valid);
        if (valid && (m & lanemask_lt()) == 0) atomicAdd(&s_cnt[w][d], (uint32_t)__popcll(m));
    }
    __syncthreads();
    // per-wave starting positions: global digit offset of this block + earlier waves
    {
        uint32_t run = offsets[(size_t)tid * nblocks + blockIdx.x];
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            const uint32_t c = s_cnt[k][tid];
            s_cnt[k][tid] = run;
            run += c;
        }
    }
    __syncthreads();
    // phase 2: stable ranks and scatter
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t idx = base + (uint64_t)r * kWave + lane;
        const bool valid = idx < count;
        const uint32_t d = (key[r] >> shift) & (kRadix - 1);
        const uint64_t m = match8(d, valid);
        const uint32_t rank = (uint32_t)__popcll(m & lanemask_lt());
        const int leader = __ffsll((unsigned long long)m) - 1;
        uint32_t start = 0;
        if (valid && rank == 0) start = atomicAdd(&s_cnt[w][d], (uint32_t)__popcll(m));
        start = __shfl(start, leader < 0 ? 0 : leader);
        if (valid) {
            const uint32_t pos = start + rank;
            kout[pos] = key[r];
            vout[pos] = val[r];
        }
    }
}

// ------------------------------------------------------------------------------------------------
// Exclusive scan (three kernels: block sums, scan of block sums, block-local scan + carry).
// ------------------------------------------------------------------------------------------------
constexpr int kScanIPT = 16;
constexpr int kScanTile = kBlock * kScanIPT;

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive prefix, *total = block sum.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T* s_w, T* total) {
    const int tid = threadIdx.x, w = tid / kWave, lane = __lane_id();
    T inc = wave_incl_scan(x);
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    T wbase = 0, tot = 0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
        if (k < w) wbase += s_w[k];
        tot += s_w[k];
    }
    __syncthreads();
    *total = tot;
    return wbase + inc - x;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const TI* __restrict__ in, int64_t n, TO* __restrict__ part) {
    __shared__ TO s_w[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    TO acc = 0;
    for (int r = 0; r < kScanIPT; ++r) {
        const int64_t idx = base + (int64_t)r * kBlock + threadIdx.x;
        if (idx < n) acc += (TO)in[idx];
    }
    TO tot;
    block_excl_scan<TO>(acc, s_w, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: in-place exclusive scan of part[0..nb); writes the grand total.
template <typename TO>
__global__ __launch_bounds__(1024) void k_scan_partials(TO* __restrict__ part, int64_t nb, TO* __restrict__ total_out) {
    __shared__ TO s_w[1024 / kWave];
    TO carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += blockDim.x) {
        const int64_t idx = c0 + threadIdx.x;
        TO x = idx < nb ? part[idx] : (TO)0;
        TO tot;
        TO ex = block_excl_scan<TO>(x, s_w, &tot);
        if (idx < nb) part[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_scan_down(const TI* __restrict__ in, int64_t n, const TO* __restrict__ part,
                                                      TO* __restrict__ out) {
    __shared__ TO s_w[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
    TO v[kScanIPT];
    TO acc = 0;
#pragma unroll
    for (int r = 0; r < kScanIPT; ++r) {
        const int64_t idx = base + r;
        v[r] = idx < n ? (TO)in[idx] : (TO)0;
        acc += v[r];
    }
    TO tot;
    TO run = part[blockIdx.x] + block_excl_scan<TO>(acc, s_w, &tot);
#pragma unroll
    for (int r = 0; r < kScanIPT; ++r) {
        const int64_t idx = base + r;
        if (idx < n) out[idx] = run;
        run += v[r];
    }
}

template <typename TI, typename TO>
qg_status scan_excl(const TI* in, int64_t n, TO* out, TO* part, TO* total, hipStream_t s, const char* tag = "scan") {
    QG_TIMED(tag, s);
    const int64_t nb = std::max<int64_t>(1, ceil_div(n, kScanTile));
    k_scan_reduce<TI, TO><<<(unsigned)nb, kBlock, 0, s>>>(in, n, part);
    k_scan_partials<TO><<<1, 1024, 0, s>>>(part, nb, total);
    k_scan_down<TI, TO><<<(unsigned)nb, kBlock, 0, s>>>(in, n, part, out);
    QG_LAUNCH_CHECK("scan");
    return QG_OK;
}

inline int64_t scan_parts(int64_t n) { return std::max<int64_t>(1, ceil_div(n, kScanTile)); }

// ------------------------------------------------------------------------------------------------
// Binning kernels
// ------------------------------------------------------------------------------------------------
__global__ void k_depth_keys(int64_t n, ViewTable vt, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= n * vt.V) return;
    const int v = (int)(item / n);
    const int64_t i = item - (int64_t)v * n;
    const ProjDev& p = vt.proj[v];
    const int nt = p.ntiles[i];
    keys[item] = nt > 0 ? __float_as_uint(p.depth[i]) : 0xFFFFFFFFu;
    vals[item] = (uint32_t)item;
}

__global__ void k_gather_counts(int64_t items, int64_t n, ViewTable vt, const uint32_t* __restrict__ sorted,
                                uint32_t* __restrict__ cnt) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= items) return;
    const uint32_t item = sorted[k];
    const int v = (int)(item / n);
    const int64_t i = item - (int64_t)v * n;
    cnt[k] = (uint32_t)vt.proj[v].ntiles[i];
}

// Converts the 64-bit total into the count the tile sort uses (0 on overflow) and the caller's num_pairs.
__global__ void k_finish_count(const uint64_t* __restrict__ total, int64_t capacity, uint32_t* __restrict__ sort_count,
                               int64_t* __restrict__ num_pairs) {
    const uint64_t t = *total;
    *num_pairs = (int64_t)t;
    *sort_count = t <= (uint64_t)capacity ? (uint32_t)t : 0u;
}

// Emission, one thread per output pair (load-balanced whatever the rectangle sizes): a block owns 1024
// consecutive output positions; the (view, Gaussian) items that cover them are consecutive in depth order
// (every item with a non-empty rectangle owns at least one position, empty ones were sorted last), so the
// block loads their offsets into LDS and each position finds its item by binary search there.
constexpr int kEmitPer = 1024;

__global__ __launch_bounds__(256) void k_emit(int64_t items, int64_t n, ViewTable vt,
                                              const uint32_t* __restrict__ sorted,
                                              const uint64_t* __restrict__ offs,
                                              const uint32_t* __restrict__ sort_count,
                                              uint32_t* __restrict__ tkeys, uint32_t* __restrict__ tvals) {
    __shared__ uint64_t s_off[kEmitPer];
    __shared__ int64_t s_k0;
    const uint64_t P = *sort_count;
    const uint64_t base = (uint64_t)blockIdx.x * kEmitPer;
    if (base >= P) return;
    if (threadIdx.x == 0) {
        // last k with offs[k] <= base
        int64_t lo = 0, hi = items - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (offs[mid] <= base)
                lo = mid;
            else
                hi = mid - 1;
        }
        s_k0 = lo;
    }
    __syncthreads();
    const int64_t k0 = s_k0;
    for (int t = threadIdx.x; t < kEmitPer; t += 256) {
        const int64_t k = k0 + t;
        s_off[t] = k < items ? offs[k] : ~0ull;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kEmitPer; t += 256) {
        const uint64_t p = base + t;
        if (p >= P) break;
        int lo = 0, hi = kEmitPer - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= p)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint32_t j = (uint32_t)(p - s_off[lo]);
        const uint32_t item = sorted[k0 + lo];
        const int v = (int)(item / n);
        const int64_t i = item - (int64_t)v * n;
        const int4 r = reinterpret_cast<const int4*>(vt.proj[v].rect)[i];
        const uint32_t w = (uint32_t)(r.z - r.x);
        const uint32_t ty = (uint32_t)r.y + j / w, tx = (uint32_t)r.x + j % w;
        tkeys[p] = vt.cam[v].tile_off + ty * (uint32_t)vt.cam[v].grid_w + tx;
        tvals[p] = (uint32_t)i;
    }
}

__global__ void k_ranges(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ sort_count,
                         uint32_t* __restrict__ ranges) {
    const uint32_t P = *sort_count;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint32_t t = tkeys[p];
    if (p == 0 || tkeys[p - 1] != t) ranges[2 * (size_t)t] = (uint32_t)p;
    if (p == (int64_t)P - 1 || tkeys[p + 1] != t) ranges[2 * (size_t)t + 1] = (uint32_t)p + 1;
}

__global__ void k_keys64(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ tvals,
                         const uint32_t* __restrict__ sort_count, ViewTable vt, uint64_t* __restrict__ keys) {
    const uint32_t P = *sort_count;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint32_t t = tkeys[p];
    int v = 0;
    for (int k = 1; k < vt.V; ++k)
        if (t >= vt.cam[k].tile_off) v = k;
    const uint32_t db = __float_as_uint(vt.proj[v].depth[tvals[p]]);
    keys[p] = ((uint64_t)t << 32) | db;
}

template <int IPT>
qg_status radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                     const uint32_t* count_ptr, uint32_t count_fixed, int64_t max_count, int shift, uint32_t* hist,
                     uint32_t* hist_scan, uint32_t* part, hipStream_t s, const char* const* tags) {
    const int nblocks = (int)std::max<int64_t>(1, ceil_div(max_count, IPT * kBlock));
    {
        QG_TIMED(tags[0], s);
        k_radix_hist<IPT><<<nblocks, kBlock, 0, s>>>(kin, count_ptr, count_fixed, shift, hist, nblocks);
    }
    qg_status st = scan_excl<uint32_t, uint32_t>(hist, (int64_t)kRadix * nblocks, hist_scan, part, nullptr, s, tags[1]);
    if (st != QG_OK) return st;
    {
        QG_TIMED(tags[2], s);
        k_radix_scatter<IPT><<<nblocks, kBlock, 0, s>>>(kin, vin, kout, vout, count_ptr, count_fixed, shift, hist_scan,
                                                       nblocks);
    }
    QG_LAUNCH_CHECK("radix_pass");
    return QG_OK;
}

qg_status radix_pass_any(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                         const uint32_t* count_ptr, uint32_t count_fixed, int64_t max_count, int shift,
                         uint32_t* hist, uint32_t* hist_scan, uint32_t* part, hipStream_t s, const char* const* tags) {
    if (max_count <= (1 << 22))
        return radix_pass<4>(kin, vin, kout, vout, count_ptr, count_fixed, max_count, shift, hist, hist_scan, part, s,
                             tags);
    return radix_pass<16>(kin, vin, kout, vout, count_ptr, count_fixed, max_count, shift, hist, hist_scan, part, s,
                          tags);
}

const char* const kDepthTags[3] = {"sort_depth_hist", "sort_depth_scan", "sort_depth_scatter"};
const char* const kTileTags[3] = {"sort_tile_hist", "sort_tile_scan", "sort_tile_scatter"};

int64_t radix_blocks(int64_t max_count) {
    const int ipt = max_count <= (1 << 22) ? 4 : 16;
    return std::max<int64_t>(1, ceil_div(max_count, ipt * kBlock));
}

struct BinWs {
    uint32_t *dkA, *dkB, *dvA, *dvB;  // depth sort, V*n
    uint32_t* cnt;                    // V*n
    uint64_t* offs;                   // V*n
    uint64_t* part64;                 // scan partials (64-bit)
    uint64_t* total64;
    uint32_t* sort_count;
    uint32_t *tkA, *tkB, *tvB;        // tile sort, capacity
    uint32_t *hist, *hist_scan, *part32;
    size_t bytes;
};

BinWs bin_ws_layout(char* base, int64_t n, int32_t V, int64_t capacity) {
    BinWs w{};
    size_t off = 0;
    auto take = [&](size_t b) {
        char* p = base ? base + off : nullptr;
        off += align_up(b);
        return p;
    };
    const int64_t items = n * V;
    const int64_t it1 = std::max<int64_t>(items, 1);
    const int64_t cap1 = std::max<int64_t>(capacity, 1);
    w.dkA = (uint32_t*)take(4 * it1);
    w.dkB = (uint32_t*)take(4 * it1);
    w.dvA = (uint32_t*)take(4 * it1);
    w.dvB = (uint32_t*)take(4 * it1);
    w.cnt = (uint32_t*)take(4 * it1);
    w.offs = (uint64_t*)take(8 * it1);
    w.part64 = (uint64_t*)take(8 * scan_parts(it1));
    w.total64 = (uint64_t*)take(8);
    w.sort_count = (uint32_t*)take(4);
    w.tkA = (uint32_t*)take(4 * cap1);
    w.tkB = (uint32_t*)take(4 * cap1);
    w.tvB = (uint32_t*)take(4 * cap1);
    const int64_t hb = kRadix * std::max(radix_blocks(cap1), radix_blocks(it1));
    w.hist = (uint32_t*)take(4 * hb);
    w.hist_scan = (uint32_t*)take(4 * hb);
    w.part32 = (uint32_t*)take(4 * scan_parts(hb));
    w.bytes = off;
    return w;
}

}  // namespace

}  // namespace qg

using namespace qg;

extern "C" size_t qg_bin_workspace_size(int64_t n, int32_t V, int64_t capacity, int64_t total_tiles) {
    (void)total_tiles;
    if (n < 0 || V < 1 || capacity < 0) return 0;
    return bin_ws_layout(nullptr, n, V, capacity).bytes;
}

extern "C" qg_status qg_bin(int64_t n, const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                            int64_t capacity, uint32_t* vals, uint64_t* keys, uint32_t* tile_ranges,
                            int64_t* num_pairs, void* ws, size_t ws_bytes, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && n < (1ll << 31), "n=%lld outside [0, 2^31)", (long long)n);
    QG_REQUIRE(capacity >= 0 && capacity <= 0xFFFFFFFFll, "capacity=%lld outside [0, 2^32)", (long long)capacity);
    ViewTable vt;
    if (!make_view_table(cams, proj, V, tiling, true, &vt)) return QG_ERR_ARG;
    QG_REQUIRE((int64_t)n * V < (1ll << 32), "n*V too large");
    QG_REQUIRE(tile_ranges && num_pairs, "tile_ranges and num_pairs are required");
    QG_REQUIRE(capacity == 0 || vals, "vals is NULL");
    BinWs w = bin_ws_layout((char*)ws, n, V, capacity);
    QG_REQUIRE(ws && ws_bytes >= w.bytes, "workspace too small: %zu < %zu", ws_bytes, w.bytes);
    hipStream_t s = (hipStream_t)stream;
    const int64_t items = n * V;
    const int64_t T = vt.total_tiles;
    qg_status st = qg_zero(tile_ranges, 8 * T, stream);
    if (st != QG_OK) return st;
    if (items == 0) {
        st = qg_zero(w.total64, 8, stream);
        if (st != QG_OK) return st;
        k_finish_count<<<1, 1, 0, s>>>(w.total64, capacity, w.sort_count, num_pairs);
        QG_LAUNCH_CHECK("qg_bin");
        return QG_OK;
    }
    // 1. depth keys and the 4-pass depth sort over (view, Gaussian) items
    {
        QG_TIMED("bin_depth_keys", s);
        k_depth_keys<<<(unsigned)ceil_div(items, 256), 256, 0, s>>>(n, vt, w.dkA, w.dvA);
    }
    QG_LAUNCH_CHECK("qg_bin depth keys");
    uint32_t *ka = w.dkA, *va = w.dvA, *kb = w.dkB, *vb = w.dvB;
    for (int pass = 0; pass < 4; ++pass) {
        st = radix_pass_any(ka, va, kb, vb, nullptr, (uint32_t)items, items, 8 * pass, w.hist, w.hist_scan, w.part32, s,
                            kDepthTags);
        if (st != QG_OK) return st;
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    const uint32_t* sorted_items = va;
    // 2. tile counts in depth order, scan, emission
    {
        QG_TIMED("bin_counts", s);
        k_gather_counts<<<(unsigned)ceil_div(items, 256), 256, 0, s>>>(items, n, vt, sorted_items, w.cnt);
    }
    st = scan_excl<uint32_t, uint64_t>(w.cnt, items, w.offs, w.part64, w.total64, s, "bin_count_scan");
    if (st != QG_OK) return st;
    k_finish_count<<<1, 1, 0, s>>>(w.total64, capacity, w.sort_count, num_pairs);
    QG_LAUNCH_CHECK("qg_bin count");
    if (capacity == 0) return QG_OK;
    int tbits = 1;
    while ((1ll << tbits) < T) ++tbits;
    const int tpasses = (tbits + kRadixBits - 1) / kRadixBits;
    uint32_t* vbuf0 = (tpasses % 2 == 1) ? w.tvB : vals;
    uint32_t* vbuf1 = (tpasses % 2 == 1) ? vals : w.tvB;
    {
        QG_TIMED("bin_emit", s);
        k_emit<<<(unsigned)ceil_div(capacity, kEmitPer), 256, 0, s>>>(items, n, vt, sorted_items, w.offs,
                                                                      w.sort_count, w.tkA, vbuf0);
    }
    QG_LAUNCH_CHECK("qg_bin emit");
    // 3. stable sort by tile id
    uint32_t *tk_in = w.tkA, *tk_out = w.tkB, *tv_in = vbuf0, *tv_out = vbuf1;
    for (int pass = 0; pass < tpasses; ++pass) {
        st = radix_pass_any(tk_in, tv_in, tk_out, tv_out, w.sort_count, 0u, capacity, 8 * pass, w.hist, w.hist_scan,
                            w.part32, s, kTileTags);
        if (st != QG_OK) return st;
        std::swap(tk_in, tk_out);
        std::swap(tv_in, tv_out);
    }
    // tk_in / tv_in hold the sorted pairs; tv_in == vals by construction
    // 4. tile ranges (and optional 64-bit keys)
    {
        QG_TIMED("bin_ranges", s);
        k_ranges<<<(unsigned)ceil_div(capacity, 256), 256, 0, s>>>(tk_in, w.sort_count, tile_ranges);
    }
    QG_LAUNCH_CHECK("qg_bin ranges");
    if (keys) {
        k_keys64<<<(unsigned)ceil_div(capacity, 256), 256, 0, s>>>(tk_in, tv_in, w.sort_count, vt, keys);
        QG_LAUNCH_CHECK("qg_bin keys");
    }
    return QG_OK;
}
