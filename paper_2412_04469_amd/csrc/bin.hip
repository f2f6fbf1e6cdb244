// Tile binning by (tile, depth) keys with device LSD radix sorts.
//
// The blend of Eq. 2 visits, per pixel, the Gaussians in depth order; tiling restricts each pixel to the
// Gaussians whose tile rectangle covers its tile.  The order wanted is that of the 64-bit key
// (global tile << 32 | depth bits), ties by Gaussian index.  All pairs of one (view, Gaussian) share the
// depth bits, so the pairs are only ever sorted by their tile bits (2 passes for up to 65,536 tiles), and the
// depth order comes from one of two routes:
//   * short tile lists (the capacity allows at most 512 pairs per tile on average): the pairs are emitted in
//     (view, Gaussian) order, the stable tile sort keeps that order within each tile, and one wavefront per
//     tile sorts its list by (depth bits, position) -- by depth, ties by Gaussian index;
//   * otherwise the depth bits are sorted once per (view, Gaussian) by 4 radix passes over V*n items (instead
//     of 4 passes over P pairs), and the pairs are emitted in that order.
//
// Every 8-bit pass is reduce-then-scan, three kernels with no waits between workgroups: each block counts
// its items' digits, one workgroup per digit scans those counts over the blocks, and each block then
// places its items (stable ranks by wave64 ballot matching on the digit bits, per-wave digit counters in
// LDS), orders them by digit in LDS and writes them out in digit runs.  The first depth pass makes its keys
// from the projection on the fly.  The per-(view, Gaussian) tile counts are scanned the same way, without
// waits: each block sums its items' counts, then each block adds up the sums of the blocks before it, scans
// its own items and writes the items that have pairs, compacted, for the emission kernel.
#include <algorithm>
#include <mutex>

#include "qg_internal.h"

namespace qg {

namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
// Threads per radix block above 2^22 items: 8192 items per block, so each block's digit runs (and the
// contiguous writes they make) are twice as long as with 256 threads.
constexpr int kRsBigBlock = 512;
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

// Block-wide exclusive scan of one value per thread; *total = block sum.
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

// Counts digit d of this lane into the LDS histogram h.  When every active lane of the wave holds the same
// digit (the high digits of neighbouring keys usually agree) one lane adds the wave's count, instead of 64
// atomics on one address.
__device__ __forceinline__ void hist_add(uint32_t* h, uint32_t d) {
    const uint64_t active = __ballot(true);
    const uint32_t first = __builtin_amdgcn_readfirstlane(d);
    const uint64_t same = __ballot(d == first);
    if (same == active) {
        if (__lane_id() == (uint32_t)(__ffsll((unsigned long long)active) - 1))
            atomicAdd(&h[first], (uint32_t)__popcll(active));
    } else {
        atomicAdd(&h[d], 1u);
    }
}

// ------------------------------------------------------------------------------------------------
// One stable 8-bit radix pass: reduce, then scan, then scatter.
// Block b owns IPT * 256 consecutive items; item r of lane l in wave w sits at b*TILE + w*(IPT*64) + r*64 + l
// (wave-contiguous, so within a wave the rounds are in element order and the waves are in element order).
//   k_rs_count: the block's digit counts -> cnt[d * nb_cap + b] (digit-major);
//   k_rs_scan: per digit (one workgroup each), the exclusive scan of its counts over the blocks in place, and
//              the digit's total;
//   k_rs_scatter: the block's stable ranks (ballot matching), its digits' output starts (digit base from the
//              totals + the scanned count of the earlier blocks), ordered through LDS and written by digit runs,
//              so neighbouring threads write neighbouring words.
// The item count is read on the device (count_ptr) or given (count_ptr == nullptr: count_fixed).  With
// kGen (the first depth pass) there is no input array: item k = v*n + i is (view v, Gaussian i), its key the
// bits of its depth (0xFFFFFFFF, last, if its rectangle is empty) and its value k.
// ------------------------------------------------------------------------------------------------
struct RsSrc {
    const uint32_t* keys;  // [count], or nullptr with kGen
    const uint32_t* vals;
    const float* depth[QG_MAX_VIEWS];
    const int32_t* ntiles[QG_MAX_VIEWS];
    int64_t n;
};

template <bool kGen>
__device__ __forceinline__ uint32_t rs_key(const RsSrc& src, uint64_t idx) {
    if constexpr (kGen) {
        const int v = (int)(idx / (uint64_t)src.n);
        const int64_t i = (int64_t)idx - (int64_t)v * src.n;
        return src.ntiles[v][i] > 0 ? __float_as_uint(src.depth[v][i]) : 0xFFFFFFFFu;
    } else {
        return src.keys[idx];
    }
}

template <bool kGen>
__device__ __forceinline__ uint32_t rs_val(const RsSrc& src, uint64_t idx) {
    if constexpr (kGen)
        return (uint32_t)idx;
    else
        return src.vals[idx];
}

template <int IPT, int BLK, bool kGen>
__global__ __launch_bounds__(BLK) void k_rs_count(RsSrc src, const uint32_t* __restrict__ count_ptr,
                                                  uint32_t count_fixed, int pass, uint32_t* __restrict__ cnt,
                                                  int64_t nb_cap) {
    constexpr int kTile = IPT * BLK;
    __shared__ uint32_t s_h[kRadix];
    const uint32_t count = count_ptr ? *count_ptr : count_fixed;
    const uint64_t blk0 = (uint64_t)blockIdx.x * kTile;
    if (blk0 >= count) return;
    if (threadIdx.x < kRadix) s_h[threadIdx.x] = 0;
    __syncthreads();
    const int w = threadIdx.x / kWave, lane = __lane_id();
    const uint64_t base = blk0 + (uint64_t)w * (IPT * kWave);
    const int shift = kRadixBits * pass;
    uint32_t key[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t idx = base + (uint64_t)r * kWave + lane;
        key[r] = idx < count ? rs_key<kGen>(src, idx) : 0u;
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t idx = base + (uint64_t)r * kWave + lane;
        if (idx < count) hist_add(s_h, (key[r] >> shift) & (kRadix - 1));
    }
    __syncthreads();
    if (threadIdx.x < kRadix) cnt[(size_t)threadIdx.x * nb_cap + blockIdx.x] = s_h[threadIdx.x];
}

// One workgroup per digit: exclusive scan of cnt[d][0 .. nb) in place, nb from the item count; tot[d] = total.
constexpr int kRsScanThreads = 1024;

template <int IPT, int BLK>
__global__ __launch_bounds__(kRsScanThreads) void k_rs_scan(uint32_t* __restrict__ cnt, int64_t nb_cap,
                                                            const uint32_t* __restrict__ count_ptr,
                                                            uint32_t count_fixed, uint32_t* __restrict__ tot) {
    __shared__ uint32_t s_w[kRsScanThreads / kWave];
    const int64_t nb = ceil_div((int64_t)(count_ptr ? *count_ptr : count_fixed), IPT * BLK);
    uint32_t* row = cnt + (size_t)blockIdx.x * nb_cap;
    const int tid = threadIdx.x, w = tid / kWave, lane = __lane_id();
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kRsScanThreads) {
        const int64_t b = b0 + tid;
        const uint32_t x = b < nb ? row[b] : 0u;
        const uint32_t inc = wave_incl_scan(x);
        if (lane == kWave - 1) s_w[w] = inc;
        __syncthreads();
        uint32_t wb = 0, all = 0;
#pragma unroll
        for (int k = 0; k < kRsScanThreads / kWave; ++k) {
            if (k < w) wb += s_w[k];
            all += s_w[k];
        }
        if (b < nb) row[b] = carry + wb + inc - x;
        carry += all;
        __syncthreads();
    }
    if (tid == 0) tot[blockIdx.x] = carry;
}

template <int IPT, int BLK, bool kGen>
__global__ __launch_bounds__(BLK) void k_rs_scatter(RsSrc src, uint32_t* __restrict__ kout,
                                                       uint32_t* __restrict__ vout,
                                                       const uint32_t* __restrict__ count_ptr, uint32_t count_fixed,
                                                       int pass, const uint32_t* __restrict__ cnt, int64_t nb_cap,
                                                       const uint32_t* __restrict__ tot) {
    constexpr int kTile = IPT * BLK;
    constexpr int kW = BLK / kWave;
    __shared__ uint32_t s_cnt[kW][kRadix];
    __shared__ uint32_t s_w[kW];
    __shared__ uint32_t s_goff[kRadix];
    __shared__ uint32_t s_key[kTile], s_val[kTile];
    const int tid = threadIdx.x, w = tid / kWave, lane = __lane_id();
    const uint32_t count = count_ptr ? *count_ptr : count_fixed;
    const uint64_t blk0 = (uint64_t)blockIdx.x * kTile;
    if (blk0 >= count) return;
    const uint64_t base = blk0 + (uint64_t)w * (IPT * kWave);
    uint32_t key[IPT], val[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t idx = base + (uint64_t)r * kWave + lane;
        const bool valid = idx < count;
        key[r] = valid ? rs_key<kGen>(src, idx) : 0u;
        val[r] = valid ? rs_val<kGen>(src, idx) : 0u;
    }
    // output start of digit tid before this block: digit base (scan of the totals) + the earlier blocks' count
    const bool dig = tid < kRadix;  // this thread also stands for digit tid
    const uint32_t before = dig ? cnt[(size_t)tid * nb_cap + blockIdx.x] : 0u;
    uint32_t dtot;
    const uint32_t dbase = block_excl_scan<uint32_t>(dig ? tot[tid] : 0u, s_w, &dtot);
    const int shift = kRadixBits * pass;
    for (int i = tid; i < kW * kRadix; i += BLK) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    // per-wave digit counts; each item keeps its rank among the equal digits of its round, the round's count
    // of that digit and the lowest lane holding it (8 | 8 | 16 bits)
    uint32_t info[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t idx = base + (uint64_t)r * kWave + lane;
        const bool valid = idx < count;
        const uint32_t d = (key[r] >> shift) & (kRadix - 1);
        const uint64_t m = match8(d, valid);
        const uint32_t rank = (uint32_t)__popcll(m & lanemask_lt()), c = (uint32_t)__popcll(m);
        if (valid && rank == 0) atomicAdd(&s_cnt[w][d], c);
        info[r] = rank | (c << 8) | ((uint32_t)(__ffsll((unsigned long long)m) - 1) << 16);
        __builtin_amdgcn_sched_barrier(0);  // one round at a time: the rounds' masks are not kept live together
    }
    __syncthreads();
    // block-local start of digit tid (digits in order), and per-wave local starts within it
    uint32_t btot = 0;
    if (dig) {
#pragma unroll
        for (int k = 0; k < kW; ++k) btot += s_cnt[k][tid];
    }
    uint32_t ntot;
    const uint32_t lbase = block_excl_scan<uint32_t>(btot, s_w, &ntot);
    if (dig) {
        s_goff[tid] = dbase + before - lbase;
        uint32_t run = lbase;
#pragma unroll
        for (int k = 0; k < kW; ++k) {
            const uint32_t c = s_cnt[k][tid];
            s_cnt[k][tid] = run;
            run += c;
        }
    }
    __syncthreads();
    // stable ranks, items to their block-local places in digit order
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t idx = base + (uint64_t)r * kWave + lane;
        const bool valid = idx < count;
        const uint32_t d = (key[r] >> shift) & (kRadix - 1);
        const uint32_t rank = info[r] & 0xffu;
        uint32_t start = 0;
        if (valid && rank == 0) start = atomicAdd(&s_cnt[w][d], (info[r] >> 8) & 0xffu);
        start = __shfl(start, valid ? (int)(info[r] >> 16) : 0);  // a valid lane's digit group holds itself
        if (valid) {
            const uint32_t pos = start + rank;
            s_key[pos] = key[r];
            s_val[pos] = val[r];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // the block's items in digit order (ntot of them) to their output positions
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t i = (uint32_t)(r * BLK + tid);
        if (i < ntot) {
            const uint32_t k = s_key[i];
            const uint32_t pos = i + s_goff[(k >> shift) & (kRadix - 1)];
            kout[pos] = k;
            vout[pos] = s_val[i];
        }
    }
}

// Items per thread of a pass over up to max_count items: 4 for up to 2^20 items (a wider grid), else 16; and
// threads per block: kRsBigBlock above 2^22 items (longer digit runs per block, so longer contiguous writes).
int rs_ipt(int64_t max_count) { return max_count <= (1 << 20) ? 4 : 16; }
int rs_threads(int64_t max_count) { return max_count <= (1 << 22) ? kBlock : kRsBigBlock; }
int64_t rs_blocks(int64_t max_count) {
    return std::max<int64_t>(1, ceil_div(max_count, (int64_t)rs_ipt(max_count) * rs_threads(max_count)));
}

// One pass from src to (kout, vout); cnt holds [256][nb_cap] counts with nb_cap >= rs_blocks(max_count).
template <int IPT, int BLK, bool kGen>
void rs_launch(const RsSrc& src, uint32_t* kout, uint32_t* vout, const uint32_t* count_ptr, uint32_t count_fixed,
               int64_t max_count, int pass, uint32_t* cnt, int64_t nb_cap, uint32_t* tot, hipStream_t s) {
    const unsigned nb = (unsigned)std::max<int64_t>(1, ceil_div(max_count, IPT * BLK));
    k_rs_count<IPT, BLK, kGen><<<nb, BLK, 0, s>>>(src, count_ptr, count_fixed, pass, cnt, nb_cap);
    k_rs_scan<IPT, BLK><<<kRadix, kRsScanThreads, 0, s>>>(cnt, nb_cap, count_ptr, count_fixed, tot);
    k_rs_scatter<IPT, BLK, kGen><<<nb, BLK, 0, s>>>(src, kout, vout, count_ptr, count_fixed, pass, cnt, nb_cap, tot);
}

template <bool kGen>
qg_status rs_pass(const RsSrc& src, uint32_t* kout, uint32_t* vout, const uint32_t* count_ptr, uint32_t count_fixed,
                  int64_t max_count, int pass, uint32_t* cnt, int64_t nb_cap, uint32_t* tot, hipStream_t s,
                  const char* tag) {
    {
        QG_TIMED(tag, s);
        if (rs_ipt(max_count) == 4)
            rs_launch<4, kBlock, kGen>(src, kout, vout, count_ptr, count_fixed, max_count, pass, cnt, nb_cap, tot, s);
        else if (rs_threads(max_count) == kBlock)
            rs_launch<16, kBlock, kGen>(src, kout, vout, count_ptr, count_fixed, max_count, pass, cnt, nb_cap, tot, s);
        else
            rs_launch<16, kRsBigBlock, kGen>(src, kout, vout, count_ptr, count_fixed, max_count, pass, cnt, nb_cap, tot, s);
    }
    QG_LAUNCH_CHECK("radix pass");
    return QG_OK;
}

// ------------------------------------------------------------------------------------------------
// Binning kernels
// ------------------------------------------------------------------------------------------------
// Zeroes the tile ranges, num_pairs and the sort count
// (one grid-stride pass over a list of word ranges).
struct ZeroList {
    uint32_t* p[8];
    int64_t words[8];
    int n;
};

__global__ void k_bin_init(ZeroList z) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int k = 0; k < z.n; ++k)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < z.words[k]; i += stride) z.p[k][i] = 0u;
}

// Exclusive scan (64-bit) of the tile counts of the items in order (depth order, or item order when `sorted` is
// null), reduce then apply: k_count_reduce sums each block's items (pairs and items with a non-empty
// rectangle) and clears the tile ranges; k_count_apply adds up the sums of the blocks before its own, scans its
// items, and writes the items with a non-empty rectangle in order, compacted, with their first pair positions
// (comp_item, comp_offs).  Its last block writes the total, the tile sort's count (0 on overflow), the number of
// compacted items and the caller's num_pairs.  A thread owns kScanIPT consecutive items.
constexpr int kScanIPT = 4;
constexpr int kScanTile = kBlock * kScanIPT;

__device__ __forceinline__ uint32_t item_at(const uint32_t* sorted, int64_t k) {
    return sorted ? sorted[k] : (uint32_t)k;
}

__device__ __forceinline__ uint64_t item_tiles(const ViewTable& vt, int64_t n, uint32_t item) {
    int v = 0;
    while (v + 1 < vt.V && (int64_t)item >= (int64_t)(v + 1) * n) ++v;
    return (uint64_t)vt.proj[v].ntiles[(int64_t)item - (int64_t)v * n];
}

__global__ __launch_bounds__(kBlock) void k_count_reduce(int64_t items, int64_t n, ViewTable vt,
                                                         const uint32_t* __restrict__ sorted,
                                                         uint64_t* __restrict__ bsum, uint32_t* __restrict__ vsum,
                                                         uint32_t* __restrict__ ranges, int64_t range_words) {
    __shared__ uint64_t s_w[kWaves];
    __shared__ uint32_t s_v[kWaves];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < range_words; i += (int64_t)gridDim.x * kBlock)
        ranges[i] = 0u;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
    uint64_t acc = 0;
    uint32_t vis = 0;
#pragma unroll
    for (int r = 0; r < kScanIPT; ++r) {
        const int64_t k = base + r;
        if (k < items) {
            const uint64_t c = item_tiles(vt, n, item_at(sorted, k));
            acc += c;
            vis += c > 0;
        }
    }
    uint64_t tot;
    block_excl_scan<uint64_t>(acc, s_w, &tot);
    uint32_t vtot;
    block_excl_scan<uint32_t>(vis, s_v, &vtot);
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = tot;
        vsum[blockIdx.x] = vtot;
    }
}

__global__ __launch_bounds__(kBlock) void k_count_apply(int64_t items, int64_t n, ViewTable vt,
                                                        const uint32_t* __restrict__ sorted,
                                                        const uint64_t* __restrict__ bsum,
                                                        const uint32_t* __restrict__ vsum,
                                                        uint32_t* __restrict__ comp_item,
                                                        uint64_t* __restrict__ comp_offs, int64_t capacity,
                                                        uint32_t* __restrict__ sort_count,
                                                        uint32_t* __restrict__ n_comp,
                                                        uint32_t* __restrict__ long_count,
                                                        int64_t* __restrict__ num_pairs) {
    __shared__ uint64_t s_w[kWaves];
    __shared__ uint32_t s_v[kWaves];
    // start of this block: the sums of the blocks before it
    uint64_t pre = 0;
    uint32_t vpre = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kBlock) {
        pre += bsum[b];
        vpre += vsum[b];
    }
    uint64_t start;
    block_excl_scan<uint64_t>(pre, s_w, &start);
    uint32_t vstart;
    block_excl_scan<uint32_t>(vpre, s_v, &vstart);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
    uint64_t c[kScanIPT];
    uint32_t it[kScanIPT];
    uint64_t acc = 0;
    uint32_t vis = 0;
#pragma unroll
    for (int r = 0; r < kScanIPT; ++r) {
        const int64_t k = base + r;
        it[r] = k < items ? item_at(sorted, k) : 0u;
        c[r] = k < items ? item_tiles(vt, n, it[r]) : 0;
        acc += c[r];
        vis += c[r] > 0;
    }
    uint64_t btot;
    const uint64_t ex = block_excl_scan<uint64_t>(acc, s_w, &btot);
    uint32_t vbtot;
    const uint32_t vex = block_excl_scan<uint32_t>(vis, s_v, &vbtot);
    if (threadIdx.x == 0 && (int64_t)(blockIdx.x + 1) * kScanTile >= items) {  // the last block
        const uint64_t t = start + btot;
        *num_pairs = (int64_t)t;
        *sort_count = t <= (uint64_t)capacity ? (uint32_t)t : 0u;
        *n_comp = vstart + vbtot;
        *long_count = 0u;
    }
    uint64_t run = start + ex;
    uint32_t slot = vstart + vex;
#pragma unroll
    for (int r = 0; r < kScanIPT; ++r) {
        if (c[r] > 0) {
            comp_item[slot] = it[r];
            comp_offs[slot] = run;
            ++slot;
        }
        run += c[r];
    }
}

// Emission, load-balanced whatever the rectangle sizes: a block owns 1024 consecutive output positions, four
// consecutive ones per thread.  The compacted items that cover them are consecutive (each owns at least one
// position), so at most 1024 of them do, and the block loads their offsets into LDS; a thread finds the item
// of its first position by binary search there and walks forward for the next three, and writes its four keys
// and values with one 16-byte store each.
constexpr int kEmitPer = 1024;
constexpr int kEmitPerThread = kEmitPer / 256;

// A block takes per_block consecutive chunks: the first item of each later chunk is read off the previous
// chunk's LDS window when the window reaches it, so only the first chunk pays the search over offs.
__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ n_comp, int64_t n, ViewTable vt,
                                              const uint32_t* __restrict__ comp_item,
                                              const uint64_t* __restrict__ offs,
                                              const uint32_t* __restrict__ sort_count,
                                              uint32_t* __restrict__ tkeys, uint32_t* __restrict__ tvals,
                                              int64_t per_block) {
    __shared__ uint64_t s_off[kEmitPer + 1];
    __shared__ int64_t s_k0, s_next;
    const uint64_t P = *sort_count;
    const int64_t items = *n_comp;  // >= 1 whenever P > 0
    if (threadIdx.x == 0) s_next = -1;
    const int64_t c_end = ((int64_t)blockIdx.x + 1) * per_block;
    for (int64_t chunk = (int64_t)blockIdx.x * per_block; chunk < c_end && (uint64_t)chunk * kEmitPer < P; ++chunk) {
        const uint64_t base = (uint64_t)chunk * kEmitPer;
        __syncthreads();  // the previous chunk is done with s_off, and s_next is set
        const int64_t carried = s_next;
        if (carried >= 0) {
            if (threadIdx.x == 0) s_k0 = carried;
        } else if (threadIdx.x < kWave) {
            // last k with offs[k] <= base (offs is non-decreasing, offs[0] = 0): 64 probes per round, so the
            // range shrinks 64-fold per dependent load
            const int lane = (int)threadIdx.x;
            int64_t lo = 0, hi = items - 1;
            while (hi > lo) {
                const int64_t step = (hi - lo + kWave - 1) / kWave;
                const int64_t pos = lo + (int64_t)(lane + 1) * step;
                const bool le = pos <= hi && offs[pos] <= base;
                const int cnt = (int)__popcll(__ballot(le));
                lo += (int64_t)cnt * step;
                hi = std::min<int64_t>(hi, lo + step - 1);
            }
            if (lane == 0) s_k0 = lo;
        }
        __syncthreads();
        const int64_t k0 = s_k0;
        // the window: the offsets of items k0, k0 + 1, ..., 256 at a time, until one starts past the chunk (the
        // chunk's 1024 positions belong to at most 1024 items, so at most kEmitPer + 1 entries; past the last
        // item a sentinel)
        const uint64_t nb = base + kEmitPer;  // the next chunk's first position
        int wn = 0;
        for (;;) {
            const int t = wn + (int)threadIdx.x;
            if (t <= kEmitPer) {
                const int64_t k = k0 + t;
                s_off[t] = k < items ? offs[k] : ~0ull;
            }
            __syncthreads();
            wn = std::min(wn + 256, kEmitPer + 1);
            if (wn > kEmitPer || s_off[wn - 1] >= nb) break;
        }
        if (threadIdx.x == 0) {
            // the next chunk's first item, from this window when it holds it (items with pairs have increasing
            // offsets), else found by the search
            int64_t nx = -1;
            if (s_off[wn - 1] == nb) {
                nx = k0 + wn - 1;
            } else if (s_off[wn - 1] > nb) {
                int lo = 0, hi = wn - 2;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= nb)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                nx = k0 + lo;
            }
            s_next = nx;
        }
        const uint64_t p0 = base + (uint64_t)threadIdx.x * kEmitPerThread;
        if (p0 >= P) continue;
        int lo = 0, hi = wn - 2;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= p0)
                lo = mid;
            else
                hi = mid - 1;
        }
        uint32_t key[kEmitPerThread], val[kEmitPerThread];
        int cur = -1;
        uint32_t w = 1, x0 = 0, y0 = 0, toff = 0, gw = 0, gi = 0;
        float inv_w = 1.f;
#pragma unroll
        for (int j = 0; j < kEmitPerThread; ++j) {
            const uint64_t p = p0 + j;
            key[j] = val[j] = 0u;
            if (p >= P) continue;
            while (s_off[lo + 1] <= p) ++lo;  // the owner of p (s_off[wn - 1] lies past the chunk: the walk stops)
            if (lo != cur) {
                cur = lo;
                const uint32_t item = comp_item[k0 + lo];
                int v = 0;
                while (v + 1 < vt.V && (int64_t)item >= (int64_t)(v + 1) * n) ++v;
                gi = (uint32_t)((int64_t)item - (int64_t)v * n);
                const int4 r = reinterpret_cast<const int4*>(vt.proj[v].rect)[gi];
                w = (uint32_t)(r.z - r.x);
                x0 = (uint32_t)r.x;
                y0 = (uint32_t)r.y;
                toff = vt.cam[v].tile_off;
                gw = (uint32_t)vt.cam[v].grid_w;
                inv_w = 1.f / (float)w;
            }
            // (row, column) of the j-th tile of the rectangle: j < 2^22, so the float quotient is within one of
            // the integer quotient, and one correction step makes it exact
            const uint32_t jj = (uint32_t)(p - s_off[lo]);
            uint32_t q = (uint32_t)((float)jj * inv_w);
            int rr = (int)jj - (int)(q * w);
            if (rr < 0) {
                --q;
                rr += (int)w;
            } else if (rr >= (int)w) {
                ++q;
                rr -= (int)w;
            }
            key[j] = toff + (y0 + q) * gw + x0 + (uint32_t)rr;
            val[j] = gi;
        }
        // (tkeys is workspace, 256-byte aligned; tvals may be the caller's array, which need not be)
        if (p0 + kEmitPerThread <= P && (reinterpret_cast<uintptr_t>(tvals) & 15) == 0) {
            *reinterpret_cast<uint4*>(tkeys + p0) = make_uint4(key[0], key[1], key[2], key[3]);
            *reinterpret_cast<uint4*>(tvals + p0) = make_uint4(val[0], val[1], val[2], val[3]);
        } else {
#pragma unroll
            for (int j = 0; j < kEmitPerThread; ++j)
                if (p0 + j < P) {
                    tkeys[p0 + j] = key[j];
                    tvals[p0 + j] = val[j];
                }
        }
    }
}

// Tile ranges from the sorted keys, four positions per thread (one 16-byte load and the two neighbours).
constexpr int kRangesPerThread = 4;

__global__ void k_ranges(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ sort_count,
                         uint32_t* __restrict__ ranges) {
    const uint64_t P = *sort_count;
    const uint64_t p0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangesPerThread;
    if (p0 >= P) return;
    uint32_t k[kRangesPerThread + 1];
    if (p0 + kRangesPerThread <= P) {
        const uint4 q = *reinterpret_cast<const uint4*>(tkeys + p0);
        k[0] = q.x;
        k[1] = q.y;
        k[2] = q.z;
        k[3] = q.w;
    } else {
#pragma unroll
        for (int j = 0; j < kRangesPerThread; ++j) k[j] = p0 + j < P ? tkeys[p0 + j] : 0u;
    }
    k[kRangesPerThread] = p0 + kRangesPerThread < P ? tkeys[p0 + kRangesPerThread] : 0u;
    uint32_t prev = p0 > 0 ? tkeys[p0 - 1] : 0u;
#pragma unroll
    for (int j = 0; j < kRangesPerThread; ++j) {
        const uint64_t p = p0 + j;
        if (p >= P) break;
        const uint32_t t = k[j];
        if (p == 0 || prev != t) ranges[2 * (size_t)t] = (uint32_t)p;
        if (p + 1 == P || k[j + 1] != t) ranges[2 * (size_t)t + 1] = (uint32_t)p + 1;
        prev = t;
    }
}

// ------------------------------------------------------------------------------------------------
// Per-tile depth order.  When every tile's list is short, the pairs are emitted in (view, Gaussian) order
// instead of depth order, and the stable tile sort then leaves each tile's list in Gaussian order.  Each list
// is then sorted by the key (depth bits << 32 | Gaussian), the depth bits being the ones the depth passes
// sort by (a tile's Gaussians all belong to its view).  A Gaussian appears at most once in a list, so the
// keys are distinct, and equal depths stay in Gaussian order, the order the depth passes leave them in: the
// result equals the depth-first order, and the sorted keys' low words are the list itself.
// Lists of up to kSegCap entries: one wavefront per tile, a bitonic network over the next power of two in
// registers (64 E keys, E consecutive keys per lane; exchanges between keys less than E apart stay in the
// lane, the others pair lane l with lane l ^ (distance / E)).  Longer lists are put on a work list that
// k_seg_sort_long takes: a 512-thread block per list, merge-sorting lists of up to kLongCap entries in LDS;
// longer ones are sorted run by run (kLongCap keys each) in LDS, and the runs merged by a bitonic network
// through global memory.
// ------------------------------------------------------------------------------------------------
constexpr int kSegCap = 1024;
constexpr int kLongThreads = 512;
constexpr int kChunk = 1024;     // keys per wavefront in the register half-cleaners: 16 per lane
constexpr int kLongCap = 8192;   // keys k_seg_sort_long keeps in LDS (64 KiB)

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The value of lane l ^ M (M a constant).  Inside a 16-lane row the exchange runs on the vector unit by DPP (quad
// permutations for 1, 2 and 3; row rotations by 8, and by 4 and 12 with a select, since lane l - n is rotation
// n's source; the half-row and row mirrors for 7 and 15); across rows by a lane shuffle through the LDS
// crossbar.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, true);
}

template <int M>
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t v) {
    if constexpr (M == 1) {
        return dpp_u32<0xB1>(v);  // quad_perm [1, 0, 3, 2]
    } else if constexpr (M == 2) {
        return dpp_u32<0x4E>(v);  // quad_perm [2, 3, 0, 1]
    } else if constexpr (M == 3) {
        return dpp_u32<0x1B>(v);  // quad_perm [3, 2, 1, 0]
    } else if constexpr (M == 7) {
        return dpp_u32<0x141>(v);  // row_half_mirror
    } else if constexpr (M == 15) {
        return dpp_u32<0x140>(v);  // row_mirror
    } else if constexpr (M == 8) {
        return dpp_u32<0x128>(v);  // row_ror:8
    } else if constexpr (M == 4) {
        const uint32_t a = dpp_u32<0x124>(v), b = dpp_u32<0x12C>(v);  // row_ror:4 (lane l - 4), row_ror:12 (l + 4)
        return (__lane_id() & 4) ? a : b;
    } else {
        return (uint32_t)__shfl_xor((int)v, M);
    }
}

template <int M>
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t x) {
    const uint32_t lo = xor_lane_u32<M>((uint32_t)x), hi = xor_lane_u32<M>((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t min64(uint64_t a, uint64_t b) { return b < a ? b : a; }
__device__ __forceinline__ uint64_t max64(uint64_t a, uint64_t b) { return b < a ? a : b; }

// Sort key of Gaussian g in a tile list: depth bits above, the Gaussian below.
__device__ __forceinline__ uint64_t seg_key(const float* __restrict__ depth, uint32_t g) {
    return ((uint64_t)__float_as_uint(depth[g]) << 32) | g;
}

// Ascending bitonic sort of the wave's 64 E keys; lane l holds keys l E .. l E + E - 1 in x.  The network's
// levels K and distances J are template arguments, so that every exchange compiles to straight-line code.
template <int E, int K, int J>
__device__ __forceinline__ void wave_bitonic_stage(uint64_t (&x)[E]) {
    const int lane = __lane_id();
    if constexpr (J >= E) {
        // partner key in lane ^ (J / E), same register; the lower lane of the pair keeps the minimum in an
        // ascending run (bit K of the key index clear), the maximum in a descending one: a lane takes its
        // partner's key when (key < partner's) differs from "keep the minimum" (keys are distinct except the
        // equal padding keys, where either choice is the same)
        constexpr int M = J / E;
        const bool keep_max = ((lane & M) == 0) != (((lane * E) & K) == 0);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint64_t o = xor_lane_u64<M>(x[r]);
            const bool take = (x[r] < o) == keep_max;
            x[r] = take ? o : x[r];
        }
    } else {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            if (r & J) continue;
            // swap when the pair is out of order for its run's direction
            const bool desc = K < E ? (r & K) != 0 : ((lane * E) & K) != 0;
            const uint64_t a = x[r], b = x[r ^ J];
            const bool sw = (b < a) != desc;
            x[r] = sw ? b : a;
            x[r ^ J] = sw ? a : b;
        }
    }
}

template <int E, int K, int J>
__device__ __forceinline__ void wave_bitonic_merge(uint64_t (&x)[E]) {
    if constexpr (J > 0) {
        wave_bitonic_stage<E, K, J>(x);
        wave_bitonic_merge<E, K, J / 2>(x);
    }
}

template <int E, int K = 2>
__device__ __forceinline__ void wave_bitonic(uint64_t (&x)[E]) {
    if constexpr (K <= kWave * E) {
        wave_bitonic_merge<E, K, K / 2>(x);
        wave_bitonic<E, 2 * K>(x);
    }
}

// Sorts the tile list src[0 .. L) (L <= 64 E) in registers.
template <int E>
__device__ __forceinline__ void seg_sort_regs(uint32_t* __restrict__ src, uint32_t L, const float* __restrict__ depth) {
    const int lane = __lane_id();
    uint64_t x[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t e = (uint32_t)(lane * E + r);
        x[r] = e < L ? seg_key(depth, src[e]) : ~0ull;  // padding: after every key of the list
    }
    wave_bitonic<E>(x);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t e = (uint32_t)(lane * E + r);
        if (e < L) src[e] = (uint32_t)x[r];
    }
}

// ---- k_seg_sort_long.  Lists over kLongCap entries: sorted runs of kLongCap keys are merged by the bitonic
// network in the form whose every exchange keeps the smaller key at the lower index (each merge level k
// opens by comparing key i with its mirror image in the level's block, i ^ (k - 1), and continues with
// half-cleaners i, i + j).  Keys past the list's end count as +infinity: an exchange with one of them never
// moves it, so the network runs on any length without padding the list in memory.  Half-cleaners at
// distances below kLongCap run in LDS, those below kChunk = 1024 in registers, a wavefront's 1024 keys
// strided: lane l, register r holds chunk key l + 64 r (distances below 64 pair lanes, 64 and above
// registers; the chunk's LDS loads and stores are consecutive across lanes).

// Half-cleaner at distance J over the chunk x, every pair ascending.
template <int J>
__device__ __forceinline__ void chunk_half(uint64_t (&x)[16]) {
    if constexpr (J >= 64) {
        constexpr int M = J >> 6;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (r & M) continue;
            const uint64_t a = x[r], b = x[r | M];
            x[r] = min64(a, b);
            x[r | M] = max64(a, b);
        }
    } else {
        const bool lower = (__lane_id() & J) == 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint64_t o = xor_lane_u64<J>(x[r]);
            x[r] = lower ? min64(x[r], o) : max64(x[r], o);
        }
    }
}

template <int J>
__device__ __forceinline__ void chunk_halves(uint64_t (&x)[16]) {
    if constexpr (J > 0) {
        chunk_half<J>(x);
        chunk_halves<J / 2>(x);
    }
}

__device__ __forceinline__ void chunk_merge(uint64_t (&x)[16]) { chunk_halves<kChunk / 2>(x); }

// One exchange over keys i < p < n of s[]: the smaller stays at i.
__device__ __forceinline__ void lds_exchange(uint64_t* s, uint32_t i, uint32_t p) {
    const uint64_t a = s[i], b = s[p];
    if (b < a) {
        s[i] = b;
        s[p] = a;
    }
}

// The merge sort keeps key i at s[i + i / 16]: one unused slot per 16 keys, so that lanes reading keys a few
// apart (a thread's outputs are 4 to 16 keys from its neighbour's) fall in different LDS banks.
constexpr int kLongSlots = kLongCap + kLongCap / 16;
__device__ __forceinline__ uint32_t lds_pad(uint32_t i) { return i + (i >> 4); }

// Merge sort of keys 0 .. n - 1 (key(i) gives key i; n <= kLongThreads * IPT) into s (padded): runs of 256 keys
// sorted by one wavefront each in registers (four per lane), then pairs of runs merged level by level.  Thread t produces
// outputs t IPT .. t IPT + IPT - 1 of its pair of runs (the pair's length, twice the run, is a multiple of
// IPT): a binary search along the merge path finds how many of the first ones come from each run, IPT
// merge steps collect them in registers, and after a barrier they overwrite s in place.
template <int IPT, class Key>
__device__ __forceinline__ void lds_sort_run(uint64_t* s, uint32_t n, const Key& key) {
    static_assert(IPT <= 2 * kWave, "a thread's outputs must lie in one pair of runs");
    const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    // the keys, a thread's loads issued 16 at a time before the stores
    constexpr int G = IPT < 16 ? IPT : 16;
#pragma unroll
    for (int r0 = 0; r0 < IPT; r0 += G) {
        uint64_t x[G];
#pragma unroll
        for (int r = 0; r < G; ++r) {
            const uint32_t e = tid + (uint32_t)(r0 + r) * kLongThreads;
            x[r] = e < n ? key(e) : ~0ull;
        }
#pragma unroll
        for (int r = 0; r < G; ++r) {
            const uint32_t e = tid + (uint32_t)(r0 + r) * kLongThreads;
            if (e < n) s[lds_pad(e)] = x[r];
        }
    }
    __syncthreads();
    constexpr int kRunE = 4;
    constexpr uint32_t kRun = kWave * kRunE;
    for (uint32_t c = wave; c * kRun < n; c += kLongThreads / kWave) {
        uint64_t x[kRunE];
#pragma unroll
        for (int r = 0; r < kRunE; ++r) {
            const uint32_t e = c * kRun + lane * kRunE + r;
            x[r] = e < n ? s[lds_pad(e)] : ~0ull;
        }
        wave_bitonic<kRunE>(x);
#pragma unroll
        for (int r = 0; r < kRunE; ++r) {
            const uint32_t e = c * kRun + lane * kRunE + r;
            if (e < n) s[lds_pad(e)] = x[r];
        }
    }
    __syncthreads();
    const uint32_t o0 = tid * IPT;
    for (uint32_t run = kRun; run < n; run <<= 1) {
        uint64_t out[IPT];
        if (o0 < n) {
            const uint32_t b = o0 / (2 * run) * (2 * run);
            const uint32_t a1 = min(b + run, n), na = a1 - b, nb = min(b + 2 * run, n) - a1;
            const uint32_t d = o0 - b;
            // i = number of keys of the first run among the pair's first d outputs (keys are distinct)
            uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (s[lds_pad(b + mid)] < s[lds_pad(a1 + d - mid - 1)])
                    lo = mid + 1;
                else
                    hi = mid;
            }
            uint32_t i = lo, j = d - lo;
            uint64_t ka = i < na ? s[lds_pad(b + i)] : ~0ull, kb = j < nb ? s[lds_pad(a1 + j)] : ~0ull;
#pragma unroll
            for (int r = 0; r < IPT; ++r) {
                const bool ta = ka < kb;
                out[r] = ta ? ka : kb;
                i += ta;
                j += !ta;
                if (r + 1 < IPT) {
                    const bool ok = ta ? i < na : j < nb;
                    const uint64_t nk = ok ? s[lds_pad(ta ? b + i : a1 + j)] : ~0ull;
                    ka = ta ? nk : ka;
                    kb = ta ? kb : nk;
                }
            }
        }
        __syncthreads();
        if (o0 < n) {
#pragma unroll
            for (int r = 0; r < IPT; ++r)
                if (o0 + r < n) s[lds_pad(o0 + r)] = out[r];
        }
        __syncthreads();
    }
}

// Global-memory form for lists over kLongCap keys: key i of the list is hi[i] << 32 | lo[i] (lo = the list,
// hi = a spare array at the same positions).  All the block's global writes are complete, and no stale
// line of them in the vector cache, before any thread reads them.
__device__ __forceinline__ void block_global_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// One exchange stage over the list in global memory: pair(q, i, p) gives exchange q (of `half`); exchanges
// with p >= L are skipped.  A thread loads kGlobalBatch pairs before it compares and stores any of them.
constexpr int kGlobalBatch = 8;
template <class Pair>
__device__ __forceinline__ void global_stage(uint32_t* hi, uint32_t* lo, uint64_t L, uint64_t half, const Pair& pair) {
    for (uint64_t q0 = threadIdx.x; q0 < half; q0 += (uint64_t)kGlobalBatch * kLongThreads) {
        uint64_t i[kGlobalBatch], p[kGlobalBatch], a[kGlobalBatch], b[kGlobalBatch];
        bool ok[kGlobalBatch];
#pragma unroll
        for (int r = 0; r < kGlobalBatch; ++r) {
            const uint64_t q = q0 + (uint64_t)r * kLongThreads;
            pair(q, i[r], p[r]);
            ok[r] = q < half && p[r] < L;
            a[r] = ok[r] ? ((uint64_t)hi[i[r]] << 32) | lo[i[r]] : 0ull;
            b[r] = ok[r] ? ((uint64_t)hi[p[r]] << 32) | lo[p[r]] : 0ull;
        }
#pragma unroll
        for (int r = 0; r < kGlobalBatch; ++r) {
            if (ok[r] && b[r] < a[r]) {
                hi[i[r]] = (uint32_t)(b[r] >> 32);
                lo[i[r]] = (uint32_t)b[r];
                hi[p[r]] = (uint32_t)(a[r] >> 32);
                lo[p[r]] = (uint32_t)a[r];
            }
        }
    }
    block_global_sync();
}

__device__ void seg_sort_global(uint64_t* s, uint32_t* lo, uint32_t* hi, uint64_t L, const float* __restrict__ depth) {
    const uint32_t tid = threadIdx.x;
    const uint64_t runs = (L + kLongCap - 1) / kLongCap;
    // runs of kLongCap keys sorted in LDS, then stored as hi / lo
    for (uint64_t c = 0; c < runs; ++c) {
        const uint64_t b = c * kLongCap;
        const uint32_t n = (uint32_t)(L - b < (uint64_t)kLongCap ? L - b : (uint64_t)kLongCap);
        lds_sort_run<kLongCap / kLongThreads>(s, n, [&](uint32_t e) { return seg_key(depth, lo[b + e]); });
        for (uint32_t e = tid; e < n; e += kLongThreads) {
            const uint64_t k = s[lds_pad(e)];
            hi[b + e] = (uint32_t)(k >> 32);
            lo[b + e] = (uint32_t)k;
        }
        block_global_sync();
    }
    uint64_t npow = kLongCap;
    while (npow < L) npow <<= 1;
    for (uint64_t k = 2 * (uint64_t)kLongCap; k <= npow; k <<= 1) {
        const uint64_t h = k >> 1;
        global_stage(hi, lo, L, npow / 2, [&](uint64_t q, uint64_t& i, uint64_t& p) {
            i = (q / h) * k + q % h;
            p = i ^ (k - 1);
        });
        for (uint64_t j = k >> 2; j >= (uint64_t)kLongCap; j >>= 1)
            global_stage(hi, lo, L, npow / 2, [&](uint64_t q, uint64_t& i, uint64_t& p) {
                i = (q / j) * 2 * j + q % j;
                p = i + j;
            });
        // half-cleaners below kLongCap: run by run in LDS
        for (uint64_t c = 0; c < runs; ++c) {
            const uint64_t b = c * kLongCap;
            const uint32_t n = (uint32_t)(L - b < (uint64_t)kLongCap ? L - b : (uint64_t)kLongCap);
            const uint32_t nr = (n + kChunk - 1) / kChunk * kChunk;
            for (uint32_t e0 = tid; e0 < nr; e0 += kGlobalBatch * kLongThreads) {
                uint64_t x[kGlobalBatch];
#pragma unroll
                for (int r = 0; r < kGlobalBatch; ++r) {
                    const uint32_t e = e0 + r * kLongThreads;
                    x[r] = e < n ? ((uint64_t)hi[b + e] << 32) | lo[b + e] : ~0ull;
                }
#pragma unroll
                for (int r = 0; r < kGlobalBatch; ++r) {
                    const uint32_t e = e0 + r * kLongThreads;
                    if (e < nr) s[e] = x[r];
                }
            }
            __syncthreads();
            for (uint32_t j = kLongCap / 2; j >= (uint32_t)kChunk; j >>= 1) {
                for (uint32_t q = tid; q < kLongCap / 2; q += kLongThreads) {
                    const uint32_t i = (q / j) * 2 * j + q % j, p = i + j;
                    if (p < nr) lds_exchange(s, i, p);
                }
                __syncthreads();
            }
            const uint32_t wave = tid / kWave, lane = tid % kWave;
            for (uint32_t cc = wave; cc < nr / kChunk; cc += kLongThreads / kWave) {
                uint64_t x[16];
                uint64_t* sc = s + cc * kChunk + lane;
#pragma unroll
                for (int r = 0; r < 16; ++r) x[r] = sc[64 * r];
                chunk_merge(x);
#pragma unroll
                for (int r = 0; r < 16; ++r) sc[64 * r] = x[r];
            }
            __syncthreads();
            for (uint32_t e = tid; e < n; e += kLongThreads) {
                hi[b + e] = (uint32_t)(s[e] >> 32);
                lo[b + e] = (uint32_t)s[e];
            }
            block_global_sync();
        }
    }
}

// One wavefront per tile: lists of up to kSegCap entries sorted here, longer ones appended to long_list
// (long_count entries, at most max_long) for k_seg_sort_long.
__global__ __launch_bounds__(kWave) void k_seg_sort(ViewTable vt, const uint32_t* __restrict__ ranges,
                                                    uint32_t* __restrict__ vals, uint32_t* __restrict__ long_count,
                                                    uint32_t* __restrict__ long_list, uint32_t max_long, int64_t T) {
    const int64_t t = blockIdx.x;
    if (t >= T) return;
    const uint32_t start = ranges[2 * t], L = ranges[2 * t + 1] - start;
    if (L <= 1) return;
    if (L > (uint32_t)kSegCap) {
        if (__lane_id() == 0) {
            const uint32_t q = atomicAdd(long_count, 1u);
            if (q < max_long) long_list[q] = (uint32_t)t;
        }
        return;
    }
    int v = 0;
    for (int k = 1; k < vt.V; ++k)
        if ((uint32_t)t >= vt.cam[k].tile_off) v = k;
    const float* __restrict__ depth = vt.proj[v].depth;
    uint32_t* const src = vals + start;
    if (L <= 64) {
        seg_sort_regs<1>(src, L, depth);
    } else if (L <= 128) {
        seg_sort_regs<2>(src, L, depth);
    } else if (L <= 256) {
        seg_sort_regs<4>(src, L, depth);
    } else if (L <= 512) {
        seg_sort_regs<8>(src, L, depth);
    } else {
        seg_sort_regs<16>(src, L, depth);
    }
}

// One block per listed tile (the grid strides over the list; with an empty list every block returns at once).
// spare: a free array of the capacity, the high words of the keys of lists over kLongCap entries.
__global__ __launch_bounds__(kLongThreads) void k_seg_sort_long(ViewTable vt, const uint32_t* __restrict__ ranges,
                                                                uint32_t* __restrict__ vals,
                                                                uint32_t* __restrict__ spare,
                                                                const uint32_t* __restrict__ long_count,
                                                                const uint32_t* __restrict__ long_list,
                                                                uint32_t max_long) {
    __shared__ uint64_t s[kLongSlots];
    const uint32_t nl = min(*long_count, max_long);
    for (uint32_t q = blockIdx.x; q < nl; q += gridDim.x) {
        const uint32_t t = long_list[q];
        const uint32_t start = ranges[2 * t], L = ranges[2 * t + 1] - start;
        int v = 0;
        for (int k = 1; k < vt.V; ++k)
            if (t >= vt.cam[k].tile_off) v = k;
        const float* __restrict__ depth = vt.proj[v].depth;
        uint32_t* const src = vals + start;
        if (L <= (uint32_t)kLongCap) {
            const auto key = [&](uint32_t e) { return seg_key(depth, src[e]); };
            static_assert(kLongCap == 16 * kLongThreads, "outputs per thread: 4, 8 or 16");
            if (L <= 4u * kLongThreads)
                lds_sort_run<4>(s, L, key);
            else if (L <= 8u * kLongThreads)
                lds_sort_run<8>(s, L, key);
            else
                lds_sort_run<16>(s, L, key);
            for (uint32_t e = threadIdx.x; e < L; e += kLongThreads) src[e] = (uint32_t)s[lds_pad(e)];
        } else {
            seg_sort_global(s, src, spare + start, L, depth);
        }
        __syncthreads();  // s is reused by the next tile
    }
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

struct BinWs {
    uint32_t *dkA, *dkB, *dvA, *dvB;  // depth sort, V*n (dkB then holds the compacted items)
    uint64_t* offs;                   // V*n: first pair position of each compacted item
    uint32_t* sort_count;
    uint32_t* n_comp;                 // number of compacted items
    uint32_t* long_count;             // per-tile order: number of tile lists over kSegCap entries
    uint32_t* long_list;              // per-tile order: those tiles, [max_long]
    uint32_t max_long;
    uint32_t *tkA, *tkB, *tvB;        // tile sort, capacity
    uint32_t* rs_cnt;                 // radix passes: per-block digit counts [256][nb_cnt], scanned in place
    uint32_t* rs_tot;                 // radix passes: digit totals [256]
    uint64_t* bsum;                   // count scan: per-block pair sums, [blocks]
    uint32_t* vsum;                   // count scan: per-block counts of items with pairs, [blocks]
    int64_t nb_cnt, nb_scan;
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
    w.nb_cnt = std::max(rs_blocks(it1), rs_blocks(cap1));
    w.nb_scan = std::max<int64_t>(1, ceil_div(it1, kScanTile));
    w.dkA = (uint32_t*)take(4 * it1);
    w.dkB = (uint32_t*)take(4 * it1);
    w.dvA = (uint32_t*)take(4 * it1);
    w.dvB = (uint32_t*)take(4 * it1);
    w.offs = (uint64_t*)take(8 * it1);
    w.sort_count = (uint32_t*)take(4);
    w.n_comp = (uint32_t*)take(4);
    w.long_count = (uint32_t*)take(4);
    // lists over kSegCap entries: at most capacity / (kSegCap + 1) of them fit in the capacity
    w.max_long = (uint32_t)(cap1 / (kSegCap + 1));
    w.long_list = (uint32_t*)take(4 * std::max<int64_t>(w.max_long, 1));
    w.tkA = (uint32_t*)take(4 * cap1);
    w.tkB = (uint32_t*)take(4 * cap1);
    w.tvB = (uint32_t*)take(4 * cap1);
    w.rs_cnt = (uint32_t*)take(4 * kRadix * w.nb_cnt);
    w.rs_tot = (uint32_t*)take(4 * kRadix);
    w.bsum = (uint64_t*)take(8 * w.nb_scan);
    w.vsum = (uint32_t*)take(4 * w.nb_scan);
    w.bytes = off;
    return w;
}

}  // namespace

}  // namespace qg

using namespace qg;

// The workspace of qg_bin_noalloc.  Each device the library runs on holds its own copy for the life of the
// process; host code takes that copy's address from hipGetSymbolAddress and never uses the array's name, which
// in host code is only a stand-in for it.
static __device__ __align__(256) unsigned char scratch[QG_BIN_NOALLOC_SCRATCH_BYTES];

extern "C" size_t qg_bin_workspace_size(int64_t n, int32_t V, int64_t capacity, int64_t total_tiles) {
    (void)total_tiles;
    if (n < 0 || V < 1 || capacity < 0) return 0;
    return bin_ws_layout(nullptr, n, V, capacity).bytes;
}

namespace qg {
namespace {

// Argument checks shared by qg_bin and qg_bin_noalloc (nothing is enqueued on failure).
qg_status bin_check(int64_t n, const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                    int64_t capacity, const uint32_t* vals, const uint32_t* tile_ranges, const int64_t* num_pairs,
                    ViewTable* vt) {
    QG_REQUIRE(n >= 0 && n < (1ll << 31), "n=%lld outside [0, 2^31)", (long long)n);
    QG_REQUIRE(capacity >= 0 && capacity <= 0xFFFFFFFFll, "capacity=%lld outside [0, 2^32)", (long long)capacity);
    if (!make_view_table(cams, proj, V, tiling, true, vt)) return QG_ERR_ARG;
    QG_REQUIRE((int64_t)n * V < (1ll << 32), "n*V too large");
    QG_REQUIRE(tile_ranges && num_pairs, "tile_ranges and num_pairs are required");
    QG_REQUIRE(capacity == 0 || vals, "vals is NULL");
    return QG_OK;
}

// Per-tile depth order (k_seg_sort) when the average tile list the capacity allows is at most this long;
// above, the depth passes over the (view, Gaussian) items.  Both give the same lists.
constexpr int64_t kSegAvgMax = 512;

qg_status bin_run(int64_t n, const ViewTable& vt, int32_t V, int64_t capacity, uint32_t* vals, uint64_t* keys,
                  uint32_t* tile_ranges, int64_t* num_pairs, void* ws, hipStream_t s) {
    BinWs w = bin_ws_layout((char*)ws, n, V, capacity);
    const int64_t items = n * V;
    const int64_t T = vt.total_tiles;
    int tbits = 1;
    while ((1ll << tbits) < T) ++tbits;
    const int tpasses = (tbits + kRadixBits - 1) / kRadixBits;
    if (items == 0) {  // clear the ranges, num_pairs and the sort count; nothing else to do
        ZeroList z{};
        z.p[0] = tile_ranges;
        z.words[0] = 2 * T;
        z.p[1] = (uint32_t*)num_pairs;
        z.words[1] = 2;
        z.p[2] = w.sort_count;
        z.words[2] = 1;
        z.n = 3;
        {
            QG_TIMED("bin_init", s);
            k_bin_init<<<(unsigned)std::min<int64_t>(std::max<int64_t>(ceil_div(2 * T, 256), 1), 4096), 256, 0, s>>>(z);
        }
        QG_LAUNCH_CHECK("qg_bin init");
        return QG_OK;
    }
    // 1. depth order: the 4-pass depth sort over (view, Gaussian) items (the first pass makes the keys), or,
    //    with short tile lists, none here (k_seg_sort orders each tile's list at the end)
    const bool per_tile = capacity <= kSegAvgMax * T;
    const uint32_t* sorted_items = nullptr;
    if (!per_tile) {
        RsSrc src{};
        src.n = n;
        for (int v = 0; v < V; ++v) {
            src.depth[v] = vt.proj[v].depth;
            src.ntiles[v] = vt.proj[v].ntiles;
        }
        uint32_t *ka = w.dkA, *va = w.dvA, *kb = w.dkB, *vb = w.dvB;
        for (int pass = 0; pass < 4; ++pass) {
            qg_status st;
            if (pass == 0) {
                st = rs_pass<true>(src, ka, va, nullptr, (uint32_t)items, items, pass, w.rs_cnt, w.nb_cnt, w.rs_tot,
                                   s, "sort_depth");
            } else {
                src.keys = ka;
                src.vals = va;
                st = rs_pass<false>(src, kb, vb, nullptr, (uint32_t)items, items, pass, w.rs_cnt, w.nb_cnt,
                                    w.rs_tot, s, "sort_depth");
                std::swap(ka, kb);
                std::swap(va, vb);
            }
            if (st != QG_OK) return st;
        }
        sorted_items = va;  // w.dvB after 4 passes; the keys, in w.dkB, are dead: w.dkB takes the compacted items
    }
    // 2. tile counts in order: scan, compaction of the items with pairs, total, overflow check; the ranges are
    //    cleared on the way
    uint32_t* comp_item = w.dkB;
    {
        QG_TIMED("bin_count_scan", s);
        k_count_reduce<<<(unsigned)w.nb_scan, kBlock, 0, s>>>(items, n, vt, sorted_items, w.bsum, w.vsum,
                                                              tile_ranges, 2 * T);
        k_count_apply<<<(unsigned)w.nb_scan, kBlock, 0, s>>>(items, n, vt, sorted_items, w.bsum, w.vsum, comp_item,
                                                             w.offs, capacity, w.sort_count, w.n_comp,
                                                             w.long_count, num_pairs);
    }
    QG_LAUNCH_CHECK("qg_bin count");
    if (capacity == 0) return QG_OK;
    uint32_t* vbuf0 = (tpasses % 2 == 1) ? w.tvB : vals;
    uint32_t* vbuf1 = (tpasses % 2 == 1) ? vals : w.tvB;
    {
        QG_TIMED("bin_emit", s);
        // consecutive chunks per block once the grid would exceed 8192 blocks
        const int64_t chunks = std::max<int64_t>(1, ceil_div(capacity, kEmitPer));
        const int64_t per_block = std::max<int64_t>(1, chunks / 8192);
        k_emit<<<(unsigned)ceil_div(chunks, per_block), 256, 0, s>>>(w.n_comp, n, vt, comp_item, w.offs,
                                                                    w.sort_count, w.tkA, vbuf0, per_block);
    }
    QG_LAUNCH_CHECK("qg_bin emit");
    // 3. stable sort by tile id: reduce, scan and scatter per 8-bit pass
    uint32_t *tk_in = w.tkA, *tk_out = w.tkB, *tv_in = vbuf0, *tv_out = vbuf1;
    for (int pass = 0; pass < tpasses; ++pass) {
        RsSrc ts{};
        ts.keys = tk_in;
        ts.vals = tv_in;
        qg_status st = rs_pass<false>(ts, tk_out, tv_out, w.sort_count, 0u, capacity, pass, w.rs_cnt, w.nb_cnt,
                                      w.rs_tot, s, "sort_tile");
        if (st != QG_OK) return st;
        std::swap(tk_in, tk_out);
        std::swap(tv_in, tv_out);
    }
    // tk_in / tv_in hold the sorted pairs; tv_in == vals by construction, w.tvB is spare
    // 4. tile ranges, then (per-tile order) each tile's list by depth
    {
        QG_TIMED("bin_ranges", s);
        k_ranges<<<(unsigned)std::max<int64_t>(1, ceil_div(capacity, 256 * kRangesPerThread)), 256, 0, s>>>(
            tk_in, w.sort_count, tile_ranges);
    }
    QG_LAUNCH_CHECK("qg_bin ranges");
    if (per_tile) {
        {
            QG_TIMED("bin_seg_sort", s);
            k_seg_sort<<<(unsigned)T, kWave, 0, s>>>(vt, tile_ranges, vals, w.long_count, w.long_list,
                                                     w.max_long, T);
        }
        QG_LAUNCH_CHECK("qg_bin tile depth order");
        if (w.max_long > 0) {
            QG_TIMED("bin_seg_sort_long", s);
            k_seg_sort_long<<<std::min(w.max_long, 256u), kLongThreads, 0, s>>>(vt, tile_ranges, vals, w.tvB,
                                                                                w.long_count, w.long_list,
                                                                                w.max_long);
        }
        QG_LAUNCH_CHECK("qg_bin long tile lists");
    }
    if (keys) {
        k_keys64<<<(unsigned)ceil_div(capacity, 256), 256, 0, s>>>(tk_in, tv_in, w.sort_count, vt, keys);
        QG_LAUNCH_CHECK("qg_bin keys");
    }
    return QG_OK;
}

// ---- the scratch-free variant -----------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once per device.
qg_status scratch_for_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("qg_bin_noalloc: hipGetDevice failed: %s", hipGetErrorString(e));
        return QG_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("qg_bin_noalloc: device %d outside [0, %d)", dev, kMaxDevices);
        return QG_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("qg_bin_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            return QG_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QG_OK;
}

}  // namespace
}  // namespace qg

extern "C" size_t qg_bin_noalloc_max_bytes(void) { return QG_BIN_NOALLOC_SCRATCH_BYTES; }

extern "C" qg_status qg_bin(int64_t n, const qg_projected* proj, const qg_camera* cams, int32_t V, qg_tiling tiling,
                            int64_t capacity, uint32_t* vals, uint64_t* keys, uint32_t* tile_ranges,
                            int64_t* num_pairs, void* ws, size_t ws_bytes, qg_stream stream) {
    clear_error();
    ViewTable vt;
    qg_status st = bin_check(n, proj, cams, V, tiling, capacity, vals, tile_ranges, num_pairs, &vt);
    if (st != QG_OK) return st;
    const size_t need = bin_ws_layout(nullptr, n, V, capacity).bytes;
    QG_REQUIRE(ws && ws_bytes >= need, "workspace too small: %zu < %zu", ws_bytes, need);
    return bin_run(n, vt, V, capacity, vals, keys, tile_ranges, num_pairs, ws, (hipStream_t)stream);
}

extern "C" qg_status qg_bin_noalloc(int64_t n, const qg_projected* proj, const qg_camera* cams, int32_t V,
                                    qg_tiling tiling, int64_t capacity, uint32_t* vals, uint64_t* keys,
                                    uint32_t* tile_ranges, int64_t* num_pairs, qg_stream stream) {
    clear_error();
    ViewTable vt;
    qg_status st = bin_check(n, proj, cams, V, tiling, capacity, vals, tile_ranges, num_pairs, &vt);
    if (st != QG_OK) return st;
    const size_t need = bin_ws_layout(nullptr, n, V, capacity).bytes;
    QG_REQUIRE(need <= (size_t)QG_BIN_NOALLOC_SCRATCH_BYTES,
               "qg_bin_noalloc: n=%lld, V=%d, capacity=%lld need %zu bytes of scratch, above the %zu of the "
               "library's array (use qg_bin with a workspace)",
               (long long)n, V, (long long)capacity, need, (size_t)QG_BIN_NOALLOC_SCRATCH_BYTES);
    void* ptr = nullptr;
    st = scratch_for_current_device(&ptr);
    if (st != QG_OK) return st;
    return bin_run(n, vt, V, capacity, vals, keys, tile_ranges, num_pairs, ptr, (hipStream_t)stream);
}
