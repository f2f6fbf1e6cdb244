// Viewspace-gradient difference (Eq. 9) helpers and gate initialisation (Eq. 10).
//
// d_t is the view-average of dL/dp' under the image gradient 2 (I_{t-1} - I_t) / (3HW): both MSE gradients of
// Eq. 9 are taken at the same render, so their difference is one backward pass with that image gradient.
// The gate parameter then solves Eq. 8's p_i = sigmoid(a_i - tau ln(-gamma0/gamma1)) for
// p_i = |d_i| / (|d_i| + median_j |d_j|) (Eq. 10).  The median (lower median, element (n-1)/2 of the sorted
// norms) is found exactly by a most-significant-digit-first radix select on the float bits of the norms
// (non-negative floats order like their bit patterns): four 8-bit passes, each a histogram of the
// candidates that share the digits chosen so far, then a one-thread pick of the bucket holding the rank.
#include <cmath>

#include "qg_internal.h"

namespace qg {
namespace {

__global__ void k_scaled_diff(int64_t count, const float* __restrict__ a, const float* __restrict__ b, float scale,
                              float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = scale * (a[i] - b[i]);
}

__global__ void k_norms(int64_t n, const float* __restrict__ d, uint32_t* __restrict__ bits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = d[i], y = d[n + i];
    bits[i] = __float_as_uint(sqrtf(x * x + y * y));
}

// state[0] = prefix (digits chosen so far, in place), state[1] = rank still sought among the candidates.
__global__ __launch_bounds__(256) void k_select_hist(int64_t n, const uint32_t* __restrict__ bits,
                                                     const uint32_t* __restrict__ state, int shift,
                                                     uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t prefix = state[0];
    const uint32_t hi_mask = shift >= 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t b = bits[i];
        if ((b & hi_mask) == (prefix & hi_mask)) atomicAdd(&s_h[(b >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    if (s_h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], s_h[threadIdx.x]);
}

__global__ void k_select_pick(uint32_t* __restrict__ state, uint32_t* __restrict__ hist, int shift) {
    uint32_t rank = state[1];
    uint32_t d = 0;
    for (; d < 255; ++d) {
        if (rank < hist[d]) break;
        rank -= hist[d];
    }
    state[0] |= d << shift;
    state[1] = rank;
    for (int k = 0; k < 256; ++k) hist[k] = 0;
}

__global__ void k_gate_from_median(int64_t n, const uint32_t* __restrict__ bits, const uint32_t* __restrict__ state,
                                   float shift_a, float* __restrict__ a_out, float* __restrict__ p_out,
                                   float* __restrict__ median_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float med = __uint_as_float(state[0]);
    if (i == 0 && median_out) *median_out = med;
    if (i >= n) return;
    const float nrm = __uint_as_float(bits[i]);
    const float den = nrm + med;
    float p = den > 0.f ? nrm / den : 0.f;
    p = fminf(fmaxf(p, 1e-6f), 1.f - 1e-6f);
    if (p_out) p_out[i] = p;
    a_out[i] = logf(p) - log1pf(-p) + shift_a;
}

__global__ void k_init_state(uint32_t* state, uint32_t rank, uint32_t* hist) {
    state[0] = 0;
    state[1] = rank;
    for (int k = threadIdx.x; k < 256; k += blockDim.x) hist[k] = 0;
}

}  // namespace
}  // namespace qg

using namespace qg;

extern "C" qg_status qg_scaled_diff(int64_t count, const float* a, const float* b, float scale, float* out,
                                    qg_stream stream) {
    clear_error();
    QG_REQUIRE(count >= 0, "count < 0");
    if (count == 0) return QG_OK;
    QG_REQUIRE(a && b && out, "a pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    {
        QG_TIMED("scaled_diff", s);
        k_scaled_diff<<<(unsigned)ceil_div(count, 256), 256, 0, s>>>(count, a, b, scale, out);
    }
    QG_LAUNCH_CHECK("qg_scaled_diff");
    return QG_OK;
}

extern "C" size_t qg_gate_init_workspace_size(int64_t n) {
    if (n < 0) return 0;
    return align_up((size_t)(n > 0 ? n : 1) * 4) + align_up(2 * 4) + align_up(256 * 4);
}

extern "C" qg_status qg_gate_init(int64_t n, const float* d, float gamma0, float gamma1, float tau, float* a_out,
                                  float* p_out, float* median_out, void* ws, size_t ws_bytes, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && n < (1ll << 32), "n=%lld outside [0, 2^32)", (long long)n);
    QG_REQUIRE(gamma0 < 0.f && gamma1 > 1.f && tau > 0.f, "need gamma0 < 0, gamma1 > 1, tau > 0");
    if (n == 0) return QG_OK;
    QG_REQUIRE(d && a_out, "d and a_out are required");
    QG_REQUIRE(ws && ws_bytes >= qg_gate_init_workspace_size(n), "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    uint32_t* bits = (uint32_t*)ws;
    uint32_t* state = (uint32_t*)((char*)ws + align_up((size_t)n * 4));
    uint32_t* hist = (uint32_t*)((char*)state + align_up(2 * 4));
    const unsigned grid = (unsigned)ceil_div(n, 256);
    const unsigned hgrid = (unsigned)std::min<int64_t>(ceil_div(n, 256), 1024);
    {
        QG_TIMED("gate_init", s);
        k_norms<<<grid, 256, 0, s>>>(n, d, bits);
        k_init_state<<<1, 256, 0, s>>>(state, (uint32_t)((n - 1) / 2), hist);
        for (int shift = 24; shift >= 0; shift -= 8) {
            k_select_hist<<<hgrid, 256, 0, s>>>(n, bits, state, shift, hist);
            k_select_pick<<<1, 1, 0, s>>>(state, hist, shift);
        }
        const float shift_a = tau * logf(-gamma0 / gamma1);
        k_gate_from_median<<<grid, 256, 0, s>>>(n, bits, state, shift_a, a_out, p_out, median_out);
    }
    QG_LAUNCH_CHECK("qg_gate_init");
    return QG_OK;
}
