// Compression back end of a frame's residuals: the quantised latents (Sec. 3.2: the decoder reads
// rint(l_hat)) as int8 symbols with one symbol histogram per latent dimension (GPU), and a byte-wise rANS
// coder over them (host C++), one static model per dimension built from the frame's histogram.
//
// rANS (asymmetric numeral systems, range variant, Duda 2013): state x in [2^23, 2^31), probabilities
// quantised to f_s / 2^16.  Encoding runs over the symbols backwards: while x >= 2^15 f_s emit its low byte,
// then x <- (x / f_s) 2^16 + (x mod f_s) + c_s.  Decoding runs forwards: slot = x mod 2^16 gives s by
// c_s <= slot < c_s + f_s, then x <- f_s (x >> 16) + slot - c_s, refilled byte by byte while x < 2^23.
#include <cstring>
#include <vector>

#include "qg_internal.h"

namespace qg {
namespace {

constexpr int kBins = 256;       // symbols -128 .. 127
constexpr int kProbBits = 16;
constexpr uint32_t kProbScale = 1u << kProbBits;
constexpr uint32_t kRansL = 1u << 23;

// Symbols and per-dimension histograms: one thread per Gaussian, LDS histograms per block.
__global__ __launch_bounds__(256) void k_latent_symbols(int64_t n, int64_t ld, const float* __restrict__ lat,
                                                        int L, int8_t* __restrict__ sym,
                                                        uint32_t* __restrict__ hist,
                                                        uint32_t* __restrict__ overflow) {
    __shared__ uint32_t s_h[16][kBins];
    for (int i = threadIdx.x; i < L * kBins; i += blockDim.x) s_h[i / kBins][i % kBins] = 0u;
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) {
        for (int k = 0; k < L; ++k) {
            const float v = rintf(lat[(int64_t)k * ld + g]);
            const bool in = v >= -128.f && v <= 127.f;
            const int s = in ? (int)v : 0;
            sym[g * L + k] = (int8_t)s;
            if (in)
                atomicAdd(&s_h[k][s + 128], 1u);
            else
                atomicAdd(overflow, 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L * kBins; i += blockDim.x) {
        const uint32_t c = s_h[i / kBins][i % kBins];
        if (c) atomicAdd(&hist[i], c);
    }
}

// Quantised frequencies of one model: every symbol with a non-zero count gets at least 1 of 2^16, the
// rest in proportion (floor), and the remainder goes to (or comes from) the most frequent symbols in order.
// Deterministic in the counts alone, so the encoder and the decoder build the same table.
bool normalise(const uint32_t* counts, uint32_t* freq, uint32_t* cum) {
    uint64_t total = 0;
    for (int s = 0; s < kBins; ++s) total += counts[s];
    if (total == 0) {
        for (int s = 0; s < kBins; ++s) freq[s] = cum[s] = 0;
        cum[kBins] = 0;
        return true;
    }
    int64_t sum = 0;
    for (int s = 0; s < kBins; ++s) {
        uint32_t f = 0;
        if (counts[s]) {
            f = (uint32_t)((uint64_t)counts[s] * kProbScale / total);
            if (f == 0) f = 1;
        }
        freq[s] = f;
        sum += f;
    }
    // symbols by count, largest first (ties: lower symbol first)
    int order[kBins];
    for (int s = 0; s < kBins; ++s) order[s] = s;
    for (int a = 1; a < kBins; ++a) {
        const int v = order[a];
        int b = a - 1;
        while (b >= 0 && (counts[order[b]] < counts[v] || (counts[order[b]] == counts[v] && order[b] > v))) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = v;
    }
    int64_t diff = (int64_t)kProbScale - sum;
    for (int pass = 0; diff != 0 && pass < 1 << 20; ++pass) {
        for (int k = 0; k < kBins && diff != 0; ++k) {
            const int s = order[k];
            if (!counts[s]) break;
            if (diff > 0) {
                ++freq[s];
                --diff;
            } else if (freq[s] > 1) {
                --freq[s];
                ++diff;
            }
        }
    }
    if (diff != 0) return false;
    uint32_t c = 0;
    for (int s = 0; s < kBins; ++s) {
        cum[s] = c;
        c += freq[s];
    }
    cum[kBins] = c;
    return c == kProbScale;
}

}  // namespace
}  // namespace qg

using namespace qg;

extern "C" qg_status qg_latent_symbols(int64_t n, int64_t ld, const float* latents, int32_t L, int8_t* symbols,
                                       uint32_t* hist, uint32_t* overflow, qg_stream stream) {
    clear_error();
    QG_REQUIRE(n >= 0 && ld >= n, "n=%lld ld=%lld invalid", (long long)n, (long long)ld);
    QG_REQUIRE(L >= 1 && L <= 16, "L=%d outside [1, 16]", L);
    QG_REQUIRE(n == 0 || (latents && symbols && hist && overflow), "a pointer is NULL");
    if (n == 0) return QG_OK;
    hipStream_t s = (hipStream_t)stream;
    qg_status st = qg_zero(hist, (int64_t)L * kBins * 4, stream);
    if (st != QG_OK) return st;
    st = qg_zero(overflow, 4, stream);
    if (st != QG_OK) return st;
    k_latent_symbols<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, ld, latents, L, symbols, hist, overflow);
    QG_LAUNCH_CHECK("qg_latent_symbols");
    return QG_OK;
}

extern "C" size_t qg_rans_bound(int64_t count) {
    if (count < 0) return 0;
    return (size_t)count * 3 + 64;  // at most 16 bits (2 bytes) per symbol plus the final state
}

extern "C" qg_status qg_rans_encode(int64_t count, int32_t L, const int8_t* symbols, const uint32_t* hist,
                                    uint8_t* out, size_t capacity, size_t* out_bytes) {
    clear_error();
    QG_REQUIRE(count >= 0 && L >= 1 && L <= 16 && count % L == 0, "count=%lld L=%d invalid", (long long)count, L);
    QG_REQUIRE(out && out_bytes && (count == 0 || (symbols && hist)), "a pointer is NULL");
    std::vector<uint32_t> freq((size_t)L * kBins), cum((size_t)L * (kBins + 1));
    for (int k = 0; k < L; ++k)
        QG_REQUIRE(normalise(hist + (size_t)k * kBins, &freq[(size_t)k * kBins], &cum[(size_t)k * (kBins + 1)]),
                   "model %d: frequencies do not normalise", k);
    std::vector<uint8_t> rev;
    rev.reserve((size_t)count + 8);
    uint32_t x = kRansL;
    for (int64_t i = count - 1; i >= 0; --i) {
        const int k = (int)(i % L);
        const int s = (int)symbols[i] + 128;
        const uint32_t f = freq[(size_t)k * kBins + s], c = cum[(size_t)k * (kBins + 1) + s];
        QG_REQUIRE(f > 0, "symbol %d of model %d has no count in the histogram", s - 128, k);
        const uint32_t xmax = ((kRansL >> kProbBits) << 8) * f;
        while (x >= xmax) {
            rev.push_back((uint8_t)(x & 0xffu));
            x >>= 8;
        }
        x = ((x / f) << kProbBits) + (x % f) + c;
    }
    for (int b = 0; b < 4; ++b) {
        rev.push_back((uint8_t)(x & 0xffu));
        x >>= 8;
    }
    QG_REQUIRE(rev.size() <= capacity, "output capacity %zu < %zu bytes", capacity, rev.size());
    for (size_t j = 0; j < rev.size(); ++j) out[j] = rev[rev.size() - 1 - j];
    *out_bytes = rev.size();
    return QG_OK;
}

extern "C" qg_status qg_rans_decode(int64_t count, int32_t L, const uint8_t* in, size_t in_bytes,
                                    const uint32_t* hist, int8_t* symbols) {
    clear_error();
    QG_REQUIRE(count >= 0 && L >= 1 && L <= 16 && count % L == 0, "count=%lld L=%d invalid", (long long)count, L);
    QG_REQUIRE(in && in_bytes >= 4 && (count == 0 || (symbols && hist)), "bad input");
    std::vector<uint32_t> freq((size_t)L * kBins), cum((size_t)L * (kBins + 1));
    std::vector<uint8_t> slot_sym((size_t)L * kProbScale);
    for (int k = 0; k < L; ++k) {
        uint32_t* f = &freq[(size_t)k * kBins];
        uint32_t* c = &cum[(size_t)k * (kBins + 1)];
        QG_REQUIRE(normalise(hist + (size_t)k * kBins, f, c), "model %d: frequencies do not normalise", k);
        for (int s = 0; s < kBins; ++s)
            for (uint32_t j = c[s]; j < c[s] + f[s]; ++j) slot_sym[(size_t)k * kProbScale + j] = (uint8_t)s;
    }
    size_t pos = 0;
    uint32_t x = 0;
    for (int b = 0; b < 4; ++b) x = (x << 8) | in[pos++];
    for (int64_t i = 0; i < count; ++i) {
        const int k = (int)(i % L);
        const uint32_t slot = x & (kProbScale - 1);
        const int s = slot_sym[(size_t)k * kProbScale + slot];
        symbols[i] = (int8_t)(s - 128);
        x = freq[(size_t)k * kBins + s] * (x >> kProbBits) + slot - cum[(size_t)k * (kBins + 1) + s];
        while (x < kRansL) {
            QG_REQUIRE(pos < in_bytes, "stream ends early at symbol %lld", (long long)i);
            x = (x << 8) | in[pos++];
        }
    }
    QG_REQUIRE(pos == in_bytes && x == kRansL, "stream not consumed exactly (corrupt input)");
    return QG_OK;
}
