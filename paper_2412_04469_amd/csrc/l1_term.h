// The per-element term of the L1 loss of Eq. 3, shared by the loss kernel and the blend forward's fused
// epilogue, so that both write the same gradient bits.  Internal to libqg.
#pragma once

#include "qg_internal.h"

namespace qg {

// d = x - y: adds |d| to sa and (clamp(x, 0, 1) - y)^2 to sb (the clamped image's squared error, for PSNR);
// returns the gradient gscale * sign(d) (sign(0) = 0).
__device__ __forceinline__ float l1_term(float x, float y, float gscale, float& sa, float& sb) {
    const float d = x - y;
    sa += fabsf(d);
    const float c = fminf(1.f, fmaxf(0.f, x)) - y;
    sb = __builtin_fmaf(c, c, sb);
    return d > 0.f ? gscale : (d < 0.f ? -gscale : 0.f);
}

}  // namespace qg
