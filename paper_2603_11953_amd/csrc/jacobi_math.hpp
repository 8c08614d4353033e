// Scalar helpers of the Jacobi rotations: reciprocal and reciprocal square
// root from the hardware estimates refined by Newton steps (a shorter
// dependent chain than the correctly rounded division and square root; the
// rotation parameters only need to be accurate to a few ulps).
#pragma once

#include <hip/hip_runtime.h>

namespace gsvd {

__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double h = x * y;
        const double e = __builtin_fma(-h, y, 1.0);  // 1 - x y^2
        y = __builtin_fma(0.5 * y, e, y);
    }
    return y;
}

}  // namespace gsvd
