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

// Rotation of a one-sided Jacobi step on columns x, y with al = x^T x,
// be = y^T y, ga = x^T y (ga != 0): x' = c x - s y, y' = s x + c y makes x'
// and y' orthogonal when tan 2t = 2 ga / (be - al), taken with |t| <= pi/4.
// With r = sqrt((be - al)^2 + 4 ga^2), cos 2t = |be - al| / r, so
// c^2 = (1 + |be - al| / r) / 2 and s = sin 2t / (2 c) = sign(be - al) ga / (r c).
// be - al and 2 ga are first scaled by a common power of two (exact) so that
// the larger has magnitude in [1/2, 1): r^2 then neither overflows nor
// underflows.  Two reciprocal square roots form everything.
__device__ __forceinline__ void jacobi_cs(double al, double be, double ga, double &c, double &s) {
    const double d = be - al, g2 = ga + ga;
    const int ex = __builtin_amdgcn_frexp_exp(__builtin_fmax(__builtin_fabs(d), __builtin_fabs(g2)));
    const double dn = __builtin_ldexp(d, -ex), gn = __builtin_ldexp(g2, -ex);
    const double y = rsq_nr(__builtin_fma(dn, dn, gn * gn));      // 1 / r (scaled)
    const double c2 = __builtin_fma(0.5 * __builtin_fabs(dn), y, 0.5);  // cos^2 t, in [1/2, 1]
    const double z = rsq_nr(c2);                                    // 1 / cos t
    c = c2 * z;
    const double sv = (0.5 * gn * y) * z;
    s = d < 0.0 ? -sv : sv;
}

}  // namespace gsvd
