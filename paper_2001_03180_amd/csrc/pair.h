// The FP64 pair term shared by every force loop: 1/sqrt refined to full
// precision, then m_j/r and m_j/r^3.  Kept apart from common.h so that the
// force kernel's measured HBM traffic can be tied to the sources that shape
// its code (kernels_force.hip and this file).
#pragma once
#include <hip/hip_runtime.h>

namespace mstar {

// 1/sqrt(x) for x > 0 to <= 1 ulp: the hardware estimate v_rsq_f64 (relative
// error ~5e-8) refined by the second-order expansion of (1 - e)^(-1/2) =
// 1 + e/2 + 3e^2/8 + O(e^3) with e = 1 - x y0^2 (Newton's method on
// f(y) = y^-2 - x carried one term further).
__device__ __forceinline__ double rsqrt_f64(double x) {
    double y0 = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y0, y0, 1.0);
    double c = fma(e, 0.375, 0.5);
    return fma(y0 * e, c, y0);
}

// The O(N^2) pair term: mr = m_j/r, s = m_j/r^3; accumulate phi and a.
__device__ __forceinline__ void pair_terms(double dx, double dy, double dz, double mj,
                                           double &s, double &mr) {
    double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    double y = rsqrt_f64(r2);
    mr = mj * y;
    s = mr * (y * y);
}

}  // namespace mstar
