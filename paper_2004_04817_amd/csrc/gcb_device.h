// Device helpers shared by the HIP kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

namespace gcb {

// ---------------------------------------------------------------- Eq. (2)
// Wendland C2 from the squared scaled distance r2 = (|r - r_i| / R)^2:
// eta = sqrt(r2) by one Newton step on the hardware reciprocal square root
// and one on the square root itself; t = clamp(1 - eta, 0, 1);
// phi = (1 - eta)^4 (4 eta + 1) = t^4 (5 - 4 t).  Exactly 0 for eta >= 1.
__device__ __forceinline__ double wendland_r2(double r2) {
    const double x = fmax(r2, 1e-200);
    double r = __builtin_amdgcn_rsq(x);
    double y = x * r;
    const double e = fma(-y, r, 1.0);
    r = fma(0.5 * r, e, r);
    y = x * r;
    const double d = fma(-y, y, x);
    y = fma(0.5 * r, d, y);
    const double t = fmin(fmax(1.0 - y, 0.0), 1.0);
    const double t2 = t * t;
    return (t2 * t2) * fma(-4.0, t, 5.0);
}

// Wendland C2 for the volume sweep (Eq. 6) from d = (|r - r_i| / (2R))^2, the
// squared distance of points scaled by 1/(2R).  With h = rsq(d) ~ 2/eta and
// q = d h ~ eta/2, one Newton step for the square root gives
// eta = q (3 - q h) (relative error about 1.5 e^2 for a hardware estimate of
// relative error e; e is about 5e-8, so eta is good to 1e-14), and
// phi = t^4 (5 - 4 t) with t = clamp(1 - eta, 0, 1).  d may come out slightly
// negative from the cancellation in |u|^2 + |v|^2 - 2 u.v; |d| plus a tiny
// bias keeps the square root real and away from rsq(0).  Used where only the
// displacement tolerance matters, not in the greedy's sweeps.
__device__ __forceinline__ double wendland_quarter(double d) {
    const double x = fabs(d) + 1e-200;
    const double h = __builtin_amdgcn_rsq(x);
    const double q = x * h;
    const double e = fma(-q, h, 3.0);
    const double t = fmin(fmax(fma(-q, e, 1.0), 0.0), 1.0);
    const double t2 = t * t;
    return (t2 * t2) * fma(-4.0, t, 5.0);
}

__device__ __forceinline__ double dist2(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

// Squared norm summed as (x^2 + y^2) + z^2 with no fused multiply-add, for
// the integer decisions of the starting-node rule.
__device__ __forceinline__ double sq3_exact(double x, double y, double z) {
#pragma clang fp contract(off)
    const double s = x * x + y * y;
    return s + z * z;
}

}  // namespace gcb
