// Device-side output transforms shared by the Philox and MRG32k3a kernels
// (library-internal).  Conventions: uniform FP32 = (w >> 8) 2^-24; uniform
// FP64 from two Philox words = 53 bits * 2^-53; Box-Muller on a word pair.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mirng {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// (w >> 8) * 2^-24, exact.
__device__ __forceinline__ float u01f(uint32_t w)
{
    return (float)(w >> 8) * 0x1p-24f;
}

// 53 bits of (hi:lo) * 2^-53, exact: hi 2^-32 + (lo >> 11) 2^-53.
__device__ __forceinline__ double u01d(uint32_t lo, uint32_t hi)
{
    return __builtin_fma((double)hi, 0x1p-32, (double)(lo >> 11) * 0x1p-53);
}

// 1/d for d in [1.7, 2.5]: the hardware estimate refined by two Newton
// steps (each squares the relative error; the result is within a few ulp).
__device__ __forceinline__ double recip_fast(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// sqrt(x) for x in [0, 34] as x * (1 / sqrt(x)): the hardware reciprocal square
// root of max(x, 2^-100) refined by two Newton steps, so x = 0 gives 0.
__device__ __forceinline__ double sqrt_fast(double x)
{
    const double xs = __builtin_fmax(x, 0x1p-100);
    const double h = 0.5 * xs;
    double y = __builtin_amdgcn_rsq(xs);
    double e = __builtin_fma(-h * y, y, 0.5);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-h * y, y, 0.5);
    y = __builtin_fma(y, e, y);
    return x * y;
}

// Box-Muller on one word pair.  The radius and the rotation are evaluated
// in FP64 to about 2^-34 relative error and rounded once to FP32, so each
// output is within 0.51 ulp of the exact transform of the same two inputs.
// The one division and the square root use refined hardware estimates
// (recip_fast, sqrt_fast) instead of the IEEE sequences, whose exactness
// this accuracy does not need.
//   ln u1: u1 = 2^e m, m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) with
//          s = (m - 1)/(m + 1), |s| <= 0.1716, series to s^11.
//   sin/cos(2 pi u2): 2 u2 = k 2^-23; j = nearest quarter turn; the exact
//          remainder t = (k - j 2^22) 2^-23 in [-1/4, 1/4]; Taylor series of
//          sin(pi t) to t^13 and cos(pi t) to t^14; rotate by j quarters.
__device__ __forceinline__ f32x2 box_muller(uint32_t wa, uint32_t wb)
{
    const double u1 = (double)((wa >> 8) + 1u) * 0x1p-24;
    int e;
    double m = __builtin_frexp(u1, &e);            // [0.5, 1)
    const bool low = m < 0x1.6a09e667f3bcdp-1;     // sqrt(1/2)
    m = low ? m * 2.0 : m;
    e = low ? e - 1 : e;
    const double f = m - 1.0;
    const double s = f * recip_fast(m + 1.0);
    const double s2 = s * s;
    double q = 0x1.745d1745d1746p-4;               // 1/11
    q = __builtin_fma(q, s2, 0x1.c71c71c71c71cp-4); // 1/9
    q = __builtin_fma(q, s2, 0x1.2492492492492p-3); // 1/7
    q = __builtin_fma(q, s2, 0x1.999999999999ap-3); // 1/5
    q = __builtin_fma(q, s2, 0x1.5555555555555p-2); // 1/3
    q = __builtin_fma(q, s2, 1.0);
    const double ln_m = 2.0 * s * q;
    const double ln_u1 = __builtin_fma((double)e, 0x1.62e42fefa39efp-1, ln_m);
    const double r = sqrt_fast(-2.0 * ln_u1);

    const uint32_t k = wb >> 8;
    const uint32_t j = (k + (1u << 21)) >> 22;     // 0..4
    const int32_t ti = (int32_t)k - (int32_t)(j << 22);
    const double t = (double)ti * 0x1p-23;
    const double t2 = t * t;
    double sp = -0x1.e3074fde8871fp-8;
    sp = __builtin_fma(sp, t2, 0x1.50783487ee782p-4);
    sp = __builtin_fma(sp, t2, -0x1.32d2cce62bd86p-1);
    sp = __builtin_fma(sp, t2, 0x1.466bc6775aae2p+1);
    sp = __builtin_fma(sp, t2, -0x1.4abbce625be53p+2);
    sp = __builtin_fma(sp, t2, 0x1.921fb54442d18p+1);
    sp = sp * t;                                   // sin(pi t)
    double cp = 0x1.f9d38a3763cc3p-10;
    cp = __builtin_fma(cp, t2, -0x1.a6d1f2a204a8cp-6);
    cp = __builtin_fma(cp, t2, 0x1.e1f506891babbp-3);
    cp = __builtin_fma(cp, t2, -0x1.55d3c7e3cbffap+0);
    cp = __builtin_fma(cp, t2, 0x1.03c1f081b5ac4p+2);
    cp = __builtin_fma(cp, t2, -0x1.3bd3cc9be45dep+2);
    cp = __builtin_fma(cp, t2, 1.0);               // cos(pi t)
    const float rs = (float)(r * sp);
    const float rc = (float)(r * cp);
    const uint32_t quad = j & 3u;
    // quad 0: (cos, sin) = ( C,  S); 1: (-S,  C); 2: (-C, -S); 3: ( S, -C)
    const float c_abs = (quad & 1u) ? rs : rc;
    const float s_abs = (quad & 1u) ? rc : rs;
    f32x2 z;
    z.x = (quad == 1u || quad == 2u) ? -c_abs : c_abs;
    z.y = (quad >= 2u) ? -s_abs : s_abs;
    return z;
}

// Box-Muller in FP64 on a pair of FP64 uniforms u1 in (0, 1], u2 in [0, 1):
// r = sqrt(-2 ln u1), (z0, z1) = r (cos 2 pi u2, sin 2 pi u2), with the
// device library's log, IEEE sqrt and sincospi (whose argument reduction is
// exact, as 2 u2 is).  u1 = 1 gives +-0.
__device__ __forceinline__ f64x2 box_muller64(double u1, double u2)
{
    const double r = __builtin_sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    f64x2 z;
    z.x = r * c;
    z.y = r * s;
    return z;
}

}  // namespace mirng
