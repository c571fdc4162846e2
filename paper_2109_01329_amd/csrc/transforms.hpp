// Device-side output transforms shared by the Philox and MRG32k3a kernels
// (library-internal).  Conventions: uniform FP32 = (w >> 8) 2^-24; uniform
// FP64 from two Philox words = 53 bits * 2^-53; Box-Muller on a word pair;
// uniform int32 by an exact multiply-high; inverse-CDF Gaussians on
// uniforms strictly inside (0, 1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bm_tables.hpp"

namespace mirng {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Output stores go through global (address space 1) pointers.  Where an
// output pointer reaches a kernel through a descriptor in memory, the
// compiler cannot tell its address space and emits flat stores, which also
// count against the scalar-load counter (so each descriptor load waits for
// the stores in flight).  Every output is device-visible global memory
// (device, pinned host or managed), never LDS or scratch.
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) uint64_t g_u64;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;

// Adding 1.5 * 2^52 to a double of magnitude below 2^51 rounds it to an
// integer (to nearest, ties to even); subtracting it again gives that
// integer, with two full-rate adds instead of a rounding instruction.
constexpr double kRound2 = 0x1.8p52;

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

// 1/d for positive normal d: the hardware estimate refined by one Newton
// step, which squares its relative error.  The gfx950 estimate (v_rcp_f64)
// measured within 4.6e-8 (2^-24.4) relative over 2^22 arguments spanning
// 2^-40 .. 2^40, and within 2.2e-15 (2^-48.7) after the step.
__device__ __forceinline__ double recip_fast(double d)
{
    const double r = __builtin_amdgcn_rcp(d);
    const double e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// sqrt(x) for x in [0, 34] as x * (1 / sqrt(x)): the hardware reciprocal
// square root of max(x, 2^-100) refined by one Newton step, so x = 0 gives
// 0.  The gfx950 estimate (v_rsq_f64) measured within 5.2e-8 (2^-24.2)
// relative over the same arguments, and within 4.1e-15 (2^-47.8) after the
// step.
__device__ __forceinline__ double sqrt_fast(double x)
{
    const double xs = __builtin_fmax(x, 0x1p-100);
    const double h = 0.5 * xs;
    double y = __builtin_amdgcn_rsq(xs);
    const double e = __builtin_fma(-h * y, y, 0.5);
    y = __builtin_fma(y, e, y);
    return x * y;
}

// ln x for positive normal x in (0, 1], to about 2^-29 relative error (the
// budget of FP32 outputs): x = 2^e m with m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 0.1716, series to s^9
// (the omitted terms stay below s^10 / 11 * 1.03 <= 2.1e-9 relative), plus
// e ln 2 (for e != 0, |ln x| >= ln 2 - |ln m|, so nothing cancels).
__device__ __forceinline__ double ln_fast(double x)
{
    int e;
    double m = __builtin_frexp(x, &e);             // [0.5, 1)
    const bool low = m < 0x1.6a09e667f3bcdp-1;     // sqrt(1/2)
    m = low ? m * 2.0 : m;
    e = low ? e - 1 : e;
    const double f = m - 1.0;
    const double s = f * recip_fast(m + 1.0);
    const double s2 = s * s;
    double q = 0x1.c71c71c71c71cp-4;               // 1/9
    q = __builtin_fma(q, s2, 0x1.2492492492492p-3); // 1/7
    q = __builtin_fma(q, s2, 0x1.999999999999ap-3); // 1/5
    q = __builtin_fma(q, s2, 0x1.5555555555555p-2); // 1/3
    q = __builtin_fma(q, s2, 1.0);
    const double ln_m = 2.0 * s * q;
    return __builtin_fma((double)e, 0x1.62e42fefa39efp-1, ln_m);
}

// LDS copies of the two Box-Muller tables (6 KiB per workgroup).  Every
// kernel that evaluates box_muller() (or its factors) calls bm_stage() at
// its start, before any of its threads returns; kernels that do not are
// given no LDS for them.  Per-lane lookups into LDS cost one ds_read_b128
// each; from constant memory the same lookups went through the vector
// memory path, where a wave's 64 scattered addresses take many cycles.
static __shared__ __attribute__((aligned(16))) double s_bm_log[129][2];
static __shared__ __attribute__((aligned(16))) double s_bm_rot[256][2];

__device__ __forceinline__ void bm_stage()
{
    for (uint32_t i = threadIdx.x; i < 129u * 2u; i += blockDim.x)
        (&s_bm_log[0][0])[i] = (&kBmLogTab[0][0])[i];
    for (uint32_t i = threadIdx.x; i < 256u * 2u; i += blockDim.x)
        (&s_bm_rot[0][0])[i] = (&kBmRotTab[0][0])[i];
    __syncthreads();
}

// Box-Muller radius r = sqrt(-2 ln u1) for FP32 outputs, u1 = v 2^-24 with
// v = (wa >> 8) + 1 in [1, 2^24], to about 2^-29 relative error:
//   v = 2^(31 - nz) m, m in [1, 2), so u1 = 2^e m with e = 7 - nz;
//   j = m's nearest multiple of 1/128 (table entry j = 0..128, |f| <= 2^-8
//   below), f = m invc_j - 1 with invc_j ~ 1 / (1 + j/128), and
//   ln u1 = e ln 2 + ln(1 / invc_j) + ln(1 + f), ln(1 + f) = f - f^2/2 + f^3/3
//   (the rest is below f^4/4, 2^-26 relative);
//   L = -2 ln u1 sums the exponent and table terms first: for u1 just below 1
//   (e = -1, j = 128) and for u1 = 1 (e = 0, j = 0) they cancel exactly, so
//   L keeps the relative accuracy of its series term;
//   r = sqrt(L) from the hardware reciprocal square root y (within 2^-24 on
//   gfx950) corrected once, r = L y + (y / 2)(L - (L y)^2); L = 0 gives 0.
__device__ __forceinline__ double bm_radius(uint32_t wa)
{
    const uint32_t v = (wa >> 8) + 1u;
    const uint32_t nz = (uint32_t)__builtin_clz(v);
    const uint32_t mi = v << nz;                               // m 2^31
    const uint32_t j = (((mi >> 23) & 255u) + 1u) >> 1;
    const double f = __builtin_fma((double)mi, s_bm_log[j][0], -1.0);
    const double f2 = f * f;
    const double q = __builtin_fma(f, 0x1.5555555555555p-2, -0.5);
    const double s = __builtin_fma(f2, q, f);                  // ln(1 + f)
    const double base = __builtin_fma((double)(7 - (int32_t)nz), -0x1.62e42fefa39efp+0,
                                      s_bm_log[j][1]);
    const double L = __builtin_fma(s, -2.0, base);
    const double y = __builtin_amdgcn_rsq(__builtin_fmax(L, 0x1p-100));
    const double r0 = L * y;
    return __builtin_fma(0.5 * y, __builtin_fma(-r0, r0, L), r0);
}

// (cos, sin) of 2 pi u2 for FP32 outputs, u2 = k 2^-24 with k = wb >> 8, to
// about 2^-29 relative error: j = k's nearest multiple of 2^16 (table entry
// j mod 256, the angle 2 pi j / 256), x = 2 pi (k - 2^16 j) 2^-24 exactly
// reduced (|x| <= pi / 256), sin x = x - x^3/6 (the rest below x^5/120) and
// cos x = 1 - x^2/2 (the rest below x^4/24 = 2^-30), then the rotation
// cos = C cos x - S sin x, sin = S cos x + C sin x by the entry's (S, C).
// The table is exact at quarter turns, so the exact zeros of cos and sin
// come out as zeros, and values next to them keep the series' relative
// accuracy (the entries there have |S| or |C| = sin(2 pi / 256), at most
// twice the result).
__device__ __forceinline__ f64x2 bm_unit(uint32_t wb)
{
    // j mod 256 = the top 8 bits of k + 2^15, and k - 2^16 j is k's low 16
    // bits read as a signed integer
    const uint32_t jr = (wb + 0x800000u) >> 24;
    const int32_t rem = (int32_t)(int16_t)(uint16_t)(wb >> 8);
    const double S = s_bm_rot[jr][0];
    const double C = s_bm_rot[jr][1];
    const double x = (double)rem * 0x1.921fb54442d18p-22;      // 2 pi 2^-24
    const double x2 = x * x;
    const double sx = __builtin_fma(x * x2, -0x1.5555555555555p-3, x);
    const double cx = __builtin_fma(x2, -0.5, 1.0);
    f64x2 cs;
    cs.x = __builtin_fma(C, cx, -(S * sx));
    cs.y = __builtin_fma(S, cx, C * sx);
    return cs;
}

// Box-Muller on one word pair, FP32 outputs: z0 = RN32(r cos), z1 = RN32(r
// sin) from the two FP64 factors above, each within about 2^-29, so every
// output is within 0.55 ulp of the exact transform of the same two inputs.
__device__ __forceinline__ f32x2 box_muller(uint32_t wa, uint32_t wb)
{
    const double r = bm_radius(wa);
    const f64x2 cs = bm_unit(wb);
    f32x2 z;
    z.x = (float)(r * cs.x);
    z.y = (float)(r * cs.y);
    return z;
}

// ln x for x in (0, 1] in FP64, to a few ulp: x = 2^e m with m in
// [sqrt(1/2), sqrt(2)), f = m - 1 (exact), s = f / (m + 1) from the refined
// reciprocal and one Newton step on the quotient, ln m = 2 atanh(s) =
// 2 s + s^3 (2/3 + 2/5 s^2 + ... + 2/21 s^18) (|s| <= 0.1716: the omitted
// terms stay below 2.4e-17 relative), plus e ln 2 with ln 2 split so that
// e ln2_hi is exact (ln2_hi has 42 significant bits, |e| < 2^11).
__device__ __forceinline__ double ln_f64(double x)
{
    int e;
    double m = __builtin_frexp(x, &e);             // [0.5, 1)
    const bool low = m < 0x1.6a09e667f3bcdp-1;     // sqrt(1/2)
    m = low ? m * 2.0 : m;
    e = low ? e - 1 : e;
    const double f = m - 1.0;
    const double d = m + 1.0;
    const double r = recip_fast(d);
    double s = f * r;
    s = __builtin_fma(r, __builtin_fma(-s, d, f), s);
    const double s2 = s * s;
    double q = 0x1.8618618618618p-4;                 // 2/21
    q = __builtin_fma(q, s2, 0x1.af286bca1af28p-4);  // 2/19
    q = __builtin_fma(q, s2, 0x1.e1e1e1e1e1e1ep-4);  // 2/17
    q = __builtin_fma(q, s2, 0x1.1111111111111p-3);  // 2/15
    q = __builtin_fma(q, s2, 0x1.3b13b13b13b14p-3);  // 2/13
    q = __builtin_fma(q, s2, 0x1.745d1745d1746p-3);  // 2/11
    q = __builtin_fma(q, s2, 0x1.c71c71c71c71cp-3);  // 2/9
    q = __builtin_fma(q, s2, 0x1.2492492492492p-2);  // 2/7
    q = __builtin_fma(q, s2, 0x1.999999999999ap-2);  // 2/5
    q = __builtin_fma(q, s2, 0x1.5555555555555p-1);  // 2/3
    const double ln_m = __builtin_fma(s * s2, q, 2.0 * s);
    const double de = (double)e;
    return __builtin_fma(de, 0x1.62e42fefa3800p-1,
                         __builtin_fma(de, 0x1.ef35793c76730p-45, ln_m));
}

// a / b in FP64 for positive normal b, to about one ulp: the refined
// reciprocal, then one Newton step on the quotient.
__device__ __forceinline__ double div_f64(double a, double b)
{
    const double r = recip_fast(b);
    const double q = a * r;
    return __builtin_fma(r, __builtin_fma(-q, b, a), q);
}

// sqrt(x) for x in [0, 80] in FP64, to about one ulp: the refined
// reciprocal square root y of max(x, 2^-200), then r = x y corrected once,
// r + (y / 2)(x - r^2); x = 0 gives 0.
__device__ __forceinline__ double sqrt_f64(double x)
{
    const double xs = __builtin_fmax(x, 0x1p-200);
    const double h = 0.5 * xs;
    double y = __builtin_amdgcn_rsq(xs);
    y = __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
    const double r = x * y;
    return __builtin_fma(0.5 * y, __builtin_fma(-r, r, x), r);
}

// Box-Muller in FP64 on a pair of FP64 uniforms u1 in (0, 1], u2 in [0, 1):
// r = sqrt(-2 ln u1), (z0, z1) = r (cos 2 pi u2, sin 2 pi u2), each within a
// few ulp.  The angle 2 pi u2 = pi x, x = 2 u2 in [0, 2], is reduced
// exactly: j = nearest quarter turn (x rounded to a multiple of 1/2) and
// t = x - j/2 in [-1/4, 1/4] (exact, by Sterbenz's lemma); sin(pi t) by
// its Taylor series through t^15 (the rest below 5.9e-17 relative) and
// cos(pi t) through t^16 (below 2.1e-18); then a rotation by j quarter
// turns.  u1 = 1 gives +-0.
__device__ __forceinline__ f64x2 box_muller64(double u1, double u2)
{
    const double r = sqrt_f64(-2.0 * ln_f64(u1));
    const double x = 2.0 * u2;
    const double jd = __builtin_fma(x, 2.0, kRound2) - kRound2;   // 0..4
    const double t = __builtin_fma(jd, -0.5, x);
    const double t2 = t * t;
    double sp = -0x1.6fadb9f155744p-16;
    sp = __builtin_fma(sp, t2, 0x1.e8f434d018d63p-12);
    sp = __builtin_fma(sp, t2, -0x1.e3074fde8871fp-8);
    sp = __builtin_fma(sp, t2, 0x1.50783487ee782p-4);
    sp = __builtin_fma(sp, t2, -0x1.32d2cce62bd86p-1);
    sp = __builtin_fma(sp, t2, 0x1.466bc6775aae2p+1);
    sp = __builtin_fma(sp, t2, -0x1.4abbce625be53p+2);
    sp = __builtin_fma(sp, t2, 0x1.921fb54442d18p+1);
    sp = sp * t;                                   // sin(pi t)
    double cp = 0x1.20c62c2f2d7f5p-18;
    cp = __builtin_fma(cp, t2, -0x1.b6e24f44b128fp-14);
    cp = __builtin_fma(cp, t2, 0x1.f9d38a3763cc3p-10);
    cp = __builtin_fma(cp, t2, -0x1.a6d1f2a204a8cp-6);
    cp = __builtin_fma(cp, t2, 0x1.e1f506891babbp-3);
    cp = __builtin_fma(cp, t2, -0x1.55d3c7e3cbffap+0);
    cp = __builtin_fma(cp, t2, 0x1.03c1f081b5ac4p+2);
    cp = __builtin_fma(cp, t2, -0x1.3bd3cc9be45dep+2);
    cp = __builtin_fma(cp, t2, 1.0);               // cos(pi t)
    const uint32_t quad = (uint32_t)jd & 3u;
    // quad 0: (cos, sin) = ( C,  S); 1: (-S,  C); 2: (-C, -S); 3: ( S, -C)
    const double c_abs = (quad & 1u) ? sp : cp;
    const double s_abs = (quad & 1u) ? cp : sp;
    f64x2 z;
    z.x = r * ((quad == 1u || quad == 2u) ? -c_abs : c_abs);
    z.y = r * ((quad >= 2u) ? -s_abs : s_abs);
    return z;
}

// Uniform int32 on [a, b): a + floor(w r / 2^32) with r = irm1 + 1 in
// [1, 2^32]; w r = w irm1 + w < 2^64, so one 32 x 32 + 32 multiply-add
// gives it exactly.  The sum wraps like the int32 it stands for.
__device__ __forceinline__ uint32_t uniform_i32(uint32_t w, int32_t ia, uint32_t irm1)
{
    const uint64_t p = (uint64_t)w * irm1 + w;
    return (uint32_t)ia + (uint32_t)(p >> 32);
}

// Coefficients of Wichura's algorithm AS 241 (PPND16; Applied Statistics
// 37(3), 1988): numerator and denominator polynomials of degree 7, lowest
// order first, for the central region (A / B), the near tails (C / D) and
// the far tails (E / F).  Kept in constant memory: read as scalar operands
// they cost no vector registers (FP64 literals would each need two).
static __constant__ double kPpnd16[6][8] = {
    {3.387132872796366608, 133.14166789178437745, 1971.5909503065514427,
     13731.693765509461125, 45921.953931549871457, 67265.770927008700853,
     33430.575583588128105, 2509.0809287301226727},
    {1.0, 42.313330701600911252, 687.1870074920579083, 5394.1960214247511077,
     21213.794301586595867, 39307.89580009271061, 28729.085735721942674,
     5226.495278852545925},
    {1.42343711074968357734, 4.6303378461565452959, 5.7694972214606914055,
     3.64784832476320460504, 1.27045825245236838258, 0.24178072517745061177,
     0.0227238449892691845833, 7.7454501427834140764e-4},
    {1.0, 2.05319162663775882187, 1.6763848301838038494, 0.68976733498510000455,
     0.14810397642748007459, 0.0151986665636164571966, 5.475938084995344946e-4,
     1.05075007164441684324e-9},
    {6.6579046435011037772, 5.4637849111641143699, 1.7848265399172913358,
     0.29656057182850489123, 0.026532189526576123093, 0.0012426609473880784386,
     2.71155556874348757815e-5, 2.01033439929228813265e-7},
    {1.0, 0.59983220655588793769, 0.13692988092273580531, 0.0148753612908506148525,
     7.868691311456132591e-4, 1.8463183175100546818e-5, 1.4215117583164458887e-7,
     2.04426310338993978564e-15}};

// Polynomial j of the table at x by Horner's rule with fused multiply-adds.
__device__ __forceinline__ double ppnd16_poly(int j, double x)
{
    double r = kPpnd16[j][7];
#pragma unroll
    for (int k = 6; k >= 0; --k) r = __builtin_fma(r, x, kPpnd16[j][k]);
    return r;
}

// Phi^-1(u) by AS 241 (as normal_quantile below) for FP32 outputs: the
// tail's logarithm, square root and both divisions use the refined
// estimates above (ln_fast, sqrt_fast for -ln t <= 34, recip_fast), so z
// carries about 2e-9 relative error (from the logarithm) before its one
// rounding to FP32.
__device__ __forceinline__ double normal_quantile_f32(double u)
{
    const double q = u - 0.5;
    if (__builtin_fabs(q) <= 0.425) {
        const double r = __builtin_fma(-q, q, 0.180625);
        return q * ppnd16_poly(0, r) * recip_fast(ppnd16_poly(1, r));
    }
    const double t = q < 0.0 ? u : 1.0 - u;
    double r = sqrt_fast(-ln_fast(t));
    double z;
    if (r <= 5.0) {
        r -= 1.6;
        z = ppnd16_poly(2, r) * recip_fast(ppnd16_poly(3, r));
    } else {
        r -= 5.0;
        z = ppnd16_poly(4, r) * recip_fast(ppnd16_poly(5, r));
    }
    return q < 0.0 ? -z : z;
}

// Standard normal quantile Phi^-1(u), u in (0, 1), in FP64 by AS 241,
// whose rational approximations have relative error near 1e-16.  Central
// region |u - 1/2| <= 0.425: z = q A(r) / B(r), q = u - 1/2 (exact),
// r = 0.180625 - q^2.  Tails: r = sqrt(-ln min(u, 1 - u)), then
// C(r - 1.6) / D(r - 1.6) for r <= 5 and E(r - 5) / F(r - 5) beyond, with
// the sign of q.  (The device library's quantile is several times larger
// and spills registers when inlined into the generation loops.)  The
// logarithm, square root and divisions are the FP64 routines above (each
// within about an ulp), so z is within a few ulp.
__device__ __forceinline__ double normal_quantile(double u)
{
    const double q = u - 0.5;
    if (__builtin_fabs(q) <= 0.425) {
        const double r = __builtin_fma(-q, q, 0.180625);
        return q * div_f64(ppnd16_poly(0, r), ppnd16_poly(1, r));
    }
    const double t = q < 0.0 ? u : 1.0 - u;   // exact; t <= 0.075
    double r = sqrt_f64(-ln_f64(t));
    double z;
    if (r <= 5.0) {
        r -= 1.6;
        z = div_f64(ppnd16_poly(2, r), ppnd16_poly(3, r));
    } else {
        r -= 5.0;
        z = div_f64(ppnd16_poly(4, r), ppnd16_poly(5, r));
    }
    return q < 0.0 ? -z : z;
}

// Inverse-CDF Gaussian from one word: u = ((w >> 8) + 1/2) 2^-24 (exact in
// FP64, strictly inside (0, 1); -ln t <= 25 ln 2), z = Phi^-1(u) in FP64,
// rounded once to FP32.
__device__ __forceinline__ float icdf_f32(uint32_t w)
{
    const double u = ((double)(w >> 8) + 0.5) * 0x1p-24;
    return (float)normal_quantile_f32(u);
}

// Four inverse-CDF Gaussians, two quantiles at a time (a rolled loop that
// rotates the words through the vector), so that the registers of two
// quantiles suffice while their two chains overlap.
__device__ __forceinline__ f32x4 icdf4_f32(u32x4 w)
{
    f32x4 f = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int j = 0; j < 2; ++j) {
        const float z0 = icdf_f32(w.x);
        const float z1 = icdf_f32(w.y);
        w = u32x4{w.z, w.w, w.x, w.y};
        f = f32x4{f.z, f.w, z0, z1};
    }
    return f;
}

// The FP64 uniform of an inverse-CDF Gaussian from two Philox words: with
// v the 53-bit value of (hi:lo) as for uniform FP64,
// u = (floor(v / 2) + 1/2) 2^-52 (53 significant bits, exact).
__device__ __forceinline__ double icdf_u64(uint32_t lo, uint32_t hi)
{
    const uint64_t v = (((uint64_t)hi << 32) | lo) >> 12;
    return ((double)v + 0.5) * 0x1p-52;
}

// Two FP64 inverse-CDF Gaussians from four Philox words, one at a time.
__device__ __forceinline__ f64x2 icdf2_f64(u32x4 w)
{
    f64x2 d = {0.0, 0.0};
#pragma unroll 1
    for (int j = 0; j < 2; ++j) {
        const double z = normal_quantile(icdf_u64(w.x, w.y));
        w = u32x4{w.z, w.w, w.x, w.y};
        d = f64x2{d.y, z};
    }
    return d;
}

}  // namespace mirng
