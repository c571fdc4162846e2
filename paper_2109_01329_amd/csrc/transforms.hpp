// Device-side output transforms shared by the Philox and MRG32k3a kernels
// (library-internal).  Conventions: uniform FP32 = (w >> 8) 2^-24; uniform
// FP64 from two Philox words = 53 bits * 2^-53; Box-Muller on a word pair;
// uniform int32 by an exact multiply-high; inverse-CDF Gaussians on
// uniforms strictly inside (0, 1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bm_tables.hpp"
#include "icdf_coeffs.hpp"

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

// A constant-memory table behind a pointer that the compiler cannot see
// through: its entries are then loaded as wave-uniform scalars and used
// directly as FMA operands (folded into FP64 literals, each would need a
// move into a VGPR pair first, on this chip one instruction per use).
typedef const __attribute__((address_space(4))) double c_f64;

__device__ __forceinline__ c_f64 *scalar_table(const double *p)
{
    c_f64 *q = (c_f64 *)p;
    asm volatile("" : "+s"(q));
    return q;
}

// a b + c with c a wave-uniform scalar: one v_fma_f64 with c in an SGPR
// pair.  (The compiler's own choice for a Horner step is v_fmac_f64, whose
// addend is also its destination, so every uniform coefficient was first
// copied into a VGPR pair: three instructions per step instead of one.)
__device__ __forceinline__ double fma_su(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// c[0] + c[1] t + ... + c[N - 1] t^(N - 1) by Horner's rule, the
// coefficients read as scalars.
template <int N>
__device__ __forceinline__ double horner_s(c_f64 *c, double t)
{
    double p = fma_su(c[N - 1], t, c[N - 2]);
#pragma unroll
    for (int k = N - 3; k >= 0; --k) p = fma_su(p, t, c[k]);
    return p;
}

// LDS copies of the two Box-Muller tables (8 KiB per workgroup).  Every
// kernel that evaluates box_muller() (or its factors), icdf_f32() or
// normal_quantile() calls bm_stage() at its start, before any of its
// threads returns; kernels that do not are given no LDS for them.  Per-lane lookups into LDS cost one ds_read_b128
// each; from constant memory the same lookups went through the vector
// memory path, where a wave's 64 scattered addresses take many cycles.
static __shared__ __attribute__((aligned(16))) double s_bm_log[129][4];
static __shared__ __attribute__((aligned(16))) double s_bm_rot[256][2];

__device__ __forceinline__ void bm_stage()
{
    for (uint32_t i = threadIdx.x; i < 129u * 4u; i += blockDim.x)
        (&s_bm_log[0][0])[i] = (&kBmLogTab[0][0])[i];
    for (uint32_t i = threadIdx.x; i < 256u * 2u; i += blockDim.x)
        (&s_bm_rot[0][0])[i] = (&kBmRotTab[0][0])[i];
    __syncthreads();
}

// Twice the Box-Muller radius, 2r = 2 sqrt(-2 ln u1), for FP32 outputs,
// u1 = v 2^-24 with v = (wa >> 8) + 1 in [1, 2^24], to about 2^-29
// relative error:
//   v = 2^(31 - nz) m, m in [1, 2), so u1 = 2^e m with e = 7 - nz;
//   j = m's nearest multiple of 1/128 (table entry j = 0..128, |f| <= 2^-8
//   below), f = m invc_j - 1 with invc_j ~ 1 / (1 + j/128), and
//   -2 ln u1 = -2 e ln 2 - 2 ln(invc_j) - 2 ln(1 + f)
//            = (nz C + T_j) + f (-2 + f (1 - 2f/3))
//   (C = 2 ln 2 to 50 bits, T_j = 2 ln(invc_j) - 7 C from the table; the
//   series' rest is below f^4/2, 2^-26 relative to its first term, and
//   |f| <= 2^-9 where L is small);
//   nz C + T_j is exactly 0 for u1 = 1 (nz = 7, j = 0) and for u1 just
//   below 1 (nz = 8, j = 128), so L keeps the relative accuracy of its
//   series term there;
//   y = the hardware reciprocal square root of L (within 2^-24 on gfx950),
//   r0 = L y, and 2r = r0 (3 - r0 y), one Newton step whose halving moves
//   into the rotation table (which holds half of sin and cos).  L = 0
//   (u1 = 1) gives 0: y is taken of L + 2^-100, which is L itself for
//   every other L (all above 2^-24), one full-rate add where v_max_f64
//   issues at half rate.
// The table entry's byte offset j * 32 is ((mi >> 19) - 4080) & 0x1FE0 for
// mi = m 2^31: mi >> 19 is 4096 (m's leading bit) + 16 g + (4 lower bits)
// with g m's top 8 fraction bits, so the difference is 16 (g + 1) plus
// those bits, in [16, 4111], and the mask leaves 32 floor((g + 1) / 2).
__device__ __forceinline__ double bm_radius2(uint32_t wa)
{
    const uint32_t v = (wa >> 8) + 1u;
    const uint32_t nz = (uint32_t)__builtin_clz(v);
    const uint32_t mi = v << nz;                               // m 2^31
    const uint32_t off = ((mi >> 19) - 4080u) & 0x1FE0u;
    const double *ent = (const double *)((const char *)&s_bm_log[0][0] + off);
    const double f = __builtin_fma((double)mi, ent[0], -1.0);
    const double base = __builtin_fma((double)nz, 0x1.62e42fefa39f0p+0, ent[1]);
    const double q1 = __builtin_fma(f, -0x1.5555555555555p-1, 1.0);
    const double q2 = __builtin_fma(f, q1, -2.0);
    const double L = __builtin_fma(f, q2, base);
    const double y = __builtin_amdgcn_rsq(L + 0x1p-100);
    const double r0 = L * y;
    return r0 * __builtin_fma(-r0, y, 3.0);
}

// Half of (cos, sin) of 2 pi u2 for FP32 outputs, u2 = k 2^-24 with
// k = wb >> 8, to about 2^-29 relative error: j = k's nearest multiple of
// 2^16 (table entry j mod 256, the angle 2 pi j / 256), and the rest of the
// angle x = K t with t = k - 2^16 j (an integer, |t| <= 2^15) and
// K = 2 pi 2^-24, |x| <= pi / 256:
//   sin x = t (K - K^3 t^2 / 6) (the rest below x^5/120) and
//   cos x = 1 - K^2 t^2 / 2 (the rest below x^4/24 = 2^-30), with t^2
//   exact, then the rotation cos = C cos x - S sin x, sin = S cos x + C sin x
//   by the entry's (S, C) / 2.
// The table is exact at quarter turns, so the exact zeros of cos and sin
// come out as zeros, and values next to them keep the series' relative
// accuracy (the entries there have |S| or |C| = sin(2 pi / 256) / 2, at
// most twice the result).
__device__ __forceinline__ f64x2 bm_unit_half(uint32_t wb)
{
    // j mod 256 = the top 8 bits of k + 2^15, and k - 2^16 j is k's low 16
    // bits read as a signed integer
    const uint32_t jr = (wb + 0x800000u) >> 24;
    const double t = (double)(int32_t)(int16_t)(uint16_t)(wb >> 8);
    const double S = s_bm_rot[jr][0];
    const double C = s_bm_rot[jr][1];
    const double t2 = t * t;
    const double cx = __builtin_fma(t2, -0x1.3bd3cc9be45dep-44, 1.0);   // -K^2 / 2
    const double sx = t * __builtin_fma(t2, -0x1.4abbce625be53p-67, 0x1.921fb54442d18p-22);
    f64x2 cs;
    cs.x = __builtin_fma(C, cx, -(S * sx));
    cs.y = __builtin_fma(S, cx, C * sx);
    return cs;
}

// Box-Muller on one word pair, FP32 outputs: z0 = RN32(2r (cos / 2)),
// z1 = RN32(2r (sin / 2)) from the two FP64 factors above, each within
// about 2^-29, so every output is within 0.55 ulp of the exact transform
// of the same two inputs.
__device__ __forceinline__ f32x2 box_muller(uint32_t wa, uint32_t wb)
{
    const double r2 = bm_radius2(wa);
    const f64x2 cs = bm_unit_half(wb);
    f32x2 z;
    z.x = (float)(r2 * cs.x);
    z.y = (float)(r2 * cs.y);
    return z;
}

// sqrt(x) for x = 0 or x in [2^-60, 80] in FP64, to about one ulp: the
// refined reciprocal square root y of xs = x + 2^-200 (x itself but for
// x = 0; one full-rate add where v_max_f64 issues at half rate), then
// r = x y corrected once, r + (y / 2)(x - r^2); x = 0 gives 0.
__device__ __forceinline__ double sqrt_f64(double x)
{
    const double xs = x + 0x1p-200;
    const double h = 0.5 * xs;
    double y = __builtin_amdgcn_rsq(xs);
    y = __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
    const double r = x * y;
    return __builtin_fma(0.5 * y, __builtin_fma(-r, r, x), r);
}

// Series of the FP64 table-driven transforms, lowest order first:
// ln(1 + f) / f - 1 over f = -1/2 + f/3 - ... + f^5/7 (|f| <= 2^-8: the rest
// below f^7/8 < 2^-59); (sin x / x - 1) / x^2 = -1/6 + x^2/120 - x^4/5040
// and (cos x - 1) / x^2 = -1/2 + x^2/24 - x^4/720 for |x| <= pi/256 (the
// rest below 1.5e-21 and 1.3e-20 relative).
static __constant__ double kLn1pSeries[6] = {
    -0.5, 0x1.5555555555555p-2, -0.25, 0x1.999999999999ap-3, -0x1.5555555555555p-3,
    0x1.2492492492492p-3};
static __constant__ double kSinSmall[3] = {-0x1.5555555555555p-3, 0x1.1111111111111p-7,
                                           -0x1.a01a01a01a01ap-13};
static __constant__ double kCosSmall[3] = {-0.5, 0x1.5555555555555p-5, -0x1.6c16c16c16c17p-10};

// ln u for u in [2^-64, 1] in FP64, within about an ulp, from the LDS log
// table: u = 2^e m (e and m in [1, 2) from u's bits), j = m's nearest
// multiple of 1/128, f = m invc_j - 1 (|f| <= 2^-8), and
// ln u = (e ln2_hi + hi_j) + ((e ln2_lo + lo_j) + ln(1 + f)), with
// hi_j + lo_j = ln(1 / invc_j).  e ln2_hi + hi_j is exact, and for u just
// below 1 (e = -1, j = 128) both exponent-table sums are exactly 0, so the
// result keeps the series' relative accuracy where ln u is small.
__device__ __forceinline__ double ln_tab64(double u)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, u);
    const uint32_t hi = (uint32_t)(b >> 32);
    const int32_t e = (int32_t)(hi >> 20) - 1023;
    const uint32_t j = (((hi >> 12) & 255u) + 1u) >> 1;
    const double m31 =
        __builtin_bit_cast(double, (b & 0x000FFFFFFFFFFFFFull) | 0x41E0000000000000ull);
    const double f = __builtin_fma(m31, s_bm_log[j][0], -1.0);
    const double s = __builtin_fma(f * f, horner_s<6>(scalar_table(kLn1pSeries), f), f);
    const double de = (double)e;
    const double h = __builtin_fma(de, 0x1.62e42fefa3800p-1, s_bm_log[j][2]);
    const double l = __builtin_fma(de, 0x1.ef35793c76730p-45, s_bm_log[j][3]);
    return h + (l + s);
}

// Box-Muller in FP64 on a pair of FP64 uniforms u1 in (0, 1], u2 in [0, 1):
// 2r = sqrt(-8 ln u1) (ln_tab64, the FP64 square root), and half of
// (cos, sin) of 2 pi u2 from the rotation table in LDS: j = u2's nearest
// multiple of 1/256 (by the 1.5 * 2^52 rounding constant), t = u2 - j/256
// exactly (Sterbenz), x = 2 pi t (|x| <= pi/256), sin x and cos x by their
// series through x^7 and x^6, rotated by the entry (S, C) = (sin, cos)(2 pi
// j / 256) / 2.  The entries are exact at quarter turns, so zeros stay
// exact (u1 = 1 gives +-0); next to them the entries' |S| or |C| is at most
// twice the result.  Each factor is within a few ulp.  Needs the tables in
// LDS.
__device__ __forceinline__ f64x2 box_muller64(double u1, double u2)
{
    const double r = sqrt_f64(-8.0 * ln_tab64(u1));
    const double jb = __builtin_fma(u2, 256.0, kRound2);        // 1.5 2^52 + j
    const double jd = jb - kRound2;
    const uint32_t j = (uint32_t)__builtin_bit_cast(uint64_t, jb) & 255u;
    const double t = __builtin_fma(jd, -0x1p-8, u2);
    const double x = t * 0x1.921fb54442d18p+2;                  // 2 pi t
    const double x2 = x * x;
    const double sx = __builtin_fma(x * x2, horner_s<3>(scalar_table(kSinSmall), x2), x);
    const double cx = __builtin_fma(x2, horner_s<3>(scalar_table(kCosSmall), x2), 1.0);
    const double S = s_bm_rot[j][0];
    const double C = s_bm_rot[j][1];
    f64x2 z;
    z.x = r * __builtin_fma(C, cx, -(S * sx));
    z.y = r * __builtin_fma(S, cx, C * sx);
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

// -ln a for a in [2^-24, 1], to about 2^-45 absolute error, from the FP32
// Box-Muller log table (in LDS): a = 2^e m with e and m in [1, 2) read from
// a's bits, j = m's nearest multiple of 1/128 (|f| <= 2^-8 below),
// f = m invc_j - 1, and -ln a = -e ln 2 + ln(invc_j) - ln(1 + f)
// = (7 - e) C/2 + T_j/2 - ln(1 + f) with the table's T_j = 2 ln(invc_j) - 7 C
// (C = 2 ln 2 to 50 bits, off by at most 2^-50 relative, which costs
// (7 - e) 2^-51 absolute) and ln(1 + f) = f - f^2/2 + f^3/3 (the rest below
// f^4/4 = 2^-34).  As in the Box-Muller radius, the exponent and table terms
// cancel exactly where a is just below 1 (e = -1, j = 128).
__device__ __forceinline__ double neg_ln_tab(double a)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, a);
    const uint32_t hi = (uint32_t)(b >> 32);
    const int32_t e7 = 1030 - (int32_t)(hi >> 20);             // 7 - e
    const uint32_t j = (((hi >> 12) & 255u) + 1u) >> 1;
    // m 2^31: a's significand under the exponent 1023 + 31
    const double m31 =
        __builtin_bit_cast(double, (b & 0x000FFFFFFFFFFFFFull) | 0x41E0000000000000ull);
    const double f = __builtin_fma(m31, s_bm_log[j][0], -1.0);
    const double f2 = f * f;
    const double q = __builtin_fma(f, 0x1.5555555555555p-2, -0.5);
    const double s = __builtin_fma(f2, q, f);                  // ln(1 + f)
    // ((7 - e) C + T_j) / 2 - s: the halving is exact
    return __builtin_fma(0.5, __builtin_fma((double)e7, 0x1.62e42fefa39f0p+0, s_bm_log[j][1]), -s);
}

// Inverse-CDF Gaussian from one word, FP32 output: u = ((w >> 8) + 1/2)
// 2^-24, and Phi^-1(u) = sqrt(2) erfinv(x) with x = 2u - 1, written as
// x F(w) with w = -ln(1 - x^2) (the erfinv form of M. Giles, GPU Computing
// Gems 2011; polynomials fitted for this range in icdf_coeffs.hpp):
//   x = (2k + 1 - 2^24) 2^-24 and 1 - x^2 = (1 - x)(1 + x) are exact in FP64
//   (26- and 25-bit factors), w = -ln(1 - x^2) <= 23 ln 2 from neg_ln_tab;
//   F = P(w - 3.125) for w < 6.25 (all but 0.1% of uniforms), else
//   Q(sqrt(w) - 3.25), each fitted within 6e-10 relative; sqrt from the
//   hardware reciprocal square root corrected once.
// z = x F is rounded once to FP32.  F varies slowly with w, so w's absolute
// error costs far below 2^-40 relative.  Needs the Box-Muller tables in LDS.
struct IcdfArg {
    double x, w;
};

__device__ __forceinline__ IcdfArg icdf_arg(uint32_t wd)
{
    const int32_t xi = (int32_t)(((wd >> 8) << 1) + 1u) - (1 << 24);
    IcdfArg a;
    a.x = (double)xi * 0x1p-24;
    a.w = neg_ln_tab((1.0 - a.x) * (1.0 + a.x));
    return a;
}

__device__ __forceinline__ double icdf_tail(double w)
{
    const double y = __builtin_amdgcn_rsq(w);
    const double r0 = w * y;
    const double t = __builtin_fma(0.5 * y, __builtin_fma(-r0, r0, w), r0) - 3.25;
    return horner_s<11>(scalar_table(kIcdfTail), t);
}

__device__ __forceinline__ float icdf_f32(uint32_t wd)
{
    const IcdfArg a = icdf_arg(wd);
    const double p = a.w < 6.25 ? horner_s<13>(scalar_table(kIcdfCentral), a.w - 3.125)
                                : icdf_tail(a.w);
    return (float)(a.x * p);
}

// Four inverse-CDF Gaussians, each with exactly icdf_f32's operations: the
// four central polynomials run interleaved (each scalar coefficient is read
// once for four FMAs, and four independent chains hide the FMA latency),
// and the tail, which about one word in a thousand takes, replaces a
// sample's central value under a branch of its own.
__device__ __forceinline__ f32x4 icdf4_f32(u32x4 wv)
{
    const uint32_t wd[4] = {wv.x, wv.y, wv.z, wv.w};
    IcdfArg a[4];
    double t[4], p[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = icdf_arg(wd[k]);
        t[k] = a[k].w - 3.125;
    }
    c_f64 *c = scalar_table(kIcdfCentral);
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = fma_su(c[12], t[k], c[11]);
#pragma unroll
    for (int j = 10; j >= 0; --j) {
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] = fma_su(p[k], t[k], c[j]);
    }
    f32x4 f;
    float *fo = (float *)&f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!(a[k].w < 6.25)) p[k] = icdf_tail(a[k].w);
        fo[k] = (float)(a[k].x * p[k]);
    }
    return f;
}

// Standard normal quantile Phi^-1(u), u in (0, 1), in FP64: the erfinv form
// of icdf_f32 with the FP64 polynomials of icdf_coeffs.hpp (fitted within
// 1.1e-16 relative):
//   x = 2u - 1 (exact for u >= 1/4; else within half an ulp, which x's role
//   as a factor of the result tolerates);
//   1 - x^2 = 4u(1 - u) from u itself, so that it keeps its relative
//   accuracy however close u is to 0 or 1, and w = -ln(1 - x^2) from
//   ln_tab64 (w <= 51 ln 2 for u >= 2^-53);
//   F = P(w - 3.125) for w < 6.25 (all but 0.1% of uniforms), else with
//   s = sqrt(w) (the FP64 square root), Q1(s - 3.25) for s < 4 and
//   Q2(s - 5.05) beyond; z = x F.
// F changes slowly with w (d ln F / dw < 0.3), so w's absolute error costs
// about as much relative error in z.  Needs the Box-Muller tables in LDS.
struct QuantArg {
    double x, w;
};

__device__ __forceinline__ QuantArg quantile_arg(double u)
{
    QuantArg a;
    a.x = __builtin_fma(u, 2.0, -1.0);
    a.w = -ln_tab64(4.0 * u * (1.0 - u));
    return a;
}

// F beyond the central range, w >= 6.25.
__device__ __forceinline__ double quantile_outer(double w)
{
    const double r = sqrt_f64(w);
    if (r < 4.0)
        return horner_s<21>(scalar_table(kIcdf64Mid), r - 3.25);
    return horner_s<19>(scalar_table(kIcdf64Tail), r - 5.05);
}

__device__ __forceinline__ double normal_quantile(double u)
{
    const QuantArg a = quantile_arg(u);
    const double p = a.w < 6.25 ? horner_s<25>(scalar_table(kIcdf64Central), a.w - 3.125)
                                : quantile_outer(a.w);
    return a.x * p;
}

// Two quantiles, each with exactly normal_quantile's operations, their
// central polynomials interleaved as in icdf4_f32.
__device__ __forceinline__ f64x2 normal_quantile2(double u0, double u1)
{
    const QuantArg a[2] = {quantile_arg(u0), quantile_arg(u1)};
    const double t[2] = {a[0].w - 3.125, a[1].w - 3.125};
    c_f64 *c = scalar_table(kIcdf64Central);
    double p[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) p[k] = fma_su(c[24], t[k], c[23]);
#pragma unroll
    for (int j = 22; j >= 0; --j) {
#pragma unroll
        for (int k = 0; k < 2; ++k) p[k] = fma_su(p[k], t[k], c[j]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
        if (!(a[k].w < 6.25)) p[k] = quantile_outer(a[k].w);
    return f64x2{a[0].x * p[0], a[1].x * p[1]};
}

// The FP64 uniform of an inverse-CDF Gaussian from two Philox words: with
// v the 53-bit value of (hi:lo) as for uniform FP64,
// u = (floor(v / 2) + 1/2) 2^-52 (53 significant bits, exact).
__device__ __forceinline__ double icdf_u64(uint32_t lo, uint32_t hi)
{
    const uint64_t v = (((uint64_t)hi << 32) | lo) >> 12;
    return ((double)v + 0.5) * 0x1p-52;
}

// Two FP64 inverse-CDF Gaussians from four Philox words.
__device__ __forceinline__ f64x2 icdf2_f64(u32x4 w)
{
    return normal_quantile2(icdf_u64(w.x, w.y), icdf_u64(w.z, w.w));
}

}  // namespace mirng
