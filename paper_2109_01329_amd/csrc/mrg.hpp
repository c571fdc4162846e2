// MRG32k3a device code shared by the plain / substream kernel and the
// batched kernel (L'Ecuyer, Oper. Res. 1999).
//
// A workgroup of kMrgThreads threads produces outputs in passes: thread t
// runs L consecutive steps of its own sequence into its LDS row, then the
// group writes the rows back with 16-byte stores on the output's 16-byte
// grid.  Rows are padded by 16 bytes so that 8 consecutive lanes reading
// 16 bytes hit distinct banks.
//
// The recurrence runs in FP64 on balanced residues: all products are below
// 2^53 and exact, and the quotient by m is rounded to the nearest integer
// with the 1.5 * 2^52 constant; the output combines the two components'
// canonical residues in 32-bit integer arithmetic.  The results are the
// exact integers of the definition.
#pragma once

#include "internal.hpp"
#include "transforms.hpp"

namespace mirng {

constexpr int kMrgThreads = 256;
constexpr int kMatWords = 18;   // two 3x3 matrices (component 1, component 2)
constexpr int kCDigits = 4;     // chunk index < 64^4 = 2^24

// x mod m1 for any 64-bit x (2^32 = 209 mod m1).
__device__ __forceinline__ uint32_t red_m1(uint64_t x)
{
    x = (x >> 32) * 209u + (x & 0xFFFFFFFFull);
    x = (x >> 32) * 209u + (x & 0xFFFFFFFFull);
    return (uint32_t)(x >= kM1 ? x - kM1 : x);
}

// x mod m2 for any 64-bit x (2^32 = 22853 mod m2).
__device__ __forceinline__ uint32_t red_m2(uint64_t x)
{
    x = (x >> 32) * 22853u + (x & 0xFFFFFFFFull);
    x = (x >> 32) * 22853u + (x & 0xFFFFFFFFull);
    return (uint32_t)(x >= kM2 ? x - kM2 : x);
}

// v <- M v for both components; M points at 18 words (comp 1 then comp 2).
__device__ __forceinline__ void apply_mat(const uint32_t *M, uint32_t v[6])
{
    uint32_t r[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const uint64_t a = red_m1((uint64_t)M[3 * i] * v[0]) +
                           (uint64_t)red_m1((uint64_t)M[3 * i + 1] * v[1]) +
                           red_m1((uint64_t)M[3 * i + 2] * v[2]);
        r[i] = red_m1(a);
        const uint64_t b = red_m2((uint64_t)M[9 + 3 * i] * v[3]) +
                           (uint64_t)red_m2((uint64_t)M[9 + 3 * i + 1] * v[4]) +
                           red_m2((uint64_t)M[9 + 3 * i + 2] * v[5]);
        r[3 + i] = red_m2(b);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = r[i];
}

constexpr double kM1d = 4294967087.0;
constexpr double kM2d = 4294944443.0;
constexpr double kInvM1 = 1.0 / 4294967087.0;
constexpr double kInvM2 = 1.0 / 4294944443.0;
constexpr double kNorm = 1.0 / 4294967088.0;   // 1 / (m1 + 1), rounded once

struct MrgState {
    double a0, a1, a2;   // x1[n-3], x1[n-2], x1[n-1]
    double b0, b1, b2;   // x2[n-3], x2[n-2], x2[n-1]
};

__device__ __forceinline__ MrgState mrg_state(const uint32_t v[6])
{
    return MrgState{(double)v[0], (double)v[1], (double)v[2],
                    (double)v[3], (double)v[4], (double)v[5]};
}

// Adding 1.5 * 2^52 to a double of magnitude below 2^51 rounds it to an
// integer (round to nearest even); subtracting it again gives that integer.
constexpr double kRound = 0x1.8p52;

// p mod m as a balanced representative r in [-m/2 - 2, m/2 + 2]: k =
// RN(p * RN(1/m)) is within 4e-10 of p / m (|p / m| < 2^21), so
// r = fma(-k, m, p) = p - k m is exact.
__device__ __forceinline__ double mod_balanced(double p, double m, double inv_m)
{
    const double k = __builtin_fma(p, inv_m, kRound) - kRound;
    return __builtin_fma(-k, m, p);
}

// One step; returns the combined output y in [1, m1].
// The state words are integers held as doubles, each either in [0, m) (the
// start state) or a balanced representative in [-m/2 - 2, m/2 + 2] (every
// word a step writes), so |p| = |a x[n-2] - b x[n-3]| stays below 7.8e15 <
// 2^53 for both components and every product is exact; the recurrence is
// linear modulo m, so any representative gives the right residues.  Only
// the output needs the canonical residues x1 in [0, m1), x2 in [0, m2):
// with i = the balanced word as an int32, (uint32) i + m (mod 2^32) =
// (uint32) i - 209 (m1) or - 22853 (m2) for negative i, and
// y = x1 - x2 (+ m1 = - 209 mod 2^32 when x1 <= x2) in 32-bit wrap-around
// arithmetic.  Only full-rate FP64 adds, multiplies and FMAs touch the
// state.
//
// The canonical residue is one v_mad_i32_i24: the sign bit of i (0 or 1,
// a 24-bit operand) times -k (k = 209 or 22853), plus i.  (The compiler's
// own form of the same select is a shift, an AND and an add.)
__device__ __forceinline__ uint32_t canon_residue(int32_t i, int32_t neg_k)
{
    uint32_t r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"((uint32_t)i >> 31), "s"(neg_k), "v"(i));
    return r;
}

__device__ __forceinline__ uint32_t mrg_step(MrgState &s)
{
    const double p1 = mod_balanced(__builtin_fma(1403580.0, s.a1, -810728.0 * s.a0), kM1d,
                                   kInvM1);
    const double p2 = mod_balanced(__builtin_fma(527612.0, s.b2, -1370589.0 * s.b0), kM2d,
                                   kInvM2);
    s.a0 = s.a1; s.a1 = s.a2; s.a2 = p1;
    s.b0 = s.b1; s.b1 = s.b2; s.b2 = p2;
    const int32_t i1 = (int32_t)p1;
    const int32_t i2 = (int32_t)p2;
    const uint32_t x1 = canon_residue(i1, -209);
    const uint32_t x2 = canon_residue(i2, -22853);
    return x1 - x2 - (x1 <= x2 ? 209u : 0u);
}

// Uniform FP32 of an output y: (y >> 8) 2^-24.
__device__ __forceinline__ float y_to_u01f(uint32_t y)
{
    return (float)(y >> 8) * 0x1p-24f;
}

// Uniform FP64 of an output y: y RN(1 / (m1 + 1)).
__device__ __forceinline__ double y_to_u01d(uint32_t y)
{
    return (double)y * kNorm;
}

template <int KIND>
struct MrgShape {
    static constexpr int ESZ = elem_bytes(KIND);
    static constexpr int L = 128 / ESZ;          // outputs per thread per pass
    static constexpr int ROW = L * ESZ + 16;     // LDS row slot, bytes
    static constexpr int OFF = 16;               // the row's outputs start here
    static constexpr int VPR = L * ESZ / 16;     // 16-byte vectors per row
    static constexpr int EPV = 16 / ESZ;         // elements per vector
};

// Thread t's row in the pass buffer.  The 16 bytes before the row's outputs
// hold, when the output is not 16-byte aligned, the previous pass's last
// elements (see mrg_store_pass).
template <int KIND>
__device__ __forceinline__ char *mrg_row(char *lds, uint32_t t)
{
    return lds + t * MrgShape<KIND>::ROW + MrgShape<KIND>::OFF;
}

// One 16-byte vector of outputs (EPV of them) from the next steps of `s`.
template <int KIND>
__device__ __forceinline__ u32x4 mrg_vec(MrgState &s, const Epilogue &ep)
{
    u32x4 pk;
    if constexpr (KIND == kBits) {
        pk.x = mrg_step(s); pk.y = mrg_step(s);
        pk.z = mrg_step(s); pk.w = mrg_step(s);
    } else if constexpr (KIND == kU32F || KIND == kGauss || KIND == kIcdf) {
        f32x4 f;
        if constexpr (KIND == kU32F) {
            f.x = y_to_u01f(mrg_step(s)); f.y = y_to_u01f(mrg_step(s));
            f.z = y_to_u01f(mrg_step(s)); f.w = y_to_u01f(mrg_step(s));
        } else {
            u32x4 y;
            y.x = mrg_step(s); y.y = mrg_step(s);
            y.z = mrg_step(s); y.w = mrg_step(s);
            if constexpr (KIND == kGauss) {
                f.xy = box_muller(y.x, y.y);
                f.zw = box_muller(y.z, y.w);
            } else {
                f = icdf4_f32(y);
            }
        }
        if (ep.ranged) {
            f.x = __builtin_fmaf(f.x, ep.d32, ep.a32);
            f.y = __builtin_fmaf(f.y, ep.d32, ep.a32);
            f.z = __builtin_fmaf(f.z, ep.d32, ep.a32);
            f.w = __builtin_fmaf(f.w, ep.d32, ep.a32);
        }
        pk = __builtin_bit_cast(u32x4, f);
    } else if constexpr (KIND == kI32) {
        pk.x = uniform_i32(mrg_step(s), ep.ia, ep.irm1);
        pk.y = uniform_i32(mrg_step(s), ep.ia, ep.irm1);
        pk.z = uniform_i32(mrg_step(s), ep.ia, ep.irm1);
        pk.w = uniform_i32(mrg_step(s), ep.ia, ep.irm1);
    } else {
        static_assert(KIND == kU64F || KIND == kGauss64 || KIND == kIcdf64, "unknown kind");
        // u = y / (m1 + 1) as for uniform FP64: never 0 or 1
        const double u0 = y_to_u01d(mrg_step(s));
        const double u1 = y_to_u01d(mrg_step(s));
        f64x2 d;
        if constexpr (KIND == kU64F)
            d = f64x2{u0, u1};
        else if constexpr (KIND == kGauss64)
            d = box_muller64(u0, u1);
        else
            d = normal_quantile2(u0, u1);
        if (ep.ranged) {
            d.x = __builtin_fma(d.x, ep.d64, ep.a64);
            d.y = __builtin_fma(d.y, ep.d64, ep.a64);
        }
        pk = __builtin_bit_cast(u32x4, d);
    }
    return pk;
}

// Runs L steps of `s` and writes the L outputs into `row` (16-byte aligned).
// The inverse-CDF kinds, and ROLLED callers (the one-off head row), evaluate
// one 16-byte vector at a time in a rolled loop, so that the registers of
// one vector suffice; the other kinds unroll the row.
template <int KIND, bool ROLLED = false>
__device__ __forceinline__ void mrg_fill_row(MrgState &s, char *row, const Epilogue &ep)
{
    using S = MrgShape<KIND>;
    if constexpr (ROLLED || KIND == kIcdf || KIND == kIcdf64) {
#pragma unroll 1
        for (int v = 0; v < S::VPR; ++v) *(u32x4 *)(row + v * 16) = mrg_vec<KIND>(s, ep);
    } else {
#pragma unroll
        for (int v = 0; v < S::VPR; ++v) *(u32x4 *)(row + v * 16) = mrg_vec<KIND>(s, ep);
    }
}

template <int ESZ>
__device__ __forceinline__ void put_elem(char *out, uint64_t e, const char *src)
{
    if constexpr (ESZ == 4)
        *(g_u32 *)(out + e * 4) = *(const uint32_t *)src;
    else
        *(g_u64 *)(out + e * 8) = *(const uint64_t *)src;
}

// Elements between the previous 16-byte boundary and element 0 of `out`.
template <int KIND>
__device__ __forceinline__ uint32_t mrg_head(const char *out)
{
    return (uint32_t)(((uintptr_t)out & 15u) / MrgShape<KIND>::ESZ);
}

// Writes one pass back to memory.  Row t of `lds` (mrg_row) holds the L
// outputs of elements [e0 + t * stride, + L) of an output array of n
// elements whose element 0 is at `out` (element-aligned; e0 and stride are
// multiples of L), and elements at or beyond n are not written.  With h =
// mrg_head(out), the rows cut the 16-byte grid at row-local offset -h.
// - h = 0: every row is VPR whole vectors.
// - h != 0 and the whole pass inside the output: each row stores the VPR
//   whole vectors at row-local [j EPV - h, + EPV), j < VPR; the first of
//   them takes its h leading elements from the 16 bytes before the row,
//   where the caller has put the previous pass's last h elements
//   (`pending`), or, in a thread's first pass (no pending), is written
//   element by element for its own EPV - h elements.  The row's last h
//   elements are left to the next pass, or to mrg_store_tail after the
//   last one: returns true.
// - otherwise, every element of row-local [-h (if pending) or 0, L) below
//   n is written, whole vectors where they lie inside; returns false.
// A misaligned output thus costs two partial vectors per thread range
// instead of two per pass.
template <int KIND>
__device__ bool mrg_store_pass(const char *lds, uint64_t e0, uint64_t stride, uint64_t n,
                               char *out, int nt, bool pending)
{
    using S = MrgShape<KIND>;
    constexpr int ESZ = S::ESZ, EPV = S::EPV, VPR = S::VPR, L = S::L;
    const uint32_t h = mrg_head<KIND>(out);
    const uint32_t t = threadIdx.x;
    if (e0 + (uint64_t)(kMrgThreads - 1) * stride + L <= n) {
        // Thread t stores vector t mod VPR of rows t / VPR + i RPI, i < VPR,
        // so its LDS and global addresses advance by fixed steps.
        constexpr uint32_t RPI = kMrgThreads / VPR;
        static_assert(RPI * VPR == kMrgThreads, "rows per step");
        const uint32_t j = t % VPR;
        const uint32_t r = t / VPR;
        if (h == 0) {
            const char *src = lds + r * S::ROW + S::OFF + j * 16;
            char *dst = out + (e0 + (uint64_t)r * stride + j * EPV) * ESZ;
            const uint64_t dstep = (uint64_t)RPI * stride * ESZ;
#pragma unroll
            for (int i = 0; i < VPR; ++i) {
                const u32x4 val = *(const u32x4 *)(src + i * RPI * S::ROW);
                if (nt)
                    __builtin_nontemporal_store(val, (g_u32x4 *)(dst + i * dstep));
                else
                    *(g_u32x4 *)(dst + i * dstep) = val;
            }
            return false;
        }
        const int32_t i0 = (int32_t)(j * EPV) - (int32_t)h;   // row-local, >= -h
        const char *src = lds + r * S::ROW + S::OFF + i0 * ESZ;
        char *dst = out + ((int64_t)(e0 + (uint64_t)r * stride) + i0) * ESZ;   // 16-aligned
        const uint64_t dstep = (uint64_t)RPI * stride * ESZ;
        // (pending is the same in every thread: the loop below then has no
        // per-lane branch, so its LDS reads issue ahead of the stores)
        const bool part = j == 0 && !pending;
#pragma unroll
        for (int i = 0; i < VPR; ++i) {
            const char *sp = src + i * RPI * S::ROW;
            u32x4 val;
            if constexpr (ESZ == 4) {
                const uint32_t *p = (const uint32_t *)sp;
                val = u32x4{p[0], p[1], p[2], p[3]};
            } else {
                const uint2 *p = (const uint2 *)sp;
                const uint2 x = p[0], y = p[1];
                val = u32x4{x.x, x.y, y.x, y.y};
            }
            if (pending || !part) {
                if (nt)
                    __builtin_nontemporal_store(val, (g_u32x4 *)(dst + i * dstep));
                else
                    *(g_u32x4 *)(dst + i * dstep) = val;
            }
        }
        if (part) {
            // a thread range's first vector: its h leading elements belong
            // to the range before, which writes them as its tail
#pragma unroll
            for (int i = 0; i < VPR; ++i) {
                const char *sp = src + i * RPI * S::ROW;
                char *dp = dst + i * dstep;
                for (int k = (int)h; k < EPV; ++k) {
                    if constexpr (ESZ == 4)
                        ((g_u32 *)dp)[k] = ((const uint32_t *)sp)[k];
                    else
                        ((g_u64 *)dp)[k] = ((const uint64_t *)sp)[k];
                }
            }
        }
        return true;
    }
    const int32_t lo = pending ? -(int32_t)h : 0;   // first row-local element to write
    const uint32_t nv = VPR + (h ? 1u : 0u);
    for (uint32_t vi = t; vi < (uint32_t)kMrgThreads * nv; vi += kMrgThreads) {
        const uint32_t row = vi / nv;
        const uint32_t j = vi - row * nv;
        const uint64_t r0 = e0 + (uint64_t)row * stride;     // element of row offset 0
        const char *src = lds + row * S::ROW + S::OFF;
        // row-local index of the vector's first element (may be negative)
        const int32_t i0 = (int32_t)(j * EPV) - (int32_t)h;
        if (r0 + (uint64_t)(i0 + EPV) <= n && i0 >= lo && i0 + EPV <= L) {
            char *dst = out + ((int64_t)r0 + i0) * ESZ;
            u32x4 val;
            if (h == 0) {
                val = *(const u32x4 *)(src + i0 * ESZ);
            } else if constexpr (ESZ == 4) {
                const uint32_t *p = (const uint32_t *)(src + i0 * 4);
                val = u32x4{p[0], p[1], p[2], p[3]};
            } else {
                const uint2 *p = (const uint2 *)(src + i0 * 8);
                const uint2 x = p[0], y = p[1];
                val = u32x4{x.x, x.y, y.x, y.y};
            }
            if (nt)
                __builtin_nontemporal_store(val, (g_u32x4 *)dst);
            else
                *(g_u32x4 *)dst = val;
        } else {
#pragma unroll
            for (int k = 0; k < EPV; ++k) {
                const int32_t i = i0 + k;
                if (i >= lo && i < L && (int64_t)r0 + i < (int64_t)n)
                    put_elem<ESZ>(out, (uint64_t)((int64_t)r0 + i), src + i * ESZ);
            }
        }
    }
    return false;
}

// Before a pass fills its row: the previous pass's last h elements go to
// the h element slots just before the row (each thread, its own row).
template <int KIND>
__device__ __forceinline__ void mrg_carry_tail(char *row, uint32_t h)
{
    using S = MrgShape<KIND>;
    for (uint32_t k = 0; k < h; ++k) {
        if constexpr (S::ESZ == 4)
            ((uint32_t *)row)[(int32_t)k - (int32_t)h] = ((const uint32_t *)row)[S::L - h + k];
        else
            ((uint64_t *)row)[(int32_t)k - (int32_t)h] = ((const uint64_t *)row)[S::L - h + k];
    }
}

// After the last pass, when it left its row's last h elements (its return
// value): thread t writes them from its row, elements r0 + L - h .. r0 + L
// - 1 with r0 = e0 + t * stride of that pass.
template <int KIND>
__device__ __forceinline__ void mrg_store_tail(const char *row, uint64_t r0, uint32_t h,
                                               char *out)
{
    using S = MrgShape<KIND>;
    for (uint32_t k = S::L - h; k < (uint32_t)S::L; ++k)
        put_elem<S::ESZ>(out, r0 + k, row + k * S::ESZ);
}

}  // namespace mirng
