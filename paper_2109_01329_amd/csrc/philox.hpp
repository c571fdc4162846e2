// Philox4x32-10 device code shared by the plain and batched kernels
// (library-internal): the bijection of Salmon et al. (SC'11), ten rounds
// with Weyl key bumps, the 128-bit block counter, the output transforms of a
// 16-byte unit, its store, and the cross-lane word shift.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "transforms.hpp"

namespace mirng {

// a ^ b ^ c in one gfx950 v_bitop3_b32 (truth table 0x96; XOR3 is symmetric
// in its inputs, so the table does not depend on operand order).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2,
                                          uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t rk0 = k0 + (uint32_t)r * kPhiloxW0;
        const uint32_t rk1 = k1 + (uint32_t)r * kPhiloxW1;
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, rk0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, rk1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    u32x4 w;
    w.x = c0; w.y = c1; w.z = c2; w.w = c3;
    return w;
}

// Block base + j as a 128-bit counter.  NC: the caller has checked that
// base[0] + j does not carry out of the low word, so the three upper words
// are the base's own (wave-uniform: the first round's product of the upper
// pair is then loop-invariant).
template <bool NC = false>
__device__ __forceinline__ u32x4 block_at(const uint32_t base[4], uint32_t k0, uint32_t k1,
                                          uint32_t j)
{
    if constexpr (NC) return philox10(base[0] + j, base[1], base[2], base[3], k0, k1);
    const uint64_t lo0 = ((uint64_t)base[1] << 32) | base[0];
    const uint64_t hi0 = ((uint64_t)base[3] << 32) | base[2];
    const uint64_t lo = lo0 + j;
    const uint64_t hi = hi0 + (lo < lo0 ? 1u : 0u);
    return philox10((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32),
                    k0, k1);
}

// 16 bytes at a 4-byte-aligned address (one global_store_dwordx4 on gfx950).
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef __attribute__((address_space(1))) u32x4_a4 g_u32x4_a4;

// Whether the range (or mean / sd) step applies: RANGED 0 never, 1 always,
// 2 as the epilogue says.  Kernels that know it per launch pass 0 or 1, so
// the loop holds no select between both results.
template <int RANGED>
__device__ __forceinline__ bool ranged(const Epilogue &ep)
{
    if constexpr (RANGED == 2) return ep.ranged != 0;
    else return RANGED != 0;
}

// Four words -> the 16 bytes they become.
template <int KIND, int RANGED = 2>
__device__ __forceinline__ u32x4 transform(const Epilogue &ep, u32x4 w)
{
    u32x4 v;
    if constexpr (KIND == kBits) {
        v = w;
    } else if constexpr (KIND == kU32F) {
        f32x4 f;
        f.x = u01f(w.x); f.y = u01f(w.y); f.z = u01f(w.z); f.w = u01f(w.w);
        if (ranged<RANGED>(ep)) {
            f.x = __builtin_fmaf(f.x, ep.d32, ep.a32);
            f.y = __builtin_fmaf(f.y, ep.d32, ep.a32);
            f.z = __builtin_fmaf(f.z, ep.d32, ep.a32);
            f.w = __builtin_fmaf(f.w, ep.d32, ep.a32);
        }
        v = __builtin_bit_cast(u32x4, f);
    } else if constexpr (KIND == kU64F) {
        f64x2 d;
        d.x = u01d(w.x, w.y);
        d.y = u01d(w.z, w.w);
        if (ranged<RANGED>(ep)) {
            d.x = __builtin_fma(d.x, ep.d64, ep.a64);
            d.y = __builtin_fma(d.y, ep.d64, ep.a64);
        }
        v = __builtin_bit_cast(u32x4, d);
    } else if constexpr (KIND == kGauss64) {
        // u1 = (v_a + 1) 2^-53 from (w.x, w.y), u2 = v_b 2^-53 from (w.z, w.w)
        f64x2 d = box_muller64(u01d(w.x, w.y) + 0x1p-53, u01d(w.z, w.w));
        if (ranged<RANGED>(ep)) {
            d.x = __builtin_fma(d.x, ep.d64, ep.a64);
            d.y = __builtin_fma(d.y, ep.d64, ep.a64);
        }
        v = __builtin_bit_cast(u32x4, d);
    } else if constexpr (KIND == kI32) {
        v.x = uniform_i32(w.x, ep.ia, ep.irm1);
        v.y = uniform_i32(w.y, ep.ia, ep.irm1);
        v.z = uniform_i32(w.z, ep.ia, ep.irm1);
        v.w = uniform_i32(w.w, ep.ia, ep.irm1);
    } else if constexpr (KIND == kIcdf) {
        f32x4 f = icdf4_f32(w);
        if (ranged<RANGED>(ep)) {
            f.x = __builtin_fmaf(f.x, ep.d32, ep.a32);
            f.y = __builtin_fmaf(f.y, ep.d32, ep.a32);
            f.z = __builtin_fmaf(f.z, ep.d32, ep.a32);
            f.w = __builtin_fmaf(f.w, ep.d32, ep.a32);
        }
        v = __builtin_bit_cast(u32x4, f);
    } else if constexpr (KIND == kIcdf64) {
        f64x2 d = icdf2_f64(w);
        if (ranged<RANGED>(ep)) {
            d.x = __builtin_fma(d.x, ep.d64, ep.a64);
            d.y = __builtin_fma(d.y, ep.d64, ep.a64);
        }
        v = __builtin_bit_cast(u32x4, d);
    } else {
        static_assert(KIND == kGauss, "unknown kind");
        f32x4 f;
        f.xy = box_muller(w.x, w.y);
        f.zw = box_muller(w.z, w.w);
        if (ranged<RANGED>(ep)) {
            f.x = __builtin_fmaf(f.x, ep.d32, ep.a32);
            f.y = __builtin_fmaf(f.y, ep.d32, ep.a32);
            f.z = __builtin_fmaf(f.z, ep.d32, ep.a32);
            f.w = __builtin_fmaf(f.w, ep.d32, ep.a32);
        }
        v = __builtin_bit_cast(u32x4, f);
    }
    return v;
}

// Store the 16 bytes of unit u at p: whole when the unit lies inside the
// output (full_lo <= u < full_lo + full_count), else element by element for
// the output indices e0 .. e0 + EPV - 1 that fall in [0, n).
template <int KIND>
__device__ __forceinline__ void put(char *p, u32x4 v, uint32_t u, uint32_t full_lo,
                                   uint32_t full_count, int64_t e0, uint64_t n, int nt)
{
    constexpr int EPV = 16 / elem_bytes(KIND);
    constexpr int ESZ = elem_bytes(KIND);
    if (u - full_lo < full_count) {
        if (nt) __builtin_nontemporal_store(v, (g_u32x4_a4 *)p);
        else *(g_u32x4_a4 *)p = v;
        return;
    }
#pragma unroll
    for (int j = 0; j < EPV; ++j) {
        const int64_t e = e0 + j;
        if (e >= 0 && e < (int64_t)n) {
            if constexpr (ESZ == 4) {
                ((g_u32 *)p)[j] = v[j];
            } else {
                ((g_u64 *)p)[j] = ((uint64_t)v[2 * j + 1] << 32) | v[2 * j];
            }
        }
    }
}

// Words q + 4 s .. q + 4 s + 3 from this lane's block and the next one.
template <int PHASE>
__device__ __forceinline__ u32x4 funnel(u32x4 cur, u32x4 nb)
{
    u32x4 w;
    if constexpr (PHASE == 1) {
        w.x = cur.y; w.y = cur.z; w.z = cur.w; w.w = nb.x;
    } else if constexpr (PHASE == 2) {
        w.x = cur.z; w.y = cur.w; w.z = nb.x; w.w = nb.y;
    } else {
        w.x = cur.w; w.y = nb.x; w.z = nb.y; w.w = nb.z;
    }
    return w;
}

// Lane i receives lane i + 1's v, lane 63 receives fill63: one DPP move
// (wave_shl:1, a GFX9-family wavefront shift; the lane that has no source
// keeps the destination's old value).
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v, uint32_t fill63)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)fill63, (int)v, 0x130, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t lane0(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// The 16 bytes of slot s of a run, stored whole or element by element.
template <int KIND, int RANGED = 2>
__device__ __forceinline__ void emit_slot(const SlotRun &r, uint32_t slot, u32x4 w)
{
    constexpr int EPV = 16 / elem_bytes(KIND);
    const int64_t e0 = (int64_t)slot * EPV - (int64_t)r.head;
    put<KIND>(r.out_base + (uint64_t)slot * 16u, transform<KIND, RANGED>(r.ep, w), slot,
              r.full_lo, r.full_count, e0, r.n, r.ep.nt);
}

// The 16 bytes of slot sb + lane of a run when the caller knows the whole
// slot lies inside the output: one unconditional 16-byte store.  sb is the
// step's (wave-uniform) first slot, so the address is a scalar base plus
// the lane's 16-byte offset.
template <int KIND, int RANGED = 2>
__device__ __forceinline__ void emit_slot_whole(const SlotRun &r, uint32_t sb, uint32_t lane,
                                                u32x4 w)
{
    const u32x4 v = transform<KIND, RANGED>(r.ep, w);
    g_u32x4_a4 *p = (g_u32x4_a4 *)(r.out_base + (uint64_t)sb * 16u) + lane;
    if (r.ep.nt) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Whether the 64 slots sb .. sb + 63 all lie in [lo, lo + width) and inside
// the output (wave-uniform when its arguments are): such a step stores 64
// whole slots with no per-lane checks.
__device__ __forceinline__ bool whole_step(const SlotRun &r, uint32_t sb, uint32_t lo,
                                           uint32_t width)
{
    return width >= 64u && sb - lo <= width - 64u && r.full_count >= 64u &&
           sb - r.full_lo <= r.full_count - 64u;
}

// Whether the blocks base + j, j <= last, stay clear of a carry out of the
// counter's low word (wave-uniform).
__device__ __forceinline__ bool no_carry(const SlotRun &r, uint64_t last)
{
    return (uint64_t)r.base[0] + last < (1ull << 32);
}

// One wave writes slots [s0, s0 + span) of a run, 64 consecutive slots per
// step (lane L takes slot s0 + 64 i + L).  For PHASE != 0 slot s needs the
// tail of block base + s and the head of block base + s + 1: lane L takes
// those words from lane L + 1 and lane 63 from lane 0 of the next step,
// which is evaluated one step ahead.  Must be called by whole waves.
// Slots s0 + 64 i + L for lane L, i < iters, storing those in [lo, hi).
// s0 may lie below lo (modulo 2^32, even "negative"): the lanes before lo
// evaluate blocks that nobody stores, which lets a caller align the steps
// to a memory grid.
// s0, lo and hi are read from lane 0, so the loop control and the
// whole-step test run on the scalar unit.
template <int KIND, int PHASE, int RANGED, bool NC>
__device__ __forceinline__ void walk_slots_body(const SlotRun &r, uint32_t s0, uint32_t lo,
                                                uint32_t hi, uint32_t lane, uint32_t iters)
{
    s0 = lane0(s0);
    lo = lane0(lo);
    const uint32_t width = lane0(hi) - lo;
    iters = lane0(iters);
    if constexpr (PHASE == 0) {
        for (uint32_t it = 0; it < iters; ++it) {
            const uint32_t sb = s0 + (it << 6);
            const uint32_t slot = sb + lane;
            const u32x4 w = block_at<NC>(r.base, r.k0, r.k1, slot);
            if (whole_step(r, sb, lo, width)) emit_slot_whole<KIND, RANGED>(r, sb, lane, w);
            else if (slot - lo < width) emit_slot<KIND, RANGED>(r, slot, w);
        }
    } else {
        u32x4 cur = block_at<NC>(r.base, r.k0, r.k1, s0 + lane);
        for (uint32_t it = 0; it < iters; ++it) {
            const uint32_t sb = s0 + (it << 6);
            const uint32_t slot = sb + lane;
            const u32x4 nxt = block_at<NC>(r.base, r.k0, r.k1, slot + 64u);
            // lane 63 takes lane 0's next-step block
            u32x4 nb;
            nb.x = from_next_lane(cur.x, lane0(nxt.x));
            if constexpr (PHASE >= 2) nb.y = from_next_lane(cur.y, lane0(nxt.y));
            if constexpr (PHASE >= 3) nb.z = from_next_lane(cur.z, lane0(nxt.z));
            const u32x4 w = funnel<PHASE>(cur, nb);
            if (whole_step(r, sb, lo, width)) emit_slot_whole<KIND, RANGED>(r, sb, lane, w);
            else if (slot - lo < width) emit_slot<KIND, RANGED>(r, slot, w);
            cur = nxt;
        }
    }
}

// Slots [lo, hi) of a run in steps of 64 starting at s0 (s0 <= lo, modulo
// 2^32; lo - s0 < 64).  Must be called by whole waves.
template <int KIND, int PHASE, int RANGED = 2>
__device__ __forceinline__ void walk_slots_from(const SlotRun &r, uint32_t s0, uint32_t lo,
                                                uint32_t hi, uint32_t lane)
{
    const uint32_t iters = (hi - s0 + 63u) >> 6;
    // the last block evaluated is the look-ahead of the last step; lo is
    // the first block anything stores
    const uint64_t last = (uint64_t)lo + (uint32_t)(s0 + (iters << 6) + 63u - lo);
    if (no_carry(r, last))
        walk_slots_body<KIND, PHASE, RANGED, true>(r, s0, lo, hi, lane, iters);
    else
        walk_slots_body<KIND, PHASE, RANGED, false>(r, s0, lo, hi, lane, iters);
}

// Slots [s0, s0 + span) of a run, 64 consecutive slots per step.
template <int KIND, int PHASE, int RANGED = 2>
__device__ __forceinline__ void walk_slots(const SlotRun &r, uint32_t s0, uint32_t span,
                                           uint32_t lane)
{
    walk_slots_from<KIND, PHASE, RANGED>(r, s0, s0, s0 + span, lane);
}

// Chunked walk: a wave writes ITERS consecutive chunks of S slots, S = 64
// for PHASE 0 and 63 otherwise.  For PHASE != 0 lane L's slot takes its
// missing words from lane L + 1's block, and lane 63 only evaluates the
// block whose head lane 62 needs (it stores nothing), so chunks are
// independent: all ITERS blocks of a lane are evaluated together (ILP) and
// a wave needs no look-ahead across chunks.  Short runs of whole chunks per
// wave keep the waves in flight on one compact, moving window of memory.
// Must be called by whole waves.
template <int KIND, int PHASE, int ITERS, int RANGED, bool NC>
__device__ __forceinline__ void walk_chunks_body(const SlotRun &r, uint32_t s0, uint32_t span,
                                                 uint32_t lane)
{
    constexpr uint32_t S = PHASE ? 63u : 64u;
    u32x4 b[ITERS];
#pragma unroll
    for (int it = 0; it < ITERS; ++it)
        b[it] = block_at<NC>(r.base, r.k0, r.k1, s0 + it * S + lane);
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const uint32_t off = it * S + lane;
        u32x4 w;
        if constexpr (PHASE == 0) {
            w = b[it];
        } else {
            u32x4 nb;
            nb.x = from_next_lane(b[it].x, 0u);
            if constexpr (PHASE >= 2) nb.y = from_next_lane(b[it].y, 0u);
            if constexpr (PHASE >= 3) nb.z = from_next_lane(b[it].z, 0u);
            w = funnel<PHASE>(b[it], nb);
        }
        if (PHASE == 0 && whole_step(r, s0 + it * S, s0, span))
            emit_slot_whole<KIND, RANGED>(r, s0 + it * S, lane, w);
        else if (lane < S && off < span)
            emit_slot<KIND, RANGED>(r, s0 + off, w);
    }
}

template <int KIND, int PHASE, int ITERS, int RANGED = 2>
__device__ __forceinline__ void walk_chunks(const SlotRun &r, uint32_t s0, uint32_t span,
                                            uint32_t lane)
{
    constexpr uint32_t S = PHASE ? 63u : 64u;
    if (no_carry(r, (uint64_t)s0 + (ITERS - 1) * S + 63u))
        walk_chunks_body<KIND, PHASE, ITERS, RANGED, true>(r, s0, span, lane);
    else
        walk_chunks_body<KIND, PHASE, ITERS, RANGED, false>(r, s0, span, lane);
}

}  // namespace mirng
