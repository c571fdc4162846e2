// Philox4x32-10 bulk generation kernels for gfx950.
//
// The engine is the counter-based Philox-4x32 bijection with 10 rounds of
// Salmon et al. (SC'11); the paper measures exactly this generator with
// uniform FP32 output (arXiv:2109.01329, Sec. 6).  Its separate range-
// transform kernel (Sec. 4.3) is fused here into the store epilogue.
//
// Work layout: the output is cut into 16-byte slots.  Every slot needs four
// consecutive engine words (4 x F32/bits, 2 x F64 from word pairs, or two
// Box-Muller pairs), so lane L of a wave computes Philox block base + slot
// and stores one 16-byte vector; a wave writes 1 KiB contiguously.  When the
// engine position is not a multiple of 4 relative to the 16-byte grid, slot
// s needs the tail of block b and the head of block b + 1: lane L takes
// those words from lane L + 1 (ds_bpermute), and lane 63 from lane 0 of the
// wave's next iteration, which is computed one iteration ahead.  Each wave
// owns a contiguous run of slots, so the extra block per run is 1/iters.
#include "internal.hpp"
#include "transforms.hpp"

namespace mirng {
namespace {

// ---------------------------------------------------------------- engine

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

// Block base + slot as a 128-bit counter.
__device__ __forceinline__ u32x4 block_at(const PhiloxFill &a, uint32_t slot)
{
    const uint64_t lo0 = ((uint64_t)a.base[1] << 32) | a.base[0];
    const uint64_t hi0 = ((uint64_t)a.base[3] << 32) | a.base[2];
    const uint64_t lo = lo0 + slot;
    const uint64_t hi = hi0 + (lo < lo0 ? 1u : 0u);
    return philox10((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi,
                    (uint32_t)(hi >> 32), a.k0, a.k1);
}

// Four words -> the 16 bytes of one slot.
template <int KIND>
__device__ __forceinline__ u32x4 transform(const PhiloxFill &a, u32x4 w)
{
    u32x4 v;
    if constexpr (KIND == kBits) {
        v = w;
    } else if constexpr (KIND == kU32F) {
        f32x4 f;
        f.x = u01f(w.x); f.y = u01f(w.y); f.z = u01f(w.z); f.w = u01f(w.w);
        if (a.ranged) {
            f.x = __builtin_fmaf(f.x, a.d32, a.a32);
            f.y = __builtin_fmaf(f.y, a.d32, a.a32);
            f.z = __builtin_fmaf(f.z, a.d32, a.a32);
            f.w = __builtin_fmaf(f.w, a.d32, a.a32);
        }
        v = __builtin_bit_cast(u32x4, f);
    } else if constexpr (KIND == kU64F) {
        f64x2 d;
        d.x = u01d(w.x, w.y);
        d.y = u01d(w.z, w.w);
        if (a.ranged) {
            d.x = __builtin_fma(d.x, a.d64, a.a64);
            d.y = __builtin_fma(d.y, a.d64, a.a64);
        }
        v = __builtin_bit_cast(u32x4, d);
    } else {
        f32x4 f;
        f.xy = box_muller(w.x, w.y);
        f.zw = box_muller(w.z, w.w);
        if (a.ranged) {
            f.x = __builtin_fmaf(f.x, a.d32, a.a32);
            f.y = __builtin_fmaf(f.y, a.d32, a.a32);
            f.z = __builtin_fmaf(f.z, a.d32, a.a32);
            f.w = __builtin_fmaf(f.w, a.d32, a.a32);
        }
        v = __builtin_bit_cast(u32x4, f);
    }
    return v;
}

template <int KIND>
__device__ __forceinline__ void emit(const PhiloxFill &a, uint32_t slot, u32x4 w)
{
    constexpr int EPV = (KIND == kU64F) ? 2 : 4;   // elements per slot
    constexpr int ESZ = 16 / EPV;
    const u32x4 v = transform<KIND>(a, w);
    char *p = a.out_base + (uint64_t)slot * 16u;
    if (slot - a.full_lo < a.full_count) {
        __builtin_nontemporal_store(v, (u32x4 *)p);
    } else {
        const int64_t e0 = (int64_t)slot * EPV - (int64_t)a.head;
        // first or last slot of the launch: element stores inside [0, n)
#pragma unroll
        for (int j = 0; j < EPV; ++j) {
            const int64_t e = e0 + j;
            if (e >= 0 && e < (int64_t)a.n) {
                if constexpr (ESZ == 4) {
                    ((uint32_t *)p)[j] = v[j];
                } else {
                    const uint64_t d = ((uint64_t)v[2 * j + 1] << 32) | v[2 * j];
                    ((uint64_t *)p)[j] = d;
                }
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

__device__ __forceinline__ uint32_t lane_pull(int addr, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)v);
}

template <int KIND, int PHASE>
__global__ __launch_bounds__(256) void philox_fill_kernel(PhiloxFill a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t first = (uint64_t)wave * a.slots_per_wave;
    if (first >= a.nslots) return;
    const uint32_t s0 = (uint32_t)first;
    const uint32_t span = min(a.slots_per_wave, a.nslots - s0);
    const uint32_t iters = (span + 63u) >> 6;

    if constexpr (PHASE == 0) {
        for (uint32_t it = 0; it < iters; ++it) {
            const uint32_t slot = s0 + (it << 6) + lane;
            const u32x4 w = block_at(a, slot);
            if (slot - s0 < span) emit<KIND>(a, slot, w);
        }
    } else {
        const int next_addr = (int)(((lane + 1u) & 63u) << 2);
        u32x4 cur = block_at(a, s0 + lane);
        for (uint32_t it = 0; it < iters; ++it) {
            const uint32_t slot = s0 + (it << 6) + lane;
            const u32x4 nxt = block_at(a, slot + 64u);
            // lane 0 offers its next-iteration block, which lane 63 needs
            const u32x4 src = (lane == 0) ? nxt : cur;
            u32x4 nb;
            nb.x = lane_pull(next_addr, src.x);
            if constexpr (PHASE >= 2) nb.y = lane_pull(next_addr, src.y);
            if constexpr (PHASE >= 3) nb.z = lane_pull(next_addr, src.z);
            const u32x4 w = funnel<PHASE>(cur, nb);
            if (slot - s0 < span) emit<KIND>(a, slot, w);
            cur = nxt;
        }
    }
}

// Gaussian pairs whose output does not sit on the 16-byte grid in pair
// units: one thread per pair, words p + 2 j and p + 2 j + 1.
__global__ __launch_bounds__(256) void philox_pairs_kernel(PhiloxPairs a)
{
    const uint64_t npairs = (a.n + 1) / 2;
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= npairs) return;
    // word position of the pair (130-bit), then its block(s)
    const uint64_t lo = a.p_lo + 2 * j;
    const uint64_t c1 = lo < a.p_lo ? 1u : 0u;
    const uint64_t mid = a.p_mid + c1;
    const uint32_t top = a.p_top + ((c1 && mid == 0) ? 1u : 0u);
    const uint64_t b_lo = (lo >> 2) | (mid << 62);
    const uint64_t b_hi = (mid >> 2) | ((uint64_t)(top & 3u) << 62);
    const uint32_t lane = (uint32_t)(lo & 3u);
    const u32x4 w0 = philox10((uint32_t)b_lo, (uint32_t)(b_lo >> 32), (uint32_t)b_hi,
                              (uint32_t)(b_hi >> 32), a.k0, a.k1);
    uint32_t wa, wb;
    if (lane < 3) {
        wa = w0[lane];
        wb = w0[lane + 1];
    } else {
        const uint64_t n_lo = b_lo + 1;
        const uint64_t n_hi = b_hi + (n_lo == 0 ? 1u : 0u);
        const u32x4 w1 = philox10((uint32_t)n_lo, (uint32_t)(n_lo >> 32), (uint32_t)n_hi,
                                  (uint32_t)(n_hi >> 32), a.k0, a.k1);
        wa = w0.w;
        wb = w1.x;
    }
    const f32x2 z = box_muller(wa, wb);
    float z0 = z.x, z1 = z.y;
    if (a.ranged) {
        z0 = __builtin_fmaf(z0, a.sd, a.mean);
        z1 = __builtin_fmaf(z1, a.sd, a.mean);
    }
    a.out[2 * j] = z0;
    if (2 * j + 1 < a.n) a.out[2 * j + 1] = z1;
}

template <int KIND>
hipError_t launch_kind(const PhiloxFill &a, dim3 grid, dim3 block, hipStream_t s)
{
    switch (a.phase) {
    case 0: hipLaunchKernelGGL((philox_fill_kernel<KIND, 0>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((philox_fill_kernel<KIND, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((philox_fill_kernel<KIND, 2>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((philox_fill_kernel<KIND, 3>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_philox_fill(const PhiloxFill &a, hipStream_t s)
{
    const PhiloxTuning &t = philox_tuning();
    const uint32_t waves_per_block = (uint32_t)t.block / 64u;
    const uint64_t waves = ((uint64_t)a.nslots + a.slots_per_wave - 1) / a.slots_per_wave;
    const dim3 grid((uint32_t)((waves + waves_per_block - 1) / waves_per_block));
    const dim3 block((uint32_t)t.block);
    switch (a.kind) {
    case kBits: return launch_kind<kBits>(a, grid, block, s);
    case kU32F: return launch_kind<kU32F>(a, grid, block, s);
    case kU64F: return launch_kind<kU64F>(a, grid, block, s);
    default: return launch_kind<kGauss>(a, grid, block, s);
    }
}

hipError_t launch_philox_pairs(const PhiloxPairs &a, hipStream_t s)
{
    const uint64_t npairs = (a.n + 1) / 2;
    const dim3 grid((uint32_t)((npairs + 255) / 256));
    hipLaunchKernelGGL(philox_pairs_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace mirng
