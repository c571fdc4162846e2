// Philox4x32-10 bulk generation kernels for gfx950.
//
// The engine is the counter-based Philox-4x32 bijection with 10 rounds of
// Salmon et al. (SC'11); the paper measures exactly this generator with
// uniform FP32 output (arXiv:2109.01329, Sec. 6).  Its separate range-
// transform kernel (Sec. 4.3) is fused here into the store epilogue.
//
// Contiguous walk (philox_fill_kernel, the default).  The output is cut
// into 16-byte slots; each wave owns a contiguous run of slots and lane L
// evaluates the Philox block of slot s0 + 64 i + L, so a wave writes 1 KiB
// contiguously per step.  When the engine position is not a multiple of 4
// relative to the 16-byte grid, slot s needs the tail of block b and the
// head of block b + 1: lane L takes those words from lane L + 1
// (ds_bpermute), and lane 63 from lane 0 of the wave's next step, which is
// computed one step ahead; the extra block per run is 1/steps.  All stores
// stay 16-byte aligned.
//
// Grid-stride walk (philox_blocks_kernel, selectable).  Whenever outputs do
// not straddle Philox blocks (bits and uniform FP32 at any position; FP64
// and Gaussian pairs at even positions) every block is 16 bytes of output
// at its element address.  A small persistent grid walks the blocks so that
// the whole GPU writes one compact moving window; a block is written with
// one 16-byte store at a possibly only 4-byte-aligned address (gfx950
// accepts dword-aligned vector stores).  No data moves between lanes.
//
// On MI355X the contiguous walk with many short-lived waves sustains the
// higher write rate once the Philox rounds are in the loop, and 16-byte
// stores at addresses that are only 4-byte aligned cost about a fifth of
// the write bandwidth (measurements in the design notes); the grid-stride
// walk is kept for the autotuner.
#include "internal.hpp"
#include "philox.hpp"
#include "transforms.hpp"

namespace mirng {
namespace {

// 16 bytes at a 4-byte-aligned address (one global_store_dwordx4 on gfx950).
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

// ---------------------------------------------------------------- engine

// Four words -> the 16 bytes they become.
template <int KIND>
__device__ __forceinline__ u32x4 transform(const Epilogue &ep, u32x4 w)
{
    u32x4 v;
    if constexpr (KIND == kBits) {
        v = w;
    } else if constexpr (KIND == kU32F) {
        f32x4 f;
        f.x = u01f(w.x); f.y = u01f(w.y); f.z = u01f(w.z); f.w = u01f(w.w);
        if (ep.ranged) {
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
        if (ep.ranged) {
            d.x = __builtin_fma(d.x, ep.d64, ep.a64);
            d.y = __builtin_fma(d.y, ep.d64, ep.a64);
        }
        v = __builtin_bit_cast(u32x4, d);
    } else {
        f32x4 f;
        f.xy = box_muller(w.x, w.y);
        f.zw = box_muller(w.z, w.w);
        if (ep.ranged) {
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
    constexpr int EPV = (KIND == kU64F) ? 2 : 4;
    constexpr int ESZ = 16 / EPV;
    if (u - full_lo < full_count) {
        if (nt) __builtin_nontemporal_store(v, (u32x4_a4 *)p);
        else *(u32x4_a4 *)p = v;
        return;
    }
#pragma unroll
    for (int j = 0; j < EPV; ++j) {
        const int64_t e = e0 + j;
        if (e >= 0 && e < (int64_t)n) {
            if constexpr (ESZ == 4) {
                ((uint32_t *)p)[j] = v[j];
            } else {
                ((uint64_t *)p)[j] = ((uint64_t)v[2 * j + 1] << 32) | v[2 * j];
            }
        }
    }
}

// ---------------------------------------------------------------- grid-stride walk

// A wave step covers BPL * 64 consecutive blocks (lane L takes c + 64 k + L,
// BPL independent Philox chains per lane); steps are strided by the number
// of waves, so the grid writes one compact window per round of steps.
template <int KIND, int BPL>
__global__ __launch_bounds__(1024) void philox_blocks_kernel(PhiloxBlocks a)
{
    constexpr int EPB = (KIND == kU64F) ? 2 : 4;      // elements per block
    constexpr int ESZ = 16 / EPB;
    constexpr uint32_t PER = 64u * BPL;               // blocks per wave step
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    for (uint64_t c = wave * PER; c < a.nblocks; c += waves * PER) {
        u32x4 w[BPL];
#pragma unroll
        for (int k = 0; k < BPL; ++k)
            w[k] = block_at(a.base, a.k0, a.k1, (uint32_t)c + k * 64u + lane);
#pragma unroll
        for (int k = 0; k < BPL; ++k) {
            const uint64_t j = c + k * 64u + lane;
            if (j < a.nblocks) {
                const int64_t e0 = (int64_t)j * EPB - (int64_t)a.head;
                put<KIND>(a.out + e0 * ESZ, transform<KIND>(a.ep, w[k]), (uint32_t)j, a.full_lo,
                          a.full_count, e0, a.n, a.ep.nt);
            }
        }
    }
}

// ---------------------------------------------------------------- contiguous walk

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

template <int KIND>
__device__ __forceinline__ void emit_slot(const PhiloxFill &a, uint32_t slot, u32x4 w)
{
    constexpr int EPV = (KIND == kU64F) ? 2 : 4;
    const int64_t e0 = (int64_t)slot * EPV - (int64_t)a.head;
    put<KIND>(a.out_base + (uint64_t)slot * 16u, transform<KIND>(a.ep, w), slot, a.full_lo,
              a.full_count, e0, a.n, a.ep.nt);
}

template <int KIND, int PHASE>
__global__ __launch_bounds__(1024) void philox_fill_kernel(PhiloxFill a)
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
            const u32x4 w = block_at(a.base, a.k0, a.k1, slot);
            if (slot - s0 < span) emit_slot<KIND>(a, slot, w);
        }
    } else {
        const int next_addr = (int)(((lane + 1u) & 63u) << 2);
        u32x4 cur = block_at(a.base, a.k0, a.k1, s0 + lane);
        for (uint32_t it = 0; it < iters; ++it) {
            const uint32_t slot = s0 + (it << 6) + lane;
            const u32x4 nxt = block_at(a.base, a.k0, a.k1, slot + 64u);
            // lane 0 offers its next-iteration block, which lane 63 needs
            const u32x4 src = (lane == 0) ? nxt : cur;
            u32x4 nb;
            nb.x = lane_pull(next_addr, src.x);
            if constexpr (PHASE >= 2) nb.y = lane_pull(next_addr, src.y);
            if constexpr (PHASE >= 3) nb.z = lane_pull(next_addr, src.z);
            if (slot - s0 < span) emit_slot<KIND>(a, slot, funnel<PHASE>(cur, nb));
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
    const uint32_t base[4] = {(uint32_t)b_lo, (uint32_t)(b_lo >> 32), (uint32_t)b_hi,
                              (uint32_t)(b_hi >> 32)};
    const uint32_t lane = (uint32_t)(lo & 3u);
    const u32x4 w0 = block_at(base, a.k0, a.k1, 0);
    uint32_t wa, wb;
    if (lane < 3) {
        wa = w0[lane];
        wb = w0[lane + 1];
    } else {
        wa = w0.w;
        wb = block_at(base, a.k0, a.k1, 1).x;
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
hipError_t launch_blocks_kind(const PhiloxBlocks &a, hipStream_t s)
{
    const dim3 grid(a.groups), block(a.block);
    switch (a.bpl) {
    case 4: hipLaunchKernelGGL((philox_blocks_kernel<KIND, 4>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((philox_blocks_kernel<KIND, 2>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((philox_blocks_kernel<KIND, 1>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_fill_kind(const PhiloxFill &a, dim3 grid, dim3 block, hipStream_t s)
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

hipError_t launch_philox_blocks(const PhiloxBlocks &a, hipStream_t s)
{
    switch (a.kind) {
    case kBits: return launch_blocks_kind<kBits>(a, s);
    case kU32F: return launch_blocks_kind<kU32F>(a, s);
    case kU64F: return launch_blocks_kind<kU64F>(a, s);
    default: return launch_blocks_kind<kGauss>(a, s);
    }
}

hipError_t launch_philox_fill(const PhiloxFill &a, hipStream_t s)
{
    const uint32_t waves_per_block = a.block / 64u;
    const uint64_t waves = ((uint64_t)a.nslots + a.slots_per_wave - 1) / a.slots_per_wave;
    const dim3 grid((uint32_t)((waves + waves_per_block - 1) / waves_per_block));
    const dim3 block(a.block);
    switch (a.kind) {
    case kBits: return launch_fill_kind<kBits>(a, grid, block, s);
    case kU32F: return launch_fill_kind<kU32F>(a, grid, block, s);
    case kU64F: return launch_fill_kind<kU64F>(a, grid, block, s);
    default: return launch_fill_kind<kGauss>(a, grid, block, s);
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
