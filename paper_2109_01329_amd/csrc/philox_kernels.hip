// Philox4x32-10 bulk generation kernels for gfx950.
//
// The engine is the counter-based Philox-4x32 bijection with 10 rounds of
// Salmon et al. (SC'11); the paper measures exactly this generator with
// uniform FP32 output (arXiv:2109.01329, Sec. 7).  Its separate range-
// transform kernel (Sec. 4.3) is fused here into the store epilogue.
//
// Contiguous walk (philox_fill_kernel).  The output is cut
// into 16-byte slots; each wave owns a contiguous run of slots and lane L
// evaluates the Philox block of slot s0 + 64 i + L, so a wave writes 1 KiB
// contiguously per step.  When the engine position is not a multiple of 4
// relative to the 16-byte grid, slot s needs the tail of block b and the
// head of block b + 1: lane L takes those words from lane L + 1 (one DPP
// wavefront shift), and lane 63 from lane 0 of the wave's next step, which
// is computed one step ahead; the extra block per run is 1/steps.  All
// stores stay 16-byte aligned.
//
// Chunked walk (philox_chunk_kernel).  As the contiguous walk, but each
// wave writes only 1, 2 or 4 chunks of 64 slots (63 at odd phases, where
// lane 63 just supplies its block's head to lane 62), evaluated together.
// Many waves of 1-4 KiB keep the in-flight stores on one compact window.
//
// Group walk (philox_group_kernel, the default).  Aligned 64-slot chunks at
// every phase: a workgroup's waves cover consecutive chunks, lane 63 of a
// chunk takes the next chunk's head from LDS, and the group's last wave
// evaluates the one block past the group (see group_chunks below).
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

// ---------------------------------------------------------------- grid-stride walk

// A wave step covers BPL * 64 consecutive blocks (lane L takes c + 64 k + L,
// BPL independent Philox chains per lane); steps are strided by the number
// of waves, so the grid writes one compact window per round of steps.
template <int KIND, int BPL>
__global__ __launch_bounds__(1024) void philox_blocks_kernel(PhiloxBlocks a)
{
    constexpr int EPB = 16 / elem_bytes(KIND);        // elements per block
    constexpr int ESZ = 16 / EPB;
    constexpr uint32_t PER = 64u * BPL;               // blocks per wave step
    if constexpr (uses_lds_tables(KIND)) bm_stage();
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

template <int KIND, int PHASE>
__global__ __launch_bounds__(1024) void philox_fill_kernel(PhiloxFill a)
{
    if constexpr (uses_lds_tables(KIND)) bm_stage();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + lane0(threadIdx.x >> 6);
    const uint64_t first = (uint64_t)wave * a.slots_per_wave;
    if (first >= a.nslots) return;
    const uint32_t s0 = (uint32_t)first;
    const uint32_t span = min(a.slots_per_wave, a.nslots - s0);
    if (has_range_step(KIND) && a.run.ep.ranged)
        walk_slots<KIND, PHASE, 1>(a.run, s0, span, lane);
    else
        walk_slots<KIND, PHASE, 0>(a.run, s0, span, lane);
}

// ---------------------------------------------------------------- chunked walk

template <int KIND, int PHASE, int ITERS>
__global__ __launch_bounds__(1024) void philox_chunk_kernel(PhiloxFill a)
{
    constexpr uint32_t PER = (PHASE ? 63u : 64u) * ITERS;   // slots per wave
    if constexpr (uses_lds_tables(KIND)) bm_stage();
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + lane0(threadIdx.x >> 6);
    const uint64_t first = wave * PER;
    if (first >= a.nslots) return;
    const uint32_t s0 = (uint32_t)first;
    const uint32_t span = min(PER, a.nslots - s0);
    if (has_range_step(KIND) && a.run.ep.ranged)
        walk_chunks<KIND, PHASE, ITERS, 1>(a.run, s0, span, lane);
    else
        walk_chunks<KIND, PHASE, ITERS, 0>(a.run, s0, span, lane);
}

// ---------------------------------------------------------------- group walk

// A group of G waves covers ITERS G consecutive chunks of 64 slots (1 KiB
// each of a 16-byte aligned run), and wave w writes chunks w, G + w, ...,
// so the waves in flight write one compact, moving window at every phase.
// At phases p != 0, slot s needs the tail of block s and the head of block
// s + 1: lanes take it from lane + 1 (DPP), lane 63 from lane 0 of the next
// chunk through LDS, and the group's last wave evaluates the one block past
// the group (so the group evaluates 64 ITERS G + 1 blocks).  Every wave
// reaches the barrier, also past the end of the run, where it stores
// nothing.
template <int KIND, int PHASE, int ITERS, int RANGED, bool NC>
__device__ __forceinline__ void group_chunks(const PhiloxFill &a, u32x4 *heads)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t g0 = blockIdx.x * nw * ITERS * 64u;   // the group's first slot
    const SlotRun &r = a.run;
    // Chunks that lie wholly inside the output store without per-lane
    // checks for the 4-byte kinds; the 8-byte kinds keep the per-lane path,
    // which measured 4-5% faster for them in this walk (and the whole-chunk
    // path 3-5% faster for uniform FP32 at two chunks per wave).
    constexpr bool kWhole = elem_bytes(KIND) == 4;
    u32x4 cur[ITERS];
#pragma unroll
    for (int it = 0; it < ITERS; ++it)
        cur[it] = block_at<NC>(r.base, r.k0, r.k1, g0 + (it * nw + w) * 64u + lane);
    if constexpr (PHASE == 0) {
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const uint32_t cb = g0 + (it * nw + w) * 64u;
            const uint32_t slot = cb + lane;
            if (kWhole && whole_step(r, cb, 0u, a.nslots))
                emit_slot_whole<KIND, RANGED>(r, cb, lane, cur[it]);
            else if (slot < a.nslots) emit_slot<KIND, RANGED>(r, slot, cur[it]);
        }
    } else {
        if (lane == 0) {
#pragma unroll
            for (int it = 0; it < ITERS; ++it) heads[it * nw + w] = cur[it];
        }
        const bool last = w + 1u == nw;
        u32x4 extra = {0u, 0u, 0u, 0u};
        if (last) extra = block_at<NC>(r.base, r.k0, r.k1, g0 + ITERS * nw * 64u);   // uniform
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const uint32_t c = it * nw + w;   // chunk within the group
            u32x4 head = extra;
            if (!last || it + 1 < ITERS) head = heads[c + 1u];
            u32x4 nb;
            nb.x = from_next_lane(cur[it].x, head.x);
            if constexpr (PHASE >= 2) nb.y = from_next_lane(cur[it].y, head.y);
            if constexpr (PHASE >= 3) nb.z = from_next_lane(cur[it].z, head.z);
            const uint32_t cb = g0 + c * 64u;
            const uint32_t slot = cb + lane;
            const u32x4 wv = funnel<PHASE>(cur[it], nb);
            if (kWhole && whole_step(r, cb, 0u, a.nslots))
                emit_slot_whole<KIND, RANGED>(r, cb, lane, wv);
            else if (slot < a.nslots) emit_slot<KIND, RANGED>(r, slot, wv);
        }
    }
}

template <int KIND, int PHASE, int ITERS>
__global__ __launch_bounds__(1024) void philox_group_kernel(PhiloxFill a)
{
    __shared__ u32x4 heads[16 * ITERS + 1];
    if constexpr (uses_lds_tables(KIND)) bm_stage();
    const uint32_t nw = blockDim.x >> 6;
    // the group's blocks, the one past it included (group-uniform choice)
    const uint64_t last = ((uint64_t)blockIdx.x + 1u) * nw * ITERS * 64u;
    const bool nc = no_carry(a.run, last);
    const bool rg = has_range_step(KIND) && a.run.ep.ranged;
    if (nc) {
        if (rg) group_chunks<KIND, PHASE, ITERS, 1, true>(a, heads);
        else group_chunks<KIND, PHASE, ITERS, 0, true>(a, heads);
    } else {
        if (rg) group_chunks<KIND, PHASE, ITERS, 1, false>(a, heads);
        else group_chunks<KIND, PHASE, ITERS, 0, false>(a, heads);
    }
}

template <int KIND, int PHASE>
void launch_group_phase(const PhiloxFill &a, dim3 grid, dim3 block, hipStream_t s)
{
    switch (a.iters) {
    case 1: hipLaunchKernelGGL((philox_group_kernel<KIND, PHASE, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((philox_group_kernel<KIND, PHASE, 2>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((philox_group_kernel<KIND, PHASE, 4>), grid, block, 0, s, a); break;
    }
}

template <int KIND>
hipError_t launch_group_kind(const PhiloxFill &a, dim3 grid, dim3 block, hipStream_t s)
{
    switch (a.phase) {
    case 0: launch_group_phase<KIND, 0>(a, grid, block, s); break;
    case 1: launch_group_phase<KIND, 1>(a, grid, block, s); break;
    case 2: launch_group_phase<KIND, 2>(a, grid, block, s); break;
    default: launch_group_phase<KIND, 3>(a, grid, block, s); break;
    }
    return hipGetLastError();
}

template <int KIND, int PHASE>
void launch_chunk_phase(const PhiloxFill &a, dim3 grid, dim3 block, hipStream_t s)
{
    switch (a.iters) {
    case 4: hipLaunchKernelGGL((philox_chunk_kernel<KIND, PHASE, 4>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((philox_chunk_kernel<KIND, PHASE, 2>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((philox_chunk_kernel<KIND, PHASE, 1>), grid, block, 0, s, a); break;
    }
}

template <int KIND>
hipError_t launch_chunk_kind(const PhiloxFill &a, dim3 grid, dim3 block, hipStream_t s)
{
    switch (a.phase) {
    case 0: launch_chunk_phase<KIND, 0>(a, grid, block, s); break;
    case 1: launch_chunk_phase<KIND, 1>(a, grid, block, s); break;
    case 2: launch_chunk_phase<KIND, 2>(a, grid, block, s); break;
    default: launch_chunk_phase<KIND, 3>(a, grid, block, s); break;
    }
    return hipGetLastError();
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
    case kGauss: return launch_blocks_kind<kGauss>(a, s);
    case kI32: return launch_blocks_kind<kI32>(a, s);
    case kIcdf: return launch_blocks_kind<kIcdf>(a, s);
    case kIcdf64: return launch_blocks_kind<kIcdf64>(a, s);
    default: return hipErrorInvalidValue;   // Gaussian FP64 pairs span whole blocks: fill walk
    }
}

hipError_t launch_philox_fill(const PhiloxFill &a, hipStream_t s)
{
    const uint32_t waves_per_block = a.block / 64u;
    const uint64_t waves = ((uint64_t)a.nslots + a.slots_per_wave - 1) / a.slots_per_wave;
    const dim3 grid((uint32_t)((waves + waves_per_block - 1) / waves_per_block));
    const dim3 block(a.block);
    if (a.group_walk) {
        switch (a.kind) {
        case kBits: return launch_group_kind<kBits>(a, grid, block, s);
        case kU32F: return launch_group_kind<kU32F>(a, grid, block, s);
        case kU64F: return launch_group_kind<kU64F>(a, grid, block, s);
        case kGauss: return launch_group_kind<kGauss>(a, grid, block, s);
        case kGauss64: return launch_group_kind<kGauss64>(a, grid, block, s);
        case kI32: return launch_group_kind<kI32>(a, grid, block, s);
        case kIcdf: return launch_group_kind<kIcdf>(a, grid, block, s);
        case kIcdf64: return launch_group_kind<kIcdf64>(a, grid, block, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (a.iters) {
        switch (a.kind) {
        case kBits: return launch_chunk_kind<kBits>(a, grid, block, s);
        case kU32F: return launch_chunk_kind<kU32F>(a, grid, block, s);
        case kU64F: return launch_chunk_kind<kU64F>(a, grid, block, s);
        case kGauss: return launch_chunk_kind<kGauss>(a, grid, block, s);
        case kGauss64: return launch_chunk_kind<kGauss64>(a, grid, block, s);
        case kI32: return launch_chunk_kind<kI32>(a, grid, block, s);
        case kIcdf: return launch_chunk_kind<kIcdf>(a, grid, block, s);
        case kIcdf64: return launch_chunk_kind<kIcdf64>(a, grid, block, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (a.kind) {
    case kBits: return launch_fill_kind<kBits>(a, grid, block, s);
    case kU32F: return launch_fill_kind<kU32F>(a, grid, block, s);
    case kU64F: return launch_fill_kind<kU64F>(a, grid, block, s);
    case kGauss: return launch_fill_kind<kGauss>(a, grid, block, s);
    case kGauss64: return launch_fill_kind<kGauss64>(a, grid, block, s);
    case kI32: return launch_fill_kind<kI32>(a, grid, block, s);
    case kIcdf: return launch_fill_kind<kIcdf>(a, grid, block, s);
    case kIcdf64: return launch_fill_kind<kIcdf64>(a, grid, block, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mirng
