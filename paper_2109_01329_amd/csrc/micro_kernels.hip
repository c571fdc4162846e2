// Measurement kernels (ceilings for the generation kernels).
#include "internal.hpp"
#include "philox.hpp"
#include "mirng_bench.h"
#include "transforms.hpp"

namespace mirng {
namespace {

// The two walks of the Philox kernels, stores only.  vpw == 0: grid-stride
// (each wave step covers bpl * 64 consecutive 16-byte vectors, steps strided
// by the number of waves).  vpw > 0: wave w owns vectors [w vpw, (w+1) vpw)
// and writes 64 consecutive vectors per step.
__global__ __launch_bounds__(1024) void store_kernel(char *out, uint64_t nvec, int nt, int bpl,
                                                     uint32_t vpw)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    u32x4 val;
    val.x = 0x3F000000u ^ lane; val.y = (uint32_t)wave; val.z = 0x12345678u; val.w = lane;
    uint64_t first, last, stride;
    const uint64_t per = vpw ? 64ull : 64ull * bpl;
    if (vpw) {
        first = wave * vpw;
        last = first + vpw < nvec ? first + vpw : nvec;
        stride = 64;
    } else {
        first = wave * per;
        last = nvec;
        stride = waves * per;
    }
    for (uint64_t c = first; c < last; c += stride) {
        for (uint64_t k = 0; k < per; k += 64) {
            const uint64_t v = c + k + lane;
            if (v < last) {
                u32x4 *q = (u32x4 *)(out + v * 16);
                if (nt) __builtin_nontemporal_store(val, q);
                else *q = val;
            }
        }
    }
}

__global__ __launch_bounds__(1024) void philox_nostore_kernel(uint64_t nblocks, uint32_t k0,
                                                              uint32_t k1, uint32_t *sink)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    uint32_t acc = 0;
    for (uint64_t b = wave * 64 + lane; b < nblocks; b += waves * 64) {
        const u32x4 w = philox10((uint32_t)b, (uint32_t)(b >> 32), 0, 0, k0, k1);
        acc ^= w.x ^ w.y ^ w.z ^ w.w;
    }
    // fold across the wave so only one word per wave is written
    for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off);
    if (lane == 0) sink[wave] = acc;
}

template <int OP>
__global__ __launch_bounds__(256) void valu_kernel(uint32_t iters, uint32_t *sink)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (OP == 0) {
        uint64_t a[8];
        uint32_t m = 0xD2511F53u ^ tid;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = tid * 8u + j;
        for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (uint64_t)m * (uint32_t)a[j] + (a[j] >> 32);
        }
        uint64_t x = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) x ^= a[j];
        sink[tid] = (uint32_t)x ^ (uint32_t)(x >> 32);
    } else if constexpr (OP == 1) {
        uint32_t a[8];
        const uint32_t k = 0x9E3779B9u * (tid + 1);
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = tid + j;
        for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = a[j] ^ a[(j + 1) & 7] ^ (k + i);
        }
        uint32_t x = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) x ^= a[j];
        sink[tid] = x;
    } else if constexpr (OP == 2 || OP == 3) {
        double a[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = 1.0 + (tid & 7) * 1e-3 + j;
        for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if constexpr (OP == 2) a[j] = __builtin_fma(a[j], 0.999999, 1e-7);
                else a[j] = __builtin_floor(a[j] * 1.0000001) + 0.5;
            }
        }
        double x = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) x += a[j];
        sink[tid] = (uint32_t)x;
    } else {
        float a[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = 1.0f + (tid & 7) * 1e-3f + j;
        for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = __builtin_fmaf(a[j], 0.999999f, 1e-7f);
        }
        float x = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) x += a[j];
        sink[tid] = (uint32_t)x;
    }
}

// One FP32-transform piece per thread (see mirng_bench_transform_f32).
__global__ __launch_bounds__(256) void transform_probe_kernel(int32_t which, uint32_t first,
                                                              uint32_t n, void *out)
{
    bm_stage();
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n) return;
    const uint32_t w = (first + i) << 8;
    if (which == 0) {
        ((double *)out)[i] = 0.5 * bm_radius2(w);                 // exact halving
    } else if (which == 1) {
        const f64x2 cs = bm_unit_half(w);
        ((double *)out)[2 * (size_t)i] = 2.0 * cs.x;             // exact doubling
        ((double *)out)[2 * (size_t)i + 1] = 2.0 * cs.y;
    } else {
        ((float *)out)[i] = icdf_f32(w);
    }
}

}  // namespace
}  // namespace mirng

using namespace mirng;

extern "C" {

// Persistent grid of the grid-stride Philox kernel for `units` 16-byte units.
static uint64_t grid_for(uint64_t units, const mirng_philox_config &tu)
{
    const uint64_t wpb = (uint64_t)tu.block / 64;
    const uint64_t steps = (units + 64ull * tu.blocks_per_lane - 1) / (64ull * tu.blocks_per_lane);
    const uint64_t want = ((uint64_t)device_cu_count() * tu.waves_per_cu + wpb - 1) / wpb;
    const uint64_t need = (steps + wpb - 1) / wpb;
    return want < need ? want : need;
}

mirng_status mirng_bench_store(void *out, uint64_t bytes, int32_t nontemporal, void *stream)
{
    if (!out || bytes % 16 || ((uintptr_t)out & 15u)) return MIRNG_E_INVALID_ARG;
    if (bytes == 0) return MIRNG_OK;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    const mirng_philox_config tu = philox_config();
    const uint64_t nvec = bytes / 16;
    uint64_t groups;
    uint32_t vpw = 0;
    if (tu.walk == 0 || tu.walk == 2 || tu.walk == 3) {
        // the store pattern of the installed walk: contiguous runs (0), or
        // runs of 1, 2 or 4 chunks (2) or one chunk (3) of 64 vectors
        const uint64_t waves_target = (uint64_t)device_cu_count() * tu.waves_per_cu;
        const uint64_t iters = (nvec + 64 * waves_target - 1) / (64 * waves_target);
        const uint64_t per_wave = tu.walk == 3   ? 64ull
                                  : tu.walk == 2 ? 64ull * tu.blocks_per_lane
                                                 : (iters ? iters : 1) * 64;
        if (per_wave >= (1ull << 32)) return MIRNG_E_INVALID_ARG;
        vpw = (uint32_t)per_wave;
        const uint64_t waves = (nvec + per_wave - 1) / per_wave;
        const uint64_t wpb = (uint64_t)tu.block / 64;
        groups = (waves + wpb - 1) / wpb;
    } else {
        groups = grid_for(nvec, tu);
    }
    if (groups >= (1ull << 31)) return MIRNG_E_INVALID_ARG;
    hipLaunchKernelGGL(store_kernel, dim3((uint32_t)groups), dim3(tu.block), 0,
                       (hipStream_t)stream, (char *)out, nvec, (int)nontemporal,
                       (int)tu.blocks_per_lane, vpw);
    return hipGetLastError() == hipSuccess ? MIRNG_OK : MIRNG_E_LAUNCH;
}

mirng_status mirng_bench_philox_nostore(uint64_t nblocks, uint32_t k0, uint32_t k1,
                                        uint32_t *sink, void *stream)
{
    if (!sink) return MIRNG_E_INVALID_ARG;
    if (nblocks == 0) return MIRNG_OK;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    mirng_philox_config tu = philox_config();
    tu.blocks_per_lane = 1;
    tu.waves_per_cu = 32;   // a full complement of resident waves, whatever the walk
    hipLaunchKernelGGL(philox_nostore_kernel, dim3((uint32_t)grid_for(nblocks, tu)),
                       dim3(tu.block), 0, (hipStream_t)stream, nblocks, k0, k1, sink);
    return hipGetLastError() == hipSuccess ? MIRNG_OK : MIRNG_E_LAUNCH;
}

mirng_status mirng_bench_transform_f32(int32_t which, uint32_t first, uint32_t n, void *out,
                                       void *stream)
{
    if (which < 0 || which > 2) return MIRNG_E_UNSUPPORTED;
    if (n == 0) return MIRNG_OK;
    if (!out || (uint64_t)first + n > (1ull << 24)) return MIRNG_E_INVALID_ARG;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    hipLaunchKernelGGL(transform_probe_kernel, dim3((n + 255u) / 256u), dim3(256), 0,
                       (hipStream_t)stream, which, first, n, out);
    return hipGetLastError() == hipSuccess ? MIRNG_OK : MIRNG_E_LAUNCH;
}

mirng_status mirng_bench_valu(int32_t op, uint32_t threads, uint32_t iters, uint32_t *sink,
                              void *stream)
{
    if (!sink || threads == 0 || threads % 256) return MIRNG_E_INVALID_ARG;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    const dim3 grid(threads / 256), block(256);
    hipStream_t s = (hipStream_t)stream;
    switch (op) {
    case 0: hipLaunchKernelGGL(valu_kernel<0>, grid, block, 0, s, iters, sink); break;
    case 1: hipLaunchKernelGGL(valu_kernel<1>, grid, block, 0, s, iters, sink); break;
    case 2: hipLaunchKernelGGL(valu_kernel<2>, grid, block, 0, s, iters, sink); break;
    case 3: hipLaunchKernelGGL(valu_kernel<3>, grid, block, 0, s, iters, sink); break;
    case 4: hipLaunchKernelGGL(valu_kernel<4>, grid, block, 0, s, iters, sink); break;
    default: return MIRNG_E_UNSUPPORTED;
    }
    return hipGetLastError() == hipSuccess ? MIRNG_OK : MIRNG_E_LAUNCH;
}

}  // extern "C"
