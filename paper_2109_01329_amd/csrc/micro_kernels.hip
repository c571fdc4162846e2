// Measurement kernels (ceilings for the generation kernels).
#include "internal.hpp"
#include "mirng_bench.h"
#include "transforms.hpp"

namespace mirng {
namespace {

__global__ __launch_bounds__(256) void store_kernel(char *out, uint64_t nvec,
                                                    uint32_t vec_per_wave, int nt)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t v0 = wave * vec_per_wave;
    if (v0 >= nvec) return;
    const uint64_t v1 = v0 + vec_per_wave < nvec ? v0 + vec_per_wave : nvec;
    u32x4 val;
    val.x = 0x3F000000u ^ lane; val.y = (uint32_t)wave; val.z = 0x12345678u; val.w = lane;
    for (uint64_t v = v0 + lane; v < v1; v += 64) {
        u32x4 *p = (u32x4 *)(out + v * 16);
        if (nt) __builtin_nontemporal_store(val, p);
        else *p = val;
    }
}

__device__ __forceinline__ u32x4 philox10_bench(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t rk0 = k0 + (uint32_t)r * kPhiloxW0;
        const uint32_t rk1 = k1 + (uint32_t)r * kPhiloxW1;
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ rk0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ rk1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    u32x4 w;
    w.x = c0; w.y = c1; w.z = c2; w.w = c3;
    return w;
}

__global__ __launch_bounds__(256) void philox_nostore_kernel(uint64_t nblocks,
                                                             uint32_t blk_per_wave,
                                                             uint32_t k0, uint32_t k1,
                                                             uint32_t *sink)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t b0 = wave * blk_per_wave;
    if (b0 >= nblocks) return;
    const uint64_t b1 = b0 + blk_per_wave < nblocks ? b0 + blk_per_wave : nblocks;
    uint32_t acc = 0;
    for (uint64_t b = b0 + lane; b < b1; b += 64) {
        const u32x4 w = philox10_bench((uint32_t)b, (uint32_t)(b >> 32), 0, 0, k0, k1);
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

}  // namespace
}  // namespace mirng

using namespace mirng;

extern "C" {

mirng_status mirng_bench_store(void *out, uint64_t bytes, int32_t nontemporal, void *stream)
{
    if (!out || bytes % 16 || ((uintptr_t)out & 15u)) return MIRNG_E_INVALID_ARG;
    if (bytes == 0) return MIRNG_OK;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    const PhiloxTuning &tu = philox_tuning();
    const uint64_t nvec = bytes / 16;
    const uint64_t waves_target = (uint64_t)device_cu_count() * tu.waves_per_cu;
    uint64_t iters = (nvec + 64 * waves_target - 1) / (64 * waves_target);
    if (iters < 1) iters = 1;
    const uint64_t per_wave = iters * 64;
    const uint64_t waves = (nvec + per_wave - 1) / per_wave;
    const uint64_t groups = (waves + 3) / 4;
    if (groups >= (1ull << 31) || per_wave >= (1ull << 32)) return MIRNG_E_INVALID_ARG;
    hipLaunchKernelGGL(store_kernel, dim3((uint32_t)groups), dim3(256), 0,
                       (hipStream_t)stream, (char *)out, nvec, (uint32_t)per_wave,
                       (int)nontemporal);
    return hipGetLastError() == hipSuccess ? MIRNG_OK : MIRNG_E_LAUNCH;
}

mirng_status mirng_bench_philox_nostore(uint64_t nblocks, uint32_t k0, uint32_t k1,
                                        uint32_t *sink, void *stream)
{
    if (!sink) return MIRNG_E_INVALID_ARG;
    if (nblocks == 0) return MIRNG_OK;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    const PhiloxTuning &tu = philox_tuning();
    const uint64_t waves_target = (uint64_t)device_cu_count() * tu.waves_per_cu;
    uint64_t iters = (nblocks + 64 * waves_target - 1) / (64 * waves_target);
    if (iters < 1) iters = 1;
    const uint64_t per_wave = iters * 64;
    const uint64_t waves = (nblocks + per_wave - 1) / per_wave;
    const uint64_t groups = (waves + 3) / 4;
    if (groups >= (1ull << 31) || per_wave >= (1ull << 32)) return MIRNG_E_INVALID_ARG;
    hipLaunchKernelGGL(philox_nostore_kernel, dim3((uint32_t)groups), dim3(256), 0,
                       (hipStream_t)stream, nblocks, (uint32_t)per_wave, k0, k1, sink);
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
