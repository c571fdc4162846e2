// Allocation-free batched generation.  The device tables of a batch (the
// request table, per-request descriptors, tile and chunk prefixes and the
// wave start table) live in one fixed file-scope device array instead of a
// batcher's allocations; the planning and generation kernels are the
// batcher's own.  Everything runs in order on the caller's stream.
#include <cstring>

#include "internal.hpp"

namespace mirng {
namespace {

constexpr size_t kNaReqs = MIRNG_NOALLOC_MAX_REQUESTS;
constexpr size_t kNaWaves = MIRNG_NOALLOC_MAX_WAVES;
constexpr size_t kNaChunks = (kNaReqs + 1023) / 1024;   // planning chunks of 1024 requests

constexpr size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the tables inside the array, each 256-byte aligned.
constexpr size_t kOffReqs = 0;
constexpr size_t kOffDesc = up256(kOffReqs + kNaReqs * sizeof(mirng_request));
constexpr size_t kOffLocalEnd = up256(kOffDesc + kNaReqs * sizeof(BatchDesc));
constexpr size_t kOffChunkTotal = up256(kOffLocalEnd + 2 * kNaReqs * sizeof(uint64_t));
constexpr size_t kOffChunkEnd = up256(kOffChunkTotal + 2 * kNaChunks * sizeof(uint64_t));
constexpr size_t kOffTotal = up256(kOffChunkEnd + 2 * kNaChunks * sizeof(uint64_t));
constexpr size_t kOffWaveStart = up256(kOffTotal + 2 * sizeof(uint64_t));
constexpr size_t kScratchBytes = up256(kOffWaveStart + kNaWaves * sizeof(uint32_t));

static_assert(kScratchBytes <= MIRNG_NOALLOC_SCRATCH_BYTES,
              "the header's scratch size must cover the table layout");

// One copy per GPU, held until the process ends.  In host code this name
// is a host-side stand-in, not a device address: host code uses the
// per-device address that noalloc_scratch_init looks up.
static __device__ __align__(256) unsigned char scratch[MIRNG_NOALLOC_SCRATCH_BYTES];

unsigned char *g_scratch_dev[kMaxDevices];   // device address of `scratch`, per GPU

}  // namespace

hipError_t noalloc_scratch_init(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    void *p = nullptr;
    const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return err;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = (unsigned char *)p;
    return hipSuccess;
}

}  // namespace mirng

using namespace mirng;

extern "C" mirng_status mirng_generate_batch_noalloc(const mirng_request *reqs, size_t count,
                                                     int32_t *statuses,
                                                     const mirng_batch_config *cfg,
                                                     void *stream)
{
    if (count == 0) return MIRNG_OK;
    if (!reqs || !statuses || ((uintptr_t)statuses & 3u)) return MIRNG_E_INVALID_ARG;
    if (count > kNaReqs) return MIRNG_E_CAPACITY;
    mirng_batch_config c = cfg ? *cfg : batch_default_config();
    const bool block_ok = c.block == 64 || c.block == 128 || c.block == 256 ||
                          c.block == 512 || c.block == 1024;
    if (!block_ok || c.waves_per_cu < 1 || c.waves_per_cu > 4096 ||
        (c.nontemporal != 0 && c.nontemporal != 1) || c.reserved != 0)
        return MIRNG_E_INVALID_ARG;
    int dev = 0;
    if (ensure_device(&dev) != hipSuccess) return MIRNG_E_DEVICE;
    unsigned char *base = g_scratch_dev[dev];
    if (!base) return MIRNG_E_DEVICE;
    MrgBatchTables tabs;
    if (mrg_batch_tables(dev, tabs) != hipSuccess) return MIRNG_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;

    BatchArgs a{};
    batch_grids(c, reqs, count, kNaWaves, a);
    a.reqs = (const mirng_request *)(base + kOffReqs);
    a.refs = nullptr;
    a.engines = nullptr;
    a.count = (uint32_t)count;
    a.nchunks = (uint32_t)((count + 1023) / 1024);
    a.desc = (BatchDesc *)(base + kOffDesc);
    a.local_end = (uint64_t *)(base + kOffLocalEnd);
    a.chunk_total = (uint64_t *)(base + kOffChunkTotal);
    a.chunk_end = (uint64_t *)(base + kOffChunkEnd);
    a.total = (uint64_t *)(base + kOffTotal);
    a.wave_start = (uint32_t *)(base + kOffWaveStart);
    a.status = statuses;
    a.pow2 = tabs.pow2;
    a.c_tab4 = tabs.c_tab4;
    a.u_tab4 = tabs.u_tab4;
    a.c_tab8 = tabs.c_tab8;
    a.u_tab8 = tabs.u_tab8;
    // the request table into the array, then planning and generation, all
    // in stream order (the Philox and MRG generation kernels one after the
    // other); every table the kernels read is written by planning first, so
    // nothing needs clearing
    hipError_t err = hipMemcpyAsync(base + kOffReqs, reqs, count * sizeof(mirng_request),
                                    hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = launch_batch_plan(a, s);
    if (err == hipSuccess) err = launch_batch_generate(a, s);
    return err == hipSuccess ? MIRNG_OK : MIRNG_E_LAUNCH;
}
