// Batcher: host side of batched generation.  A ring of staging slots, each
// with a pinned request table, device tables and completion events, so
// that successive batches (on one or several streams) overlap without the
// host waiting, except when a slot is reused while the device still needs
// it.  Per batch the host copies the request table into pinned memory (or
// not at all when the caller filled the staged slot) and enqueues on the
// batcher's own stream the upload, the planning kernel (and the scan kernel
// past 64 chunks) and the copy of the per-request statuses back to pinned
// memory; these overlap the generation of earlier batches.  The caller's
// stream waits for them and runs the generation kernels (Philox, MRG32k3a)
// that have work; with both, the MRG kernel runs on a side stream beside
// the Philox kernel and the caller's stream joins it.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.hpp"

namespace {

constexpr int kSlots = 4;
constexpr size_t kChunk = 1024;
constexpr uint64_t kMrgChunksPerGroup = 8;   // MRG chunks per group in large batches
constexpr uint64_t kMaxMrgGroups = 1u << 24;

struct Slot {
    mirng_request *h_reqs = nullptr;   // pinned
    mirng::EngineRef *h_refs = nullptr;  // pinned (engine references of server batches)
    int32_t *h_status = nullptr;       // pinned
    size_t cap = 0;
    size_t count = 0;
    int dev = -1;
    bool pending = false;              // `done` recorded and maybe not reached
    hipEvent_t done = nullptr;
    hipEvent_t planned = nullptr;      // upload, planning and status copy done
    hipEvent_t forked = nullptr;       // the caller's stream up to this batch's generation
    hipEvent_t mrg_done = nullptr;     // MRG generation done (its own stream)
    mirng_request *d_reqs = nullptr;
    mirng::EngineRef *d_refs = nullptr;
    mirng::BatchDesc *d_desc = nullptr;
    uint64_t *d_local_end = nullptr;
    uint64_t *d_chunk_total = nullptr;
    uint64_t *d_chunk_end = nullptr;
    uint64_t *d_total = nullptr;
    int32_t *d_status = nullptr;
    uint32_t *d_wave_start = nullptr;  // [wave_cap]
    size_t wave_cap = 0;
};

// Resident workgroups of the MRG generation kernel: its 36 KiB of LDS per
// group let four groups share a CU.
uint64_t mrg_groups()
{
    return (uint64_t)mirng::device_cu_count() * 4;
}

void release(Slot &s)
{
    if (s.done && s.pending) (void)hipEventSynchronize(s.done);
    if (s.h_reqs) (void)hipHostFree(s.h_reqs);
    if (s.h_refs) (void)hipHostFree(s.h_refs);
    if (s.h_status) (void)hipHostFree(s.h_status);
    if (s.d_reqs) (void)hipFree(s.d_reqs);
    if (s.d_refs) (void)hipFree(s.d_refs);
    if (s.d_desc) (void)hipFree(s.d_desc);
    if (s.d_local_end) (void)hipFree(s.d_local_end);
    if (s.d_chunk_total) (void)hipFree(s.d_chunk_total);
    if (s.d_chunk_end) (void)hipFree(s.d_chunk_end);
    if (s.d_total) (void)hipFree(s.d_total);
    if (s.d_status) (void)hipFree(s.d_status);
    if (s.d_wave_start) (void)hipFree(s.d_wave_start);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.planned) (void)hipEventDestroy(s.planned);
    if (s.mrg_done) (void)hipEventDestroy(s.mrg_done);
    if (s.forked) (void)hipEventDestroy(s.forked);
    s = Slot{};
}

// Room for the start table of `waves` Philox waves in a slot that the
// device no longer uses (after prepare).
hipError_t ensure_waves(Slot &s, size_t waves)
{
    if (s.wave_cap >= waves) return hipSuccess;
    if (s.d_wave_start) (void)hipFree(s.d_wave_start);
    s.d_wave_start = nullptr;
    s.wave_cap = 0;
    hipError_t err = hipMalloc((void **)&s.d_wave_start, waves * sizeof(uint32_t));
    if (err == hipSuccess) s.wave_cap = waves;
    return err;
}

// Waits until the device no longer uses the slot, then makes room for
// `count` requests on device `dev`.
hipError_t prepare(Slot &s, size_t count, int dev)
{
    if (s.pending) {
        hipError_t err = hipEventSynchronize(s.done);
        if (err != hipSuccess) return err;
        s.pending = false;
    }
    if (s.cap >= count && s.dev == dev) return hipSuccess;
    release(s);
    size_t cap = count < 1024 ? 1024 : count;
    const size_t nchunks = (cap + kChunk - 1) / kChunk;
    hipError_t err = hipSuccess;
    auto chk = [&](hipError_t e) { if (err == hipSuccess) err = e; };
    chk(hipHostMalloc((void **)&s.h_reqs, cap * sizeof(mirng_request), hipHostMallocDefault));
    chk(hipHostMalloc((void **)&s.h_refs, cap * sizeof(mirng::EngineRef), hipHostMallocDefault));
    chk(hipHostMalloc((void **)&s.h_status, cap * sizeof(int32_t), hipHostMallocDefault));
    chk(hipMalloc((void **)&s.d_reqs, cap * sizeof(mirng_request)));
    chk(hipMalloc((void **)&s.d_refs, cap * sizeof(mirng::EngineRef)));
    chk(hipMalloc((void **)&s.d_desc, cap * sizeof(mirng::BatchDesc)));
    chk(hipMalloc((void **)&s.d_local_end, 2 * cap * sizeof(uint64_t)));
    chk(hipMalloc((void **)&s.d_chunk_total, 2 * nchunks * sizeof(uint64_t)));
    chk(hipMalloc((void **)&s.d_chunk_end, 2 * nchunks * sizeof(uint64_t)));
    chk(hipMalloc((void **)&s.d_total, 2 * sizeof(uint64_t)));
    chk(hipMalloc((void **)&s.d_status, cap * sizeof(int32_t)));
    chk(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
    chk(hipEventCreateWithFlags(&s.planned, hipEventDisableTiming));
    chk(hipEventCreateWithFlags(&s.mrg_done, hipEventDisableTiming));
    chk(hipEventCreateWithFlags(&s.forked, hipEventDisableTiming));
    if (err != hipSuccess) {
        release(s);
        return err;
    }
    s.cap = cap;
    s.dev = dev;
    return hipSuccess;
}

// What a batch holds, from one pass over its requests: upper bounds on its
// Philox tiles and MRG chunks (the device planning finds the exact counts;
// these only size the generation grids) and which generation kernels can
// have work.
struct Work {
    uint64_t tiles = 0, chunks = 0;
    int32_t philox = 0, mrg = 0;
    int32_t wide = 0;   // a Philox request only the wide kernel holds
    int32_t mrg_wide = 0;   // an MRG request only the wide MRG kernel holds
    int32_t bm = 0;         // a request whose transform reads the LDS tables (either engine)
};

// One pass over a request table: the Work it holds, and (copy != null) its
// copy into `copy` on the way (the generate path's pinned staging).
// Branch-light: every request costs the same few operations.
Work scan_requests(const mirng_request *q, size_t count, mirng_request *copy = nullptr)
{
    uint64_t m = 0;   // kind bits (kind & 15): Philox at 0..15, MRG at 16..31, other at 32..47
    uint64_t tiles = 0, chunks = 0;
    for (size_t i = 0; i < count; ++i) {
        mirng_request r;
        std::memcpy(&r, q + i, sizeof r);
        if (copy) std::memcpy(copy + i, &r, sizeof r);
        const uint32_t k = (uint32_t)r.dist.kind & 15u;
        const bool ph = r.engine_type == MIRNG_PHILOX4X32_10;
        const bool mg = r.engine_type == MIRNG_MRG32K3A;
        m |= (uint64_t)1 << (k + (ph ? 0u : mg ? 16u : 32u));
        const uint64_t n = r.n;
        const bool ok = n - 1u < (1ull << 32) - 1u;             // 0 < n < 2^32
        const bool f64 = ((1u << MIRNG_UNIFORM_F64 | 1u << MIRNG_GAUSSIAN_F64 |
                           1u << MIRNG_GAUSSIAN_ICDF_F64) >> k) & 1u;
        // MRG: chunks of 256 threads x kBatchMrgPasses passes of L outputs
        const uint64_t per_log2 = 8 + 1 + (f64 ? 4 : 5);
        static_assert(mirng::kBatchMrgPasses == 2, "chunk size");
        chunks += (ok && mg) ? (n + ((uint64_t)1 << per_log2) - 1) >> per_log2 : 0;
        // Philox: 16-byte units of n outputs plus the head and its slack
        const uint64_t units = ((n << (f64 ? 1 : 0)) + 3) / 4 + 2;
        tiles += (ok && ph) ? (units + 63) / 64 + 1 : 0;
    }
    Work w;
    w.tiles = tiles;
    w.chunks = chunks;
    w.philox = (m & 0xFFFFull) != 0;
    w.mrg = (m & 0xFFFF0000ull) != 0;
    // Philox kinds whose transforms need many registers (FP64 Box-Muller,
    // the inverse-CDF Gaussians) live in a separate generation kernel
    const uint64_t wide = 1u << MIRNG_GAUSSIAN_F64 | 1u << MIRNG_GAUSSIAN_ICDF_F32 |
                          1u << MIRNG_GAUSSIAN_ICDF_F64;
    w.wide = (m & wide) != 0;
    w.mrg_wide = ((m >> 16) & (1u << MIRNG_GAUSSIAN_ICDF_F32 | 1u << MIRNG_GAUSSIAN_ICDF_F64)) != 0;
    uint64_t lds = 0;
    for (uint32_t kk = 0; kk < 16; ++kk)
        if (mirng::uses_lds_tables((int)kk)) lds |= (uint64_t)1 << kk;
    w.bm = (m & (lds | lds << 16 | lds << 32)) != 0;
    return w;
}

bool config_valid(const mirng_batch_config &c)
{
    const bool block_ok = c.block == 64 || c.block == 128 || c.block == 256 ||
                          c.block == 512 || c.block == 1024;
    return block_ok && c.waves_per_cu >= 1 && c.waves_per_cu <= 4096 &&
           (c.nontemporal == 0 || c.nontemporal == 1) && c.reserved == 0;
}

}  // namespace

struct mirng_batcher_s {
    std::mutex mu;
    Slot slots[kSlots];
    hipStream_t copy = nullptr;        // uploads and planning (default priority)
    hipStream_t side = nullptr;        // MRG generation beside Philox (default priority)
    int copy_dev = -1;
    int next = 0;
    int last = -1;     // slot of the most recent batch
    int staged = -1;   // slot handed out by mirng_batcher_stage
    mirng_batch_config cfg = mirng::batch_default_config();
};

namespace mirng {

mirng_batch_config batch_default_config()
{
    // the shape the autotuner picked for the calorimeter batch on MI355X
    // (512-thread groups, 128 waves of work per CU, ordinary stores)
    return mirng_batch_config{512, 128, 0, 0};
}

size_t grid_waves(const mirng_batch_config &c)
{
    const size_t wpb = (size_t)c.block / 64;
    const size_t w = (size_t)device_cu_count() * (size_t)c.waves_per_cu;
    return (w + wpb - 1) / wpb * wpb;
}

namespace {

void grids_of(const mirng_batch_config &cfg, const Work &w, uint64_t max_waves, BatchArgs &a)
{
    const uint64_t wpb = (uint64_t)cfg.block / 64;
    uint64_t waves = grid_waves(cfg);
    // Philox: no more waves than about two tiles of work each
    const uint64_t want = ((w.tiles + 1) / 2 + wpb - 1) / wpb * wpb;
    waves = std::max<uint64_t>(wpb, std::min(waves, want));
    if (max_waves) waves = std::min(waves, max_waves / wpb * wpb);
    // MRG: a chunk per group while that fills the resident groups, then
    // kMrgChunksPerGroup per group.  Chunks of different kinds cost
    // different times; many short groups let the hardware dispatcher
    // balance them where a few long ones would wait on the slowest.
    const uint64_t resident = mrg_groups();
    const uint64_t mgroups = std::min<uint64_t>(
        kMaxMrgGroups,
        std::max<uint64_t>(1, std::max(std::min(w.chunks, resident),
                                       (w.chunks + kMrgChunksPerGroup - 1) / kMrgChunksPerGroup)));
    a.waves = (uint32_t)waves;
    a.mgroups = (uint32_t)mgroups;
    a.nt = cfg.nontemporal;
    a.wide = w.wide;
    a.philox = w.philox;
    a.mrg = w.mrg;
    a.mrg_wide = w.mrg_wide;
    a.bm = w.bm;
    a.block = (uint32_t)cfg.block;
    a.groups = (uint32_t)(waves / wpb);
}

}  // namespace

void batch_grids(const mirng_batch_config &cfg, const mirng_request *reqs, size_t count,
                 uint64_t max_waves, BatchArgs &a)
{
    grids_of(cfg, scan_requests(reqs, count), max_waves, a);
}

hipError_t batcher_reserve(mirng_batcher b, size_t count)
{
    int dev = 0;
    hipError_t err = ensure_device(&dev);
    if (err != hipSuccess) return err;
    MrgBatchTables tabs;
    err = mrg_batch_tables(dev, tabs);
    if (err != hipSuccess) return err;
    std::lock_guard<std::mutex> lk(b->mu);
    for (Slot &s : b->slots) {
        err = prepare(s, count, dev);
        if (err == hipSuccess) err = ensure_waves(s, grid_waves(b->cfg));
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace mirng

using namespace mirng;

extern "C" {

mirng_status mirng_batcher_create(mirng_batcher *out)
{
    if (!out) return MIRNG_E_INVALID_ARG;
    mirng_batcher b = new (std::nothrow) mirng_batcher_s();
    if (!b) return MIRNG_E_ALLOC;
    *out = b;
    return MIRNG_OK;
}

mirng_status mirng_batcher_destroy(mirng_batcher b)
{
    if (!b) return MIRNG_OK;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        for (Slot &s : b->slots) release(s);
        if (b->copy) (void)hipStreamDestroy(b->copy);
        if (b->side) (void)hipStreamDestroy(b->side);
    }
    delete b;
    return MIRNG_OK;
}

mirng_status mirng_batcher_config_get(mirng_batcher b, mirng_batch_config *c)
{
    if (!b || !c) return MIRNG_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(b->mu);
    *c = b->cfg;
    return MIRNG_OK;
}

mirng_status mirng_batcher_config_set(mirng_batcher b, const mirng_batch_config *c)
{
    if (!b || !c || !config_valid(*c)) return MIRNG_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(b->mu);
    b->cfg = *c;
    return MIRNG_OK;
}


mirng_status mirng_batcher_stage(mirng_batcher b, size_t count, mirng_request **reqs)
{
    if (!b || !reqs) return MIRNG_E_INVALID_ARG;
    if (count >= (1ull << 31)) return MIRNG_E_INVALID_ARG;
    int dev = 0;
    if (ensure_device(&dev) != hipSuccess) return MIRNG_E_DEVICE;
    std::lock_guard<std::mutex> lk(b->mu);
    const int k = b->next;
    if (prepare(b->slots[k], count, dev) != hipSuccess) return MIRNG_E_ALLOC;
    b->next = (k + 1) % kSlots;
    b->staged = k;
    *reqs = b->slots[k].h_reqs;
    return MIRNG_OK;
}

mirng_status mirng_generate_batch(mirng_batcher b, const mirng_request *reqs, size_t count,
                                  void *stream)
{
    return generate_batch_refs(b, reqs, nullptr, count, nullptr, (hipStream_t)stream);
}

}  // extern "C"

mirng_status mirng::generate_batch_refs(mirng_batcher b, const mirng_request *reqs,
                                        const EngineRef *refs, size_t count,
                                        const mirng_state *engines, hipStream_t stream)
{
    if (!b || !reqs) return MIRNG_E_INVALID_ARG;
    if (count >= (1ull << 31)) return MIRNG_E_INVALID_ARG;
    if (count == 0) return MIRNG_OK;
    int dev = 0;
    if (ensure_device(&dev) != hipSuccess) return MIRNG_E_DEVICE;
    hipStream_t s = stream;
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->copy_dev != dev) {
        if (b->copy) (void)hipStreamDestroy(b->copy);
        if (b->side) (void)hipStreamDestroy(b->side);
        b->copy = nullptr;
        b->side = nullptr;
        b->copy_dev = -1;
        if (hipStreamCreateWithFlags(&b->copy, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess)
            return MIRNG_E_DEVICE;
        b->copy_dev = dev;
    }
    MrgBatchTables tabs;
    if (mrg_batch_tables(dev, tabs) != hipSuccess) return MIRNG_E_DEVICE;
    BatchArgs a{};
    int k;
    Work w;
    if (b->staged >= 0 && reqs == b->slots[b->staged].h_reqs &&
        count <= b->slots[b->staged].cap && b->slots[b->staged].dev == dev) {
        k = b->staged;                                   // filled in place
        if (prepare(b->slots[k], count, dev) != hipSuccess) return MIRNG_E_ALLOC;
        w = scan_requests(reqs, count);
    } else {
        k = b->next;
        if (prepare(b->slots[k], count, dev) != hipSuccess) return MIRNG_E_ALLOC;
        b->next = (k + 1) % kSlots;
        w = scan_requests(reqs, count, b->slots[k].h_reqs);   // copy and scan, one pass
    }
    grids_of(b->cfg, w, 0, a);
    b->staged = -1;
    Slot &sl = b->slots[k];
    if (refs) std::memcpy(sl.h_refs, refs, count * sizeof(EngineRef));
    sl.count = count;
    if (ensure_waves(sl, a.waves) != hipSuccess) return MIRNG_E_ALLOC;
    a.reqs = sl.d_reqs;
    a.refs = refs ? sl.d_refs : nullptr;
    a.engines = refs ? engines : nullptr;
    a.count = (uint32_t)count;
    a.nchunks = (uint32_t)((count + kChunk - 1) / kChunk);
    a.desc = sl.d_desc;
    a.local_end = sl.d_local_end;
    a.chunk_total = sl.d_chunk_total;
    a.chunk_end = sl.d_chunk_end;
    a.total = sl.d_total;
    a.wave_start = sl.d_wave_start;
    a.pow2 = tabs.pow2;
    a.c_tab4 = tabs.c_tab4;
    a.u_tab4 = tabs.u_tab4;
    a.c_tab8 = tabs.c_tab8;
    a.u_tab8 = tabs.u_tab8;
    a.status = sl.d_status;
    // upload, planning and the status copy run on the batcher's own stream,
    // where they overlap the generation of the batches before this one; the
    // caller's stream waits for them, then generates
    hipError_t err = hipMemcpyAsync(sl.d_reqs, sl.h_reqs, count * sizeof(mirng_request),
                                    hipMemcpyHostToDevice, b->copy);
    if (err == hipSuccess && refs)
        err = hipMemcpyAsync(sl.d_refs, sl.h_refs, count * sizeof(EngineRef),
                             hipMemcpyHostToDevice, b->copy);
    if (err == hipSuccess) err = launch_batch_plan(a, b->copy);
    if (err == hipSuccess)
        err = hipMemcpyAsync(sl.h_status, sl.d_status, count * sizeof(int32_t),
                             hipMemcpyDeviceToHost, b->copy);
    if (err == hipSuccess) err = hipEventRecord(sl.planned, b->copy);
    if (err == hipSuccess) err = hipStreamWaitEvent(s, sl.planned, 0);
    if (a.philox && a.mrg) {
        // both engines: the MRG kernel (VALU-bound) runs on the side stream
        // beside the Philox kernel (bound by HBM writes), after everything
        // enqueued on the caller's stream before this batch, and the
        // caller's stream joins it before the batch counts as done
        BatchArgs ph = a, mg = a;
        ph.mrg = 0;
        mg.philox = 0;
        if (err == hipSuccess) err = hipEventRecord(sl.forked, s);
        if (err == hipSuccess) err = hipStreamWaitEvent(b->side, sl.forked, 0);
        if (err == hipSuccess) err = launch_batch_generate(mg, b->side);
        if (err == hipSuccess) err = hipEventRecord(sl.mrg_done, b->side);
        if (err == hipSuccess) err = launch_batch_generate(ph, s);
        if (err == hipSuccess) err = hipStreamWaitEvent(s, sl.mrg_done, 0);
    } else if (err == hipSuccess) {
        err = launch_batch_generate(a, s);
    }
    if (err == hipSuccess) err = hipEventRecord(sl.done, s);
    if (err != hipSuccess) {
        // part of the batch may be queued: let it drain before the slot's
        // buffers can be reused
        (void)hipStreamSynchronize(b->copy);
        (void)hipStreamSynchronize(b->side);
        (void)hipStreamSynchronize(s);
        return MIRNG_E_LAUNCH;
    }
    sl.pending = true;
    b->last = k;
    return MIRNG_OK;
}

extern "C" {

mirng_status mirng_batcher_statuses(mirng_batcher b, int32_t *statuses, size_t count)
{
    if (!b || (!statuses && count)) return MIRNG_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->last < 0) return count ? MIRNG_E_INVALID_ARG : MIRNG_OK;
    Slot &sl = b->slots[b->last];
    if (count > sl.count) return MIRNG_E_INVALID_ARG;
    if (sl.pending) {
        if (hipEventSynchronize(sl.done) != hipSuccess) return MIRNG_E_DEVICE;
        sl.pending = false;
    }
    std::memcpy(statuses, sl.h_status, count * sizeof(int32_t));
    return MIRNG_OK;
}

}  // extern "C"
