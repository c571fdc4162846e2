// Serving loop: the continuous-batching scheduler over HIP streams, one
// batcher per stream (each stream holds one batch in flight at a time),
// and the server's device-resident engine table.
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "mirng_bench.h"
#include "scheduler.hpp"

namespace mirng {
namespace {

// Requests per batch for which staging memory is allocated up front.
constexpr size_t kReserve = 4096;
// Engine table entries when the configuration asks for the default (0).
constexpr size_t kDefaultEngines = 65536;

class HipExecutor : public Executor {
public:
    ~HipExecutor() override { release(); }

    hipError_t init(int dev, int streams, size_t engines)
    {
        dev_ = dev;
        hipError_t err = hipMalloc((void **)&table_, engines * sizeof(mirng_state));
        if (err != hipSuccess) return err;
        for (int k = 0; k < streams; ++k) {
            hipStream_t s = nullptr;
            err = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (err != hipSuccess) return err;
            streams_.push_back(s);
            mirng_batcher b = nullptr;
            if (mirng_batcher_create(&b) != MIRNG_OK) return hipErrorOutOfMemory;
            batchers_.push_back(b);
            err = batcher_reserve(b, kReserve);
            if (err != hipSuccess) return err;
        }
        counts_.assign((size_t)streams, 0);
        reqs_.resize((size_t)streams);
        refs_.resize((size_t)streams);
        return hipSuccess;
    }

    void release()
    {
        for (mirng_batcher b : batchers_) mirng_batcher_destroy(b);
        for (hipStream_t s : streams_) (void)hipStreamDestroy(s);
        if (table_) (void)hipFree(table_);
        table_ = nullptr;
        batchers_.clear();
        streams_.clear();
    }

    int slots() const override { return (int)streams_.size(); }

    void bind_thread() override { (void)hipSetDevice(dev_); }

    mirng_status launch(int slot, const std::vector<Job> &jobs) override
    {
        const size_t k = (size_t)slot;
        counts_[k] = jobs.size();
        std::vector<mirng_request> &reqs = reqs_[k];
        std::vector<EngineRef> &refs = refs_[k];
        reqs.resize(jobs.size());
        refs.resize(jobs.size());
        bool any_ref = false;
        for (size_t i = 0; i < jobs.size(); ++i) {
            reqs[i] = jobs[i].req;
            refs[i] = jobs[i].ref;
            any_ref |= (jobs[i].ref.flags & kRefEngine) != 0;
        }
        return generate_batch_refs(batchers_[k], reqs.data(), any_ref ? refs.data() : nullptr,
                                   reqs.size(), table_, streams_[k]);
    }

    mirng_status wait(int slot, std::vector<int32_t> &statuses) override
    {
        statuses.assign(counts_[(size_t)slot], 0);
        return mirng_batcher_statuses(batchers_[(size_t)slot], statuses.data(),
                                      statuses.size());
    }

    // Writes table entry e (host-synchronous: the entry is resident before
    // any request on it can be submitted).
    hipError_t write_entry(uint32_t e, const mirng_state &st)
    {
        (void)hipSetDevice(dev_);
        return hipMemcpy(table_ + e, &st, sizeof st, hipMemcpyHostToDevice);
    }

private:
    int dev_ = 0;
    mirng_state *table_ = nullptr;    // device engine table
    std::vector<hipStream_t> streams_;
    std::vector<mirng_batcher> batchers_;
    std::vector<size_t> counts_;
    std::vector<std::vector<mirng_request>> reqs_;   // per slot, reused
    std::vector<std::vector<EngineRef>> refs_;
};

// State of an engine `consumed` words (Philox, modulo 2^130) or steps
// (MRG32k3a) past table entry `base`.
mirng_state advanced(const mirng_state &base, const uint64_t consumed[3])
{
    mirng_state s = base;
    if (base.engine_type == MIRNG_PHILOX4X32_10) {
        const Pos130 p = pos_add(Pos130{{base.pos[0], base.pos[1], base.pos[2]}}, consumed, 3);
        for (int i = 0; i < 3; ++i) s.pos[i] = p.l[i];
    } else {
        mrg_jump(s.words, consumed, 3);
        uint64_t carry = 0;
        for (int i = 0; i < 3; ++i) {
            const uint64_t s1 = base.pos[i] + consumed[i];
            const uint64_t c1 = s1 < consumed[i] ? 1 : 0;
            const uint64_t s2 = s1 + carry;
            carry = c1 | (s2 < carry ? 1 : 0);
            s.pos[i] = s2;
        }
    }
    return s;
}

bool state_valid(const mirng_state &s)
{
    if (s.engine_type == MIRNG_PHILOX4X32_10) {
        if (s.pos[2] > 3) return false;
        for (int i = 2; i < 6; ++i)
            if (s.words[i] != 0) return false;
        return true;
    }
    if (s.engine_type != MIRNG_MRG32K3A) return false;
    for (int i = 0; i < 3; ++i)
        if (s.words[i] >= kM1 || s.words[3 + i] >= kM2) return false;
    return (s.words[0] | s.words[1] | s.words[2]) && (s.words[3] | s.words[4] | s.words[5]);
}

}  // namespace
}  // namespace mirng

struct mirng_server_s {
    mirng::HipExecutor ex;              // outlives the scheduler's threads
    mirng::Scheduler *sched = nullptr;
    std::mutex mu;                      // engine bookkeeping below
    std::vector<mirng_state> entries;   // host copies of the device table entries
    size_t max_engines = 0;
};

using namespace mirng;

namespace {

// Validates a request on a resident engine the way the batched kernel
// validates a request (so that a request admitted on an engine never
// fails on the device and its consumption is final).
mirng_status check_engine_request(const mirng_distribution *d, uint64_t n, const void *out)
{
    if (!d || d->reserved != 0) return MIRNG_E_INVALID_ARG;
    const int32_t st = check_params(d->kind, d->p0, d->p1);
    if (st != MIRNG_OK) return (mirng_status)st;
    if (n == 0) return MIRNG_OK;
    if (!out || (uintptr_t)out % (uintptr_t)elem_bytes(d->kind)) return MIRNG_E_INVALID_ARG;
    if (n >= (1ull << 32)) return MIRNG_E_CAPACITY;
    return MIRNG_OK;
}

mirng_status submit_on_engine(mirng_server s, uint32_t engine, const mirng_distribution *d,
                              uint64_t n, void *out, uint64_t *ticket,
                              const std::chrono::steady_clock::time_point *arrival)
{
    const mirng_status v = check_engine_request(d, n, out);
    if (v != MIRNG_OK) return v;
    int32_t type = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (engine >= s->entries.size()) return MIRNG_E_INVALID_ARG;
        type = s->entries[engine].engine_type;
    }
    mirng_request r{};
    r.engine_type = type;
    r.dist = *d;
    r.n = n;
    r.out = out;
    return s->sched->submit_engine(engine, r, words_consumed(type, d->kind, n), ticket, arrival);
}

}  // namespace

extern "C" {

mirng_status mirng_server_create(const mirng_server_config *cfg, mirng_server *out)
{
    if (!cfg || !out) return MIRNG_E_INVALID_ARG;
    if (cfg->streams < 1 || cfg->streams > 8 || cfg->max_engines < 0 ||
        cfg->max_engines > (1 << 24) || cfg->capacity_bytes < 1 || cfg->max_batch < 1 ||
        cfg->max_batch > (1ull << 24))
        return MIRNG_E_INVALID_ARG;
    int dev = 0;
    if (ensure_device(&dev) != hipSuccess) return MIRNG_E_DEVICE;
    mirng_server s = new (std::nothrow) mirng_server_s();
    if (!s) return MIRNG_E_ALLOC;
    s->max_engines = cfg->max_engines ? (size_t)cfg->max_engines : kDefaultEngines;
    if (s->ex.init(dev, cfg->streams, s->max_engines) != hipSuccess) {
        delete s;
        return MIRNG_E_ALLOC;
    }
    s->sched = new (std::nothrow)
        Scheduler(s->ex, cfg->capacity_bytes, (size_t)cfg->max_batch, s->max_engines);
    if (!s->sched) {
        delete s;
        return MIRNG_E_ALLOC;
    }
    *out = s;
    return MIRNG_OK;
}

mirng_status mirng_server_destroy(mirng_server s)
{
    if (!s) return MIRNG_OK;
    delete s->sched;   // finishes every accepted request
    delete s;
    return MIRNG_OK;
}

mirng_status mirng_server_submit(mirng_server s, const mirng_request *req, uint64_t *ticket)
{
    if (!s || !req || !ticket) return MIRNG_E_INVALID_ARG;
    return s->sched->submit(*req, ticket);
}

mirng_status mirng_server_engine_create(mirng_server s, int32_t type, uint64_t seed,
                                        uint64_t offset, uint32_t *engine)
{
    if (!s || !engine) return MIRNG_E_INVALID_ARG;
    if (type != MIRNG_PHILOX4X32_10 && type != MIRNG_MRG32K3A) return MIRNG_E_UNSUPPORTED;
    mirng_state st{};
    st.engine_type = type;
    if (type == MIRNG_PHILOX4X32_10) {
        st.words[0] = (uint32_t)seed;
        st.words[1] = (uint32_t)(seed >> 32);
    } else {
        mrg_seed_state(seed, st.words);
        mrg_jump(st.words, &offset, 1);
    }
    st.pos[0] = offset;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->entries.size() >= s->max_engines) return MIRNG_E_CAPACITY;
    const uint32_t e = (uint32_t)s->entries.size();
    if (s->ex.write_entry(e, st) != hipSuccess) return MIRNG_E_DEVICE;
    if (s->sched->engine_add(e, type) != MIRNG_OK) return MIRNG_E_INVALID_ARG;
    s->entries.push_back(st);
    *engine = e;
    return MIRNG_OK;
}

mirng_status mirng_server_engine_skip_ahead(mirng_server s, uint32_t engine,
                                            const uint64_t *limbs, size_t nlimbs)
{
    if (!s || nlimbs > 3 || (nlimbs > 0 && !limbs)) return MIRNG_E_INVALID_ARG;
    return s->sched->engine_skip(engine, limbs, nlimbs);
}

mirng_status mirng_server_engine_get_state(mirng_server s, uint32_t engine, mirng_state *out)
{
    if (!s || !out) return MIRNG_E_INVALID_ARG;
    int32_t type = 0;
    uint64_t consumed[3];
    // the count first: a request admitted meanwhile only moves it further
    if (s->sched->engine_consumed(engine, &type, consumed) != MIRNG_OK) return MIRNG_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (engine >= s->entries.size()) return MIRNG_E_INVALID_ARG;
    *out = advanced(s->entries[engine], consumed);
    out->reserved = 0;
    return MIRNG_OK;
}

mirng_status mirng_server_engine_set_state(mirng_server s, uint32_t engine,
                                           const mirng_state *st)
{
    if (!s || !st || !state_valid(*st)) return MIRNG_E_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (engine >= s->entries.size() || s->entries[engine].engine_type != st->engine_type)
            return MIRNG_E_INVALID_ARG;
    }
    // requests admitted on the old entry must be planned before it changes
    s->sched->drain();
    std::lock_guard<std::mutex> lk(s->mu);
    mirng_state e = *st;
    e.reserved = 0;
    if (s->ex.write_entry(engine, e) != hipSuccess) return MIRNG_E_DEVICE;
    s->entries[engine] = e;
    return s->sched->engine_add(engine, e.engine_type);
}

mirng_status mirng_server_submit_engine(mirng_server s, uint32_t engine,
                                        const mirng_distribution *d, uint64_t n, void *out,
                                        uint64_t *ticket)
{
    if (!s || !ticket) return MIRNG_E_INVALID_ARG;
    return submit_on_engine(s, engine, d, n, out, ticket, nullptr);
}

mirng_status mirng_server_poll(mirng_server s, uint64_t ticket, int32_t *done, int32_t *status)
{
    if (!s || !done || !status) return MIRNG_E_INVALID_ARG;
    return s->sched->poll(ticket, done, status);
}

mirng_status mirng_server_wait(mirng_server s, uint64_t ticket, int32_t *status,
                               double *latency_ms)
{
    if (!s || !status) return MIRNG_E_INVALID_ARG;
    return s->sched->wait(ticket, status, latency_ms);
}

mirng_status mirng_server_drain(mirng_server s)
{
    if (!s) return MIRNG_E_INVALID_ARG;
    s->sched->drain();
    return MIRNG_OK;
}

mirng_status mirng_server_stats_get(mirng_server s, mirng_server_stats *out)
{
    if (!s || !out) return MIRNG_E_INVALID_ARG;
    *out = s->sched->stats();
    return MIRNG_OK;
}

mirng_status mirng_bench_server_replay(mirng_server s, const mirng_request *reqs,
                                       const uint32_t *engines, const double *arrival_s,
                                       size_t count, uint64_t *tickets, int32_t *submit_status)
{
    if (!s || (count && (!reqs || !arrival_s || !tickets || !submit_status)))
        return MIRNG_E_INVALID_ARG;
    using Clock = std::chrono::steady_clock;
    const Clock::time_point t0 = Clock::now();
    for (size_t i = 0; i < count; ++i) {
        const Clock::time_point due =
            t0 + std::chrono::nanoseconds((int64_t)(arrival_s[i] * 1e9));
        const Clock::time_point coarse = due - std::chrono::microseconds(50);
        if (Clock::now() < coarse) std::this_thread::sleep_until(coarse);
        while (Clock::now() < due) {
        }
        tickets[i] = ~0ull;
        if (engines)
            submit_status[i] = submit_on_engine(s, engines[i], &reqs[i].dist, reqs[i].n,
                                                reqs[i].out, &tickets[i], &due);
        else
            submit_status[i] = s->sched->submit(reqs[i], &tickets[i], &due);
    }
    return MIRNG_OK;
}

}  // extern "C"
