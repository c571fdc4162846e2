// Serving loop: the continuous-batching scheduler over HIP streams, one
// batcher per stream (each stream holds one batch in flight at a time).
#include <chrono>
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

class HipExecutor : public Executor {
public:
    ~HipExecutor() override { release(); }

    hipError_t init(int dev, int streams)
    {
        dev_ = dev;
        for (int k = 0; k < streams; ++k) {
            hipStream_t s = nullptr;
            hipError_t err = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (err != hipSuccess) return err;
            streams_.push_back(s);
            mirng_batcher b = nullptr;
            if (mirng_batcher_create(&b) != MIRNG_OK) return hipErrorOutOfMemory;
            batchers_.push_back(b);
            err = batcher_reserve(b, kReserve);
            if (err != hipSuccess) return err;
        }
        counts_.assign((size_t)streams, 0);
        return hipSuccess;
    }

    void release()
    {
        for (mirng_batcher b : batchers_) mirng_batcher_destroy(b);
        for (hipStream_t s : streams_) (void)hipStreamDestroy(s);
        batchers_.clear();
        streams_.clear();
    }

    int slots() const override { return (int)streams_.size(); }

    void bind_thread() override { (void)hipSetDevice(dev_); }

    mirng_status launch(int slot, const std::vector<mirng_request> &reqs) override
    {
        counts_[(size_t)slot] = reqs.size();
        return mirng_generate_batch(batchers_[(size_t)slot], reqs.data(), reqs.size(),
                                    streams_[(size_t)slot]);
    }

    mirng_status wait(int slot, std::vector<int32_t> &statuses) override
    {
        statuses.assign(counts_[(size_t)slot], 0);
        return mirng_batcher_statuses(batchers_[(size_t)slot], statuses.data(),
                                      statuses.size());
    }

private:
    int dev_ = 0;
    std::vector<hipStream_t> streams_;
    std::vector<mirng_batcher> batchers_;
    std::vector<size_t> counts_;
};

}  // namespace
}  // namespace mirng

struct mirng_server_s {
    mirng::HipExecutor ex;              // outlives the scheduler's threads
    mirng::Scheduler *sched = nullptr;
};

using namespace mirng;

extern "C" {

mirng_status mirng_server_create(const mirng_server_config *cfg, mirng_server *out)
{
    if (!cfg || !out) return MIRNG_E_INVALID_ARG;
    if (cfg->streams < 1 || cfg->streams > 8 || cfg->reserved != 0 || cfg->capacity_bytes < 1 ||
        cfg->max_batch < 1 || cfg->max_batch > (1ull << 24))
        return MIRNG_E_INVALID_ARG;
    int dev = 0;
    if (ensure_device(&dev) != hipSuccess) return MIRNG_E_DEVICE;
    mirng_server s = new (std::nothrow) mirng_server_s();
    if (!s) return MIRNG_E_ALLOC;
    if (s->ex.init(dev, cfg->streams) != hipSuccess) {
        delete s;
        return MIRNG_E_ALLOC;
    }
    s->sched = new (std::nothrow) Scheduler(s->ex, cfg->capacity_bytes, (size_t)cfg->max_batch);
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
                                       const double *arrival_s, size_t count,
                                       uint64_t *tickets, int32_t *submit_status)
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
        submit_status[i] = s->sched->submit(reqs[i], &tickets[i], &due);
    }
    return MIRNG_OK;
}

}  // extern "C"
