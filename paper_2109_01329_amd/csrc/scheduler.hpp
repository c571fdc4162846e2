// Continuous-batching scheduler of the serving loop, independent of HIP so
// that its policy can be exercised on the host with a simulated executor.
//
// Requests wait in arrival order.  A dispatcher thread launches, whenever an
// executor slot (a stream) is free, every waiting request that fits: in
// arrival order, while the output bytes of admitted, unfinished requests
// stay within the capacity, up to max_batch per batch.  Each slot has its
// own completion thread, which waits for that slot's batch, records the
// per-request statuses and completion times, and returns the batch's bytes
// to the admission budget, so a batch on one stream completes as soon as it
// is done, whatever the batches on the other streams are doing.
//
// Resident engines: the scheduler also keeps, per engine of the server's
// device table, the words (Philox4x32-10) or steps (MRG32k3a) that the
// requests admitted on it so far consume.  A request on a resident engine
// is given that count as its start (relative to the table entry) when it is
// admitted, under the same lock that orders arrivals, and the count
// advances by the request's consumption.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "jobs.hpp"
#include "mirng.h"

namespace mirng {

// Runs batches; slot k holds at most one batch at a time.
class Executor {
public:
    virtual ~Executor() = default;
    virtual int slots() const = 0;
    // Called once on each scheduler thread before any other call from it.
    virtual void bind_thread() {}
    // Enqueue `jobs` as one batch on slot k (asynchronous).
    virtual mirng_status launch(int slot, const std::vector<Job> &jobs) = 0;
    // Block until slot k's batch has completed; statuses of its requests.
    virtual mirng_status wait(int slot, std::vector<int32_t> &statuses) = 0;
};

// Output bytes of a request as admission counts them.
uint64_t request_bytes(const mirng_request &r);

class Scheduler {
public:
    using Clock = std::chrono::steady_clock;

    Scheduler(Executor &ex, uint64_t capacity_bytes, size_t max_batch, size_t max_engines = 0);
    ~Scheduler();   // finishes every accepted request, then stops
    Scheduler(const Scheduler &) = delete;
    Scheduler &operator=(const Scheduler &) = delete;

    // `arrival` (default: now) is the time latency is measured from; an
    // open-loop load generator passes the scheduled arrival, so that a late
    // submission still counts against the latency.
    mirng_status submit(const mirng_request &r, uint64_t *ticket,
                        const Clock::time_point *arrival = nullptr);
    mirng_status poll(uint64_t ticket, int32_t *done, int32_t *status);
    mirng_status wait(uint64_t ticket, int32_t *status, double *latency_ms);
    void drain();
    mirng_server_stats stats();
    // Batches launched so far, as lists of tickets (for policy tests).
    std::vector<std::vector<uint64_t>> batch_log();

    // Resident engines.  engine_add registers slot `e` (< max_engines) with
    // engine type `type` and nothing consumed (also a reset, after its
    // table entry was rewritten).  submit_engine admits r (its
    // engine_type is replaced by the engine's) on engine e, which consumes
    // `words`; unknown engine -> INVALID_ARG.  engine_skip advances the
    // count by n = sum limbs[i] 2^(64 i) (mod 2^192).  engine_consumed
    // copies the count out.
    mirng_status engine_add(uint32_t e, int32_t type);
    mirng_status submit_engine(uint32_t e, const mirng_request &r, uint64_t words,
                               uint64_t *ticket, const Clock::time_point *arrival = nullptr);
    mirng_status engine_skip(uint32_t e, const uint64_t *limbs, size_t nlimbs);
    mirng_status engine_consumed(uint32_t e, int32_t *type, uint64_t consumed[3]);

private:
    struct Ticket {
        Clock::time_point submitted;
        Clock::time_point finished;
        uint64_t bytes = 0;
        uint64_t n = 0;
        int32_t status = 0;
        bool done = false;
    };
    struct Waiting {
        uint64_t ticket;
        Job job;
    };
    struct InFlight {
        std::vector<uint64_t> tickets;
        uint64_t bytes = 0;
        mirng_status failed = MIRNG_OK;   // launch status
    };
    struct EngineCount {
        int32_t type = 0;                 // 0: not registered
        uint64_t consumed[3] = {0, 0, 0};
    };

    mirng_status enqueue(const Job &j, uint64_t *ticket, const Clock::time_point *arrival);
    void dispatch_loop();
    void complete_loop(int slot);

    Executor &ex_;
    const uint64_t capacity_;
    const size_t max_batch_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Waiting> waiting_;
    std::vector<bool> slot_busy_;         // a batch is being launched or is in flight
    std::vector<bool> slot_ready_;        // slot_batch_[k] holds a launched batch
    std::vector<InFlight> slot_batch_;
    std::vector<Ticket> tickets_;
    std::vector<std::vector<uint64_t>> log_;
    std::vector<EngineCount> engines_;
    uint64_t inflight_bytes_ = 0;
    uint64_t max_inflight_bytes_ = 0;
    uint64_t refused_ = 0;
    uint64_t completed_ = 0;
    int launching_ = 0;               // batches between dequeue and launch
    bool stop_ = false;
    bool have_first_ = false;
    Clock::time_point first_;
    Clock::time_point last_;
    std::thread dispatcher_;
    std::vector<std::thread> completers_;
};

}  // namespace mirng
