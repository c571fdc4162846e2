// Continuous-batching scheduler (host only, no HIP): admission by in-flight
// output bytes, arrival-order batching onto free executor slots, per-slot
// completion, resident-engine positions, and latency statistics.
#include "scheduler.hpp"

#include <algorithm>
#include <cmath>

namespace mirng {

uint64_t request_bytes(const mirng_request &r)
{
    // requests the batched kernel refuses write nothing
    if (r.dist.kind < MIRNG_BITS_U32 || r.dist.kind > MIRNG_GAUSSIAN_ICDF_F64) return 0;
    if (r.n >= (1ull << 32)) return 0;
    const bool f64 = r.dist.kind == MIRNG_UNIFORM_F64 || r.dist.kind == MIRNG_GAUSSIAN_F64 ||
                     r.dist.kind == MIRNG_GAUSSIAN_ICDF_F64;
    return r.n * (f64 ? 8u : 4u);
}

namespace {

// a += b over 192-bit little-endian limbs (mod 2^192).
void add192(uint64_t a[3], const uint64_t *b, size_t nb)
{
    uint64_t carry = 0;
    for (size_t i = 0; i < 3; ++i) {
        const uint64_t add = i < nb ? b[i] : 0;
        const uint64_t s1 = a[i] + add;
        const uint64_t c1 = s1 < add ? 1 : 0;
        const uint64_t s2 = s1 + carry;
        const uint64_t c2 = s2 < carry ? 1 : 0;
        a[i] = s2;
        carry = c1 | c2;
    }
}

}  // namespace

Scheduler::Scheduler(Executor &ex, uint64_t capacity_bytes, size_t max_batch, size_t max_engines)
    : ex_(ex), capacity_(capacity_bytes), max_batch_(max_batch),
      slot_busy_((size_t)ex.slots(), false), slot_ready_((size_t)ex.slots(), false),
      slot_batch_((size_t)ex.slots()), engines_(max_engines)
{
    dispatcher_ = std::thread([this] { dispatch_loop(); });
    for (int k = 0; k < ex.slots(); ++k) completers_.emplace_back([this, k] { complete_loop(k); });
}

Scheduler::~Scheduler()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    dispatcher_.join();
    for (std::thread &t : completers_) t.join();
}

// Queues an admitted job (mu_ held by the caller).
mirng_status Scheduler::enqueue(const Job &j, uint64_t *ticket,
                                const Clock::time_point *arrival)
{
    Ticket t;
    t.submitted = arrival ? *arrival : Clock::now();
    t.bytes = request_bytes(j.req);
    t.n = j.req.n;
    const uint64_t id = tickets_.size();
    tickets_.push_back(t);
    waiting_.push_back({id, j});
    if (!have_first_ || t.submitted < first_) {
        first_ = t.submitted;
        have_first_ = true;
    }
    *ticket = id;
    cv_.notify_all();
    return MIRNG_OK;
}

mirng_status Scheduler::submit(const mirng_request &r, uint64_t *ticket,
                               const Clock::time_point *arrival)
{
    const uint64_t bytes = request_bytes(r);
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return MIRNG_E_INVALID_ARG;
    if (bytes > capacity_) {
        ++refused_;
        return MIRNG_E_CAPACITY;
    }
    Job j{};
    j.req = r;
    return enqueue(j, ticket, arrival);
}

mirng_status Scheduler::engine_add(uint32_t e, int32_t type)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (e >= engines_.size() || (type != MIRNG_PHILOX4X32_10 && type != MIRNG_MRG32K3A))
        return MIRNG_E_INVALID_ARG;
    engines_[e] = EngineCount{};
    engines_[e].type = type;
    return MIRNG_OK;
}

mirng_status Scheduler::submit_engine(uint32_t e, const mirng_request &r, uint64_t words,
                                      uint64_t *ticket, const Clock::time_point *arrival)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_ || e >= engines_.size() || engines_[e].type == 0) return MIRNG_E_INVALID_ARG;
    Job j{};
    j.req = r;
    j.req.engine_type = engines_[e].type;
    if (request_bytes(j.req) > capacity_) {
        ++refused_;
        return MIRNG_E_CAPACITY;
    }
    j.ref.slot = e;
    j.ref.flags = kRefEngine;
    for (int i = 0; i < 3; ++i) j.ref.skip[i] = engines_[e].consumed[i];
    add192(engines_[e].consumed, &words, 1);
    return enqueue(j, ticket, arrival);
}

mirng_status Scheduler::engine_skip(uint32_t e, const uint64_t *limbs, size_t nlimbs)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (e >= engines_.size() || engines_[e].type == 0 || nlimbs > 3) return MIRNG_E_INVALID_ARG;
    add192(engines_[e].consumed, limbs, nlimbs);
    return MIRNG_OK;
}

mirng_status Scheduler::engine_consumed(uint32_t e, int32_t *type, uint64_t consumed[3])
{
    std::lock_guard<std::mutex> lk(mu_);
    if (e >= engines_.size() || engines_[e].type == 0) return MIRNG_E_INVALID_ARG;
    *type = engines_[e].type;
    for (int i = 0; i < 3; ++i) consumed[i] = engines_[e].consumed[i];
    return MIRNG_OK;
}

mirng_status Scheduler::poll(uint64_t ticket, int32_t *done, int32_t *status)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (ticket >= tickets_.size()) return MIRNG_E_INVALID_ARG;
    const Ticket &t = tickets_[ticket];
    *done = t.done ? 1 : 0;
    *status = t.done ? t.status : MIRNG_OK;
    return MIRNG_OK;
}

mirng_status Scheduler::wait(uint64_t ticket, int32_t *status, double *latency_ms)
{
    std::unique_lock<std::mutex> lk(mu_);
    if (ticket >= tickets_.size()) return MIRNG_E_INVALID_ARG;
    cv_.wait(lk, [&] { return tickets_[ticket].done; });
    const Ticket &t = tickets_[ticket];
    *status = t.status;
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(t.finished - t.submitted).count();
    return MIRNG_OK;
}

void Scheduler::drain()
{
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return completed_ == tickets_.size(); });
}

std::vector<std::vector<uint64_t>> Scheduler::batch_log()
{
    std::lock_guard<std::mutex> lk(mu_);
    return log_;
}

mirng_server_stats Scheduler::stats()
{
    std::lock_guard<std::mutex> lk(mu_);
    mirng_server_stats s{};
    s.submitted = tickets_.size();
    s.refused = refused_;
    s.batches = log_.size();
    s.max_inflight_bytes = max_inflight_bytes_;
    std::vector<double> lat;
    lat.reserve(completed_);
    for (const Ticket &t : tickets_) {
        if (!t.done) continue;
        ++s.completed;
        lat.push_back(std::chrono::duration<double, std::milli>(t.finished - t.submitted).count());
        if (t.status != MIRNG_OK) {
            ++s.failed;
        } else {
            s.samples += t.n;
            s.bytes += t.bytes;
        }
    }
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        // nearest-rank percentiles
        auto pct = [&](double q) {
            size_t k = (size_t)std::ceil(q * (double)lat.size());
            return lat[k == 0 ? 0 : k - 1];
        };
        s.latency_p50_ms = pct(0.50);
        s.latency_p99_ms = pct(0.99);
        s.latency_max_ms = lat.back();
        s.span_s = std::chrono::duration<double>(last_ - first_).count();
    }
    return s;
}

void Scheduler::dispatch_loop()
{
    ex_.bind_thread();
    std::unique_lock<std::mutex> lk(mu_);
    auto free_slot = [&]() -> int {
        for (size_t k = 0; k < slot_busy_.size(); ++k)
            if (!slot_busy_[k]) return (int)k;
        return -1;
    };
    auto head_fits = [&] {
        return !waiting_.empty() &&
               inflight_bytes_ + tickets_[waiting_.front().ticket].bytes <= capacity_;
    };
    for (;;) {
        cv_.wait(lk, [&] {
            return (stop_ && waiting_.empty()) || (head_fits() && free_slot() >= 0);
        });
        if (waiting_.empty()) break;   // stopping, nothing left to launch
        const int slot = free_slot();
        std::vector<Job> jobs;
        InFlight b;
        while (!waiting_.empty() && jobs.size() < max_batch_) {
            const Waiting &w = waiting_.front();
            const uint64_t bytes = tickets_[w.ticket].bytes;
            if (inflight_bytes_ + b.bytes + bytes > capacity_) break;
            b.bytes += bytes;
            b.tickets.push_back(w.ticket);
            jobs.push_back(w.job);
            waiting_.pop_front();
        }
        inflight_bytes_ += b.bytes;
        max_inflight_bytes_ = std::max(max_inflight_bytes_, inflight_bytes_);
        slot_busy_[(size_t)slot] = true;
        log_.push_back(b.tickets);
        ++launching_;
        lk.unlock();
        const mirng_status st = ex_.launch(slot, jobs);
        lk.lock();
        --launching_;
        b.failed = st;
        slot_batch_[(size_t)slot] = std::move(b);
        slot_ready_[(size_t)slot] = true;
        cv_.notify_all();
    }
}

void Scheduler::complete_loop(int slot)
{
    ex_.bind_thread();
    const size_t k = (size_t)slot;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        cv_.wait(lk, [&] {
            return slot_ready_[k] || (stop_ && waiting_.empty() && launching_ == 0);
        });
        if (!slot_ready_[k]) break;   // stopping, nothing left for this slot
        InFlight b = std::move(slot_batch_[k]);
        slot_ready_[k] = false;
        lk.unlock();
        std::vector<int32_t> st;
        mirng_status s = b.failed;
        if (s == MIRNG_OK) s = ex_.wait(slot, st);
        const Clock::time_point now = Clock::now();
        lk.lock();
        for (size_t i = 0; i < b.tickets.size(); ++i) {
            Ticket &t = tickets_[b.tickets[i]];
            t.done = true;
            t.finished = now;
            if (s != MIRNG_OK)
                t.status = s;
            else
                t.status = i < st.size() ? st[i] : (int32_t)MIRNG_E_DEVICE;
            ++completed_;
        }
        if (now > last_) last_ = now;
        inflight_bytes_ -= b.bytes;
        slot_busy_[k] = false;
        cv_.notify_all();
    }
}

}  // namespace mirng
