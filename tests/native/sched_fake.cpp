// Host-only driver of the serving scheduler with a simulated executor: each
// slot "runs" a batch for base_us + bytes * ns_per_byte and reports the
// statuses the batched kernel would give (kinds 1-8 known; unknown kind ->
// UNSUPPORTED,
// n >= 2^32 -> CAPACITY).  Prints one JSON object for the Python tests.
//
// usage: sched_fake slots capacity max_batch ns_per_byte base_us count gap_us seed max_n
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "scheduler.hpp"

using namespace mirng;
using Clock = std::chrono::steady_clock;

class FakeExecutor : public Executor {
public:
    FakeExecutor(int slots, double ns_per_byte, double base_us)
        : n_(slots), ns_per_byte_(ns_per_byte), base_us_(base_us), busy_(slots, false),
          finish_(slots), st_(slots)
    {
    }
    int slots() const override { return n_; }
    void bind_thread() override { ++binds_; }
    mirng_status launch(int slot, const std::vector<mirng_request> &reqs) override
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (busy_[slot]) double_launch_ = true;
        busy_[slot] = true;
        int conc = 0;
        for (bool b : busy_) conc += b ? 1 : 0;
        max_conc_ = std::max(max_conc_, conc);
        uint64_t bytes = 0;
        st_[slot].clear();
        for (const mirng_request &r : reqs) {
            bytes += request_bytes(r);
            int32_t s = MIRNG_OK;
            if (r.dist.kind < 1 || r.dist.kind > 8) s = MIRNG_E_UNSUPPORTED;
            else if (r.n >= (1ull << 32)) s = MIRNG_E_CAPACITY;
            st_[slot].push_back(s);
        }
        finish_[slot] = Clock::now() + std::chrono::nanoseconds(
            (int64_t)(base_us_ * 1e3 + (double)bytes * ns_per_byte_));
        return MIRNG_OK;
    }
    mirng_status wait(int slot, std::vector<int32_t> &statuses) override
    {
        Clock::time_point t;
        {
            std::lock_guard<std::mutex> lk(mu_);
            t = finish_[slot];
        }
        std::this_thread::sleep_until(t);
        std::lock_guard<std::mutex> lk(mu_);
        statuses = st_[slot];
        busy_[slot] = false;
        return MIRNG_OK;
    }
    int n_;
    double ns_per_byte_, base_us_;
    std::mutex mu_;
    std::vector<bool> busy_;
    std::vector<Clock::time_point> finish_;
    std::vector<std::vector<int32_t>> st_;
    bool double_launch_ = false;
    int max_conc_ = 0;
    int binds_ = 0;
};

int main(int argc, char **argv)
{
    if (argc != 10) {
        std::fprintf(stderr, "usage: %s slots capacity max_batch ns_per_byte base_us count "
                             "gap_us seed max_n\n", argv[0]);
        return 2;
    }
    const int slots = std::atoi(argv[1]);
    const uint64_t capacity = std::strtoull(argv[2], nullptr, 10);
    const size_t max_batch = std::strtoull(argv[3], nullptr, 10);
    const double ns_per_byte = std::atof(argv[4]);
    const double base_us = std::atof(argv[5]);
    const int count = std::atoi(argv[6]);
    const double gap_us = std::atof(argv[7]);
    const uint64_t seed = std::strtoull(argv[8], nullptr, 10);
    const double max_n = std::atof(argv[9]);

    FakeExecutor ex(slots, ns_per_byte, base_us);
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::vector<int> ret(count);
    std::vector<uint64_t> ticket(count, ~0ull), bytes(count);
    std::vector<int32_t> expect(count), got(count, -1), kinds(count);
    std::vector<uint64_t> ns(count);
    mirng_server_stats st{};
    std::vector<std::vector<uint64_t>> log;
    {
        Scheduler sch(ex, capacity, max_batch);
        const Clock::time_point t0 = Clock::now();
        for (int i = 0; i < count; ++i) {
            mirng_request r{};
            r.engine_type = (U(rng) < 0.5) ? 1 : 2;
            const double u = U(rng);
            r.dist.kind = u < 0.05 ? 9 : 1 + (int)(U(rng) * 8) % 8;
            r.dist.p1 = 1.0;
            r.n = (uint64_t)std::floor(std::pow(10.0, U(rng) * std::log10(max_n)));
            if (U(rng) < 0.02) r.n = 1ull << 32;
            bytes[i] = request_bytes(r);
            kinds[i] = r.dist.kind;
            ns[i] = r.n;
            expect[i] = (r.dist.kind < 1 || r.dist.kind > 8) ? MIRNG_E_UNSUPPORTED
                        : (r.n >= (1ull << 32))              ? MIRNG_E_CAPACITY
                                                             : MIRNG_OK;
            if (gap_us > 0)
                std::this_thread::sleep_until(t0 + std::chrono::nanoseconds(
                                                       (int64_t)(gap_us * 1e3 * i)));
            ret[i] = sch.submit(r, &ticket[i]);
        }
        for (int i = 0; i < count; ++i) {
            if (ret[i] != MIRNG_OK) continue;
            int32_t done = 0, s = 0;
            sch.poll(ticket[i], &done, &s);
            double lat = 0.0;
            sch.wait(ticket[i], &s, &lat);
            got[i] = s;
        }
        sch.drain();
        st = sch.stats();
        log = sch.batch_log();
    }
    std::printf("{\"ret\": [");
    for (int i = 0; i < count; ++i) std::printf("%s%d", i ? "," : "", ret[i]);
    std::printf("], \"ticket\": [");
    for (int i = 0; i < count; ++i)
        std::printf("%s%lld", i ? "," : "", ret[i] ? -1LL : (long long)ticket[i]);
    std::printf("], \"kind\": [");
    for (int i = 0; i < count; ++i) std::printf("%s%d", i ? "," : "", kinds[i]);
    std::printf("], \"n\": [");
    for (int i = 0; i < count; ++i) std::printf("%s%llu", i ? "," : "", (unsigned long long)ns[i]);
    std::printf("], \"bytes\": [");
    for (int i = 0; i < count; ++i) std::printf("%s%llu", i ? "," : "", (unsigned long long)bytes[i]);
    std::printf("], \"expect\": [");
    for (int i = 0; i < count; ++i) std::printf("%s%d", i ? "," : "", expect[i]);
    std::printf("], \"status\": [");
    for (int i = 0; i < count; ++i) std::printf("%s%d", i ? "," : "", got[i]);
    std::printf("], \"batches\": [");
    for (size_t b = 0; b < log.size(); ++b) {
        std::printf("%s[", b ? "," : "");
        for (size_t j = 0; j < log[b].size(); ++j)
            std::printf("%s%llu", j ? "," : "", (unsigned long long)log[b][j]);
        std::printf("]");
    }
    std::printf("], \"double_launch\": %s, \"max_concurrent\": %d, \"binds\": %d, ",
                ex.double_launch_ ? "true" : "false", ex.max_conc_, ex.binds_);
    std::printf("\"stats\": {\"submitted\": %llu, \"refused\": %llu, \"completed\": %llu, "
                "\"failed\": %llu, \"batches\": %llu, \"samples\": %llu, \"bytes\": %llu, "
                "\"max_inflight_bytes\": %llu, \"p50\": %.6f, \"p99\": %.6f, \"max\": %.6f, "
                "\"span_s\": %.6f}}\n",
                (unsigned long long)st.submitted, (unsigned long long)st.refused,
                (unsigned long long)st.completed, (unsigned long long)st.failed,
                (unsigned long long)st.batches, (unsigned long long)st.samples,
                (unsigned long long)st.bytes, (unsigned long long)st.max_inflight_bytes,
                st.latency_p50_ms, st.latency_p99_ms, st.latency_max_ms, st.span_s);
    return 0;
}
