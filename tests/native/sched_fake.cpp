// Host-only driver of the serving scheduler with a simulated executor: each
// slot "runs" a batch for base_us * slot_factor[slot] + bytes * ns_per_byte
// and reports the statuses the batched kernel would give (kinds 1-8 known;
// unknown kind -> UNSUPPORTED, n >= 2^32 -> CAPACITY); launches listed in
// fail_at return MIRNG_E_LAUNCH.  Prints one JSON object for the Python
// tests.
//
// usage: sched_fake mode slots capacity max_batch ns_per_byte base_us count gap_us seed
//                   max_n [slot0_factor [fail_at,...]]
//   mode random:  random requests (engine, kind, n), arrivals gap_us apart
//   mode engines: requests on 8 resident engines (submit_engine, with each
//                 request's consumption = n), and a skip of 2^100 + 5 on
//                 engine 3 half-way; prints every job's engine reference
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
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
    FakeExecutor(int slots, double ns_per_byte, double base_us, double slot0_factor,
                 std::vector<int> fail_at)
        : n_(slots), ns_per_byte_(ns_per_byte), base_us_(base_us), slot0_factor_(slot0_factor),
          fail_at_(std::move(fail_at)), busy_(slots, false), finish_(slots), st_(slots)
    {
    }
    int slots() const override { return n_; }
    void bind_thread() override
    {
        std::lock_guard<std::mutex> lk(mu_);
        ++binds_;
    }
    mirng_status launch(int slot, const std::vector<Job> &jobs) override
    {
        std::lock_guard<std::mutex> lk(mu_);
        const int index = launches_++;
        for (const Job &j : jobs) refs_[j.req.seed] = j.ref;   // seed carries the request id
        if (std::find(fail_at_.begin(), fail_at_.end(), index) != fail_at_.end()) {
            failed_.push_back(index);
            return MIRNG_E_LAUNCH;
        }
        if (busy_[slot]) double_launch_ = true;
        busy_[slot] = true;
        int conc = 0;
        for (bool b : busy_) conc += b ? 1 : 0;
        max_conc_ = std::max(max_conc_, conc);
        uint64_t bytes = 0;
        st_[slot].clear();
        for (const Job &j : jobs) {
            const mirng_request &r = j.req;
            bytes += request_bytes(r);
            int32_t s = MIRNG_OK;
            if (r.dist.kind < 1 || r.dist.kind > 8) s = MIRNG_E_UNSUPPORTED;
            else if (r.n >= (1ull << 32)) s = MIRNG_E_CAPACITY;
            st_[slot].push_back(s);
        }
        const double base = base_us_ * (slot == 0 ? slot0_factor_ : 1.0);
        finish_[slot] = Clock::now() + std::chrono::nanoseconds(
            (int64_t)(base * 1e3 + (double)bytes * ns_per_byte_));
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
    double ns_per_byte_, base_us_, slot0_factor_;
    std::vector<int> fail_at_, failed_;
    std::mutex mu_;
    std::vector<bool> busy_;
    std::vector<Clock::time_point> finish_;
    std::vector<std::vector<int32_t>> st_;
    std::map<uint64_t, EngineRef> refs_;
    int launches_ = 0;
    bool double_launch_ = false;
    int max_conc_ = 0;
    int binds_ = 0;
};

static void print_u64s(const char *name, const std::vector<uint64_t> &v)
{
    std::printf("\"%s\": [", name);
    for (size_t i = 0; i < v.size(); ++i)
        std::printf("%s%llu", i ? "," : "", (unsigned long long)v[i]);
    std::printf("], ");
}

static void print_ints(const char *name, const std::vector<int32_t> &v)
{
    std::printf("\"%s\": [", name);
    for (size_t i = 0; i < v.size(); ++i) std::printf("%s%d", i ? "," : "", v[i]);
    std::printf("], ");
}

int main(int argc, char **argv)
{
    if (argc < 11) {
        std::fprintf(stderr, "usage: %s mode slots capacity max_batch ns_per_byte base_us count "
                             "gap_us seed max_n [slot0_factor [fail_at,...]]\n", argv[0]);
        return 2;
    }
    const std::string mode = argv[1];
    const int slots = std::atoi(argv[2]);
    const uint64_t capacity = std::strtoull(argv[3], nullptr, 10);
    const size_t max_batch = std::strtoull(argv[4], nullptr, 10);
    const double ns_per_byte = std::atof(argv[5]);
    const double base_us = std::atof(argv[6]);
    const int count = std::atoi(argv[7]);
    const double gap_us = std::atof(argv[8]);
    const uint64_t seed = std::strtoull(argv[9], nullptr, 10);
    const double max_n = std::atof(argv[10]);
    const double slot0_factor = argc > 11 ? std::atof(argv[11]) : 1.0;
    std::vector<int> fail_at;
    if (argc > 12) {
        std::string s = argv[12];
        size_t p = 0;
        while (p < s.size()) {
            size_t q = s.find(',', p);
            if (q == std::string::npos) q = s.size();
            if (q > p) fail_at.push_back(std::atoi(s.substr(p, q - p).c_str()));
            p = q + 1;
        }
    }
    const bool engines = mode == "engines";
    const uint32_t kEngines = 8;

    FakeExecutor ex(slots, ns_per_byte, base_us, slot0_factor, fail_at);
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::vector<int32_t> ret(count), kinds(count), expect(count), got(count, -1);
    std::vector<int32_t> eng_of(count, -1);
    std::vector<uint64_t> ticket(count, ~0ull), bytes(count), ns(count), words(count);
    std::vector<double> submit_ms(count), finish_ms(count, -1.0);
    mirng_server_stats st{};
    std::vector<std::vector<uint64_t>> log;
    std::vector<uint64_t> consumed_lo(kEngines), consumed_mid(kEngines);
    int skip_after = -1;
    {
        Scheduler sch(ex, capacity, max_batch, engines ? kEngines : 0);
        if (engines)
            for (uint32_t e = 0; e < kEngines; ++e) sch.engine_add(e, 1 + (int32_t)(e & 1));
        const Clock::time_point t0 = Clock::now();
        for (int i = 0; i < count; ++i) {
            mirng_request r{};
            r.engine_type = (U(rng) < 0.5) ? 1 : 2;
            const double u = U(rng);
            r.dist.kind = (!engines && u < 0.05) ? 9 : 1 + (int)(U(rng) * 8) % 8;
            r.dist.p1 = 1.0;
            r.n = (uint64_t)std::floor(std::pow(10.0, U(rng) * std::log10(max_n)));
            if (!engines && U(rng) < 0.02) r.n = 1ull << 32;
            r.seed = (uint64_t)i;                    // request id, echoed by the executor
            bytes[i] = request_bytes(r);
            kinds[i] = r.dist.kind;
            ns[i] = r.n;
            expect[i] = (r.dist.kind < 1 || r.dist.kind > 8) ? MIRNG_E_UNSUPPORTED
                        : (r.n >= (1ull << 32))              ? MIRNG_E_CAPACITY
                                                             : MIRNG_OK;
            if (gap_us > 0)
                std::this_thread::sleep_until(t0 + std::chrono::nanoseconds(
                                                       (int64_t)(gap_us * 1e3 * i)));
            submit_ms[i] = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
            if (engines) {
                const uint32_t e = (uint32_t)(U(rng) * kEngines) % kEngines;
                eng_of[i] = (int32_t)e;
                words[i] = r.n;
                ret[i] = sch.submit_engine(e, r, r.n, &ticket[i]);
                if (i == count / 2) {
                    const uint64_t skip[2] = {5, 1ull << 36};   // 2^100 + 5
                    sch.engine_skip(3, skip, 2);
                    skip_after = i;
                }
            } else {
                ret[i] = sch.submit(r, &ticket[i]);
            }
        }
        for (int i = 0; i < count; ++i) {
            if (ret[i] != MIRNG_OK) continue;
            int32_t done = 0, s = 0;
            sch.poll(ticket[i], &done, &s);
            double lat = 0.0;
            sch.wait(ticket[i], &s, &lat);
            got[i] = s;
            finish_ms[i] = submit_ms[i] + lat;
        }
        sch.drain();
        st = sch.stats();
        log = sch.batch_log();
        for (uint32_t e = 0; e < kEngines && engines; ++e) {
            int32_t type = 0;
            uint64_t c[3] = {0, 0, 0};
            sch.engine_consumed(e, &type, c);
            consumed_lo[e] = c[0];
            consumed_mid[e] = c[1];
        }
    }
    std::vector<uint64_t> tk(count), skip_lo(count, 0), skip_mid(count, 0), slot_of(count, 0);
    std::vector<int32_t> fin_ms_us(count);
    for (int i = 0; i < count; ++i) {
        tk[i] = ret[i] ? ~0ull : ticket[i];
        auto it = ex.refs_.find((uint64_t)i);
        if (it != ex.refs_.end()) {
            skip_lo[i] = it->second.skip[0];
            skip_mid[i] = it->second.skip[1];
            slot_of[i] = it->second.flags ? it->second.slot : ~0ull;
        }
        fin_ms_us[i] = (int32_t)std::lround(finish_ms[i] * 1000.0);
    }
    std::printf("{");
    print_ints("ret", ret);
    print_u64s("ticket", tk);
    print_ints("kind", kinds);
    print_u64s("n", ns);
    print_u64s("bytes", bytes);
    print_ints("expect", expect);
    print_ints("status", got);
    print_ints("finish_us", fin_ms_us);
    print_ints("engine", eng_of);
    print_u64s("skip_lo", skip_lo);
    print_u64s("skip_mid", skip_mid);
    print_u64s("ref_slot", slot_of);
    print_u64s("consumed_lo", consumed_lo);
    print_u64s("consumed_mid", consumed_mid);
    std::printf("\"skip_after\": %d, ", skip_after);
    std::printf("\"failed_launches\": [");
    for (size_t i = 0; i < ex.failed_.size(); ++i) std::printf("%s%d", i ? "," : "", ex.failed_[i]);
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
