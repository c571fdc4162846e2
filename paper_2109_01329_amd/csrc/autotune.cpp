// Autotuner: times candidate launch shapes on the caller's workload with
// HIP events and installs the fastest.  Candidates are measured in
// interleaved rounds after a pre-warm, so that clock ramp-up and drift do
// not favour whichever shape runs first; the score is the median round.
// Each measurement follows a few untimed launches of the same shape, so
// that it sees the steady state of back-to-back launches (a launch after
// an idle gap runs faster while the last-level cache absorbs its writes).
#include <algorithm>
#include <chrono>
#include <functional>
#include <vector>

#include "internal.hpp"

namespace {

constexpr int kWarm = 3;   // untimed launches before each measurement

// Time `reps` back-to-back calls of run(); ms per call, or < 0 on error.
float time_reps(const std::function<mirng_status()> &run, hipStream_t s, int reps,
                hipEvent_t a, hipEvent_t b)
{
    if (hipEventRecord(a, s) != hipSuccess) return -1.0f;
    for (int i = 0; i < reps; ++i)
        if (run() != MIRNG_OK) return -1.0f;
    if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return -1.0f;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0f;
    return ms / (float)reps;
}

// Generic tuner over `count` candidates; apply(i) installs candidate i.
// Returns the index of the best candidate, or -1 on failure.
int tune(size_t count, const std::function<void(size_t)> &apply,
         const std::function<mirng_status()> &run, hipStream_t s, int prewarm_ms, int rounds,
         int reps, float *best_ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return -1;
    }
    int best = -1;
    std::vector<std::vector<float>> t(count);
    const auto t0 = std::chrono::steady_clock::now();
    apply(0);
    bool ok = true;
    while (ok && std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                         .count() < prewarm_ms) {
        ok = time_reps(run, s, 4, a, b) >= 0.0f;
    }
    for (int r = 0; ok && r < rounds; ++r) {
        for (size_t i = 0; ok && i < count; ++i) {
            apply(i);
            for (int w = 0; ok && w < kWarm; ++w) ok = run() == MIRNG_OK;   // untimed
            const float ms = ok ? time_reps(run, s, reps, a, b) : -1.0f;
            ok = ms >= 0.0f;
            t[i].push_back(ms);
        }
    }
    if (ok) {
        float bms = 0.0f;
        for (size_t i = 0; i < count; ++i) {
            std::vector<float> v = t[i];
            std::sort(v.begin(), v.end());
            const float med = v[v.size() / 2];
            if (best < 0 || med < bms) {
                best = (int)i;
                bms = med;
            }
        }
        if (best_ms) *best_ms = bms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

// The Philox launch shapes the autotuner times, in timing order.
std::vector<mirng_philox_config> philox_candidates()
{
    std::vector<mirng_philox_config> cand;
    for (int block : {256, 512, 1024})
        for (int wpc : {64, 128, 256, 512, 1024})
            for (int nt : {0, 1}) cand.push_back({0, block, wpc, 1, nt, 0});
    for (int bpl : {1, 2}) cand.push_back({1, 256, 8, bpl, 0, 0});
    for (int block : {256, 1024})
        for (int iters : {1, 2, 4})
            for (int nt : {0, 1}) cand.push_back({2, block, 1, iters, nt, 0});
    for (int block : {128, 256, 512, 1024})
        for (int chunks : {1, 2})
            for (int nt : {0, 1}) cand.push_back({3, block, 1, chunks, nt, 0});
    return cand;
}

bool tune_args_ok(int32_t prewarm_ms, int32_t rounds, int32_t reps)
{
    return prewarm_ms >= 0 && prewarm_ms <= 60000 && rounds >= 1 && rounds <= 64 && reps >= 1 &&
           reps <= 10000;
}

}  // namespace

using namespace mirng;

extern "C" {

mirng_status mirng_autotune_philox(int32_t kind, uint64_t offset, uint64_t n, void *out,
                                   void *stream, int32_t prewarm_ms, int32_t rounds,
                                   int32_t reps, mirng_philox_config *best, float *best_ms)
{
    if (kind < kBits || kind > kIcdf64) return MIRNG_E_UNSUPPORTED;
    if (!out || n == 0 || !tune_args_ok(prewarm_ms, rounds, reps)) return MIRNG_E_INVALID_ARG;
    if ((uintptr_t)out % (uintptr_t)elem_bytes(kind)) return MIRNG_E_INVALID_ARG;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    const std::vector<mirng_philox_config> cand = philox_candidates();
    // every launch runs at the caller's position, so at its phase; the
    // result is installed for this kind at this phase only
    const int phase = (int)philox_phase(kind, offset, (uintptr_t)out);
    mirng_philox_config prev{};
    const bool had_own = philox_config_kind_set(kind, phase, &prev);
    mirng_engine e = nullptr;
    if (mirng_engine_create(MIRNG_PHILOX4X32_10, 0x5EED5EEDull, offset, &e) != MIRNG_OK)
        return MIRNG_E_ALLOC;
    mirng_state start;
    (void)mirng_engine_get_state(e, &start);
    // the unit range (or mean 0, sd 1); [0, 2^31) for uniform int32
    const mirng_distribution d = {kind, 0, 0.0, kind == kI32 ? 2147483648.0 : 1.0};
    auto run = [&]() {
        (void)mirng_engine_set_state(e, &start);
        return mirng_generate(e, &d, n, out, stream);
    };
    float ms = 0.0f;
    const int k = tune(cand.size(),
                       [&](size_t i) { philox_config_set_kind(kind, phase, &cand[i]); }, run,
                       (hipStream_t)stream, prewarm_ms, rounds, reps, &ms);
    mirng_engine_destroy(e);
    if (k < 0) {
        philox_config_set_kind(kind, phase, had_own ? &prev : nullptr);
        return MIRNG_E_LAUNCH;
    }
    // installed for this kind and phase only; other kinds and phases keep
    // their shapes
    philox_config_set_kind(kind, phase, &cand[k]);
    if (best) *best = cand[k];
    if (best_ms) *best_ms = ms;
    return MIRNG_OK;
}

int32_t mirng_philox_candidates(mirng_philox_config *out, int32_t max)
{
    const std::vector<mirng_philox_config> cand = philox_candidates();
    for (int32_t i = 0; out && i < max && i < (int32_t)cand.size(); ++i) out[i] = cand[(size_t)i];
    return (int32_t)cand.size();
}

mirng_status mirng_autotune_batch(mirng_batcher b, const mirng_request *reqs, size_t count,
                                  void *stream, int32_t prewarm_ms, int32_t rounds,
                                  int32_t reps, mirng_batch_config *best, float *best_ms)
{
    if (!b || !reqs || count == 0 || !tune_args_ok(prewarm_ms, rounds, reps))
        return MIRNG_E_INVALID_ARG;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    std::vector<mirng_batch_config> cand;
    for (int block : {256, 512, 1024})
        for (int wpc : {32, 64, 128, 256, 512})
            for (int nt : {0, 1}) cand.push_back({block, wpc, nt, 0});
    mirng_batch_config prev;
    if (mirng_batcher_config_get(b, &prev) != MIRNG_OK) return MIRNG_E_INVALID_ARG;
    auto run = [&]() { return mirng_generate_batch(b, reqs, count, stream); };
    float ms = 0.0f;
    const int k = tune(cand.size(), [&](size_t i) { (void)mirng_batcher_config_set(b, &cand[i]); },
                       run, (hipStream_t)stream, prewarm_ms, rounds, reps, &ms);
    if (k < 0) {
        (void)mirng_batcher_config_set(b, &prev);
        return MIRNG_E_LAUNCH;
    }
    (void)mirng_batcher_config_set(b, &cand[k]);
    if (best) *best = cand[k];
    if (best_ms) *best_ms = ms;
    return MIRNG_OK;
}

}  // extern "C"
