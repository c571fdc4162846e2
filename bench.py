#!/usr/bin/env python3
"""Benchmark of the mirng hot path on one MI355X.

Headline (one "step"): create a Philox4x32-10 engine at a bulk-workload seed
and offset and generate n = 2^28 uniform FP32 samples into a resident 1 GiB
device buffer -- the generator and output the paper measures (Philox4x32x10
uniform FP32 batches, arXiv:2109.01329 Sec. 7), at the bulk size.  `value`
is samples per second of those steps (Gsamples/s); the roofline object
prices the generation kernel's average duration (HIP events on the stream it
runs on) against HBM write bandwidth.

Also reported (one line, extra keys): every other engine x output cell of
the bulk workload at n = 2^28, MRG32k3a substreams (65536 x 4096 FP64),
the store-only and no-store ceilings, and the oracle timed on the host
cores over the same headline workload.

Before the W untimed warmup steps the headline step runs for --prewarm-s
seconds (default 0.4): the first ~100 launches of a fresh process run ~15%
slower while clocks ramp; the JSON line reports the pre-warm.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


# HBM bytes per launch of the headline kernel (uniform FP32, 2^28 samples at
# the bulk draw's phase 1) for every launch shape the autotuner can install
# (walk, block, waves per CU, blocks per lane, streaming stores):
# WRITE_SIZE x 1.0 + FETCH_SIZE x 2.0 (KiB, the second of two launches per
# shape), each factor being what the same counter reads for a plain 1 GiB
# device copy (WRITE 1048576 KiB, FETCH 524300 KiB).  Walks 1 and 2 at
# this phase write a little more than the 1 GiB of outputs (partial lines
# of 4-byte-aligned blocks and of 63-slot chunks).  Reset whenever the
# uniform FP32 kernels' code changes.
TRAFFIC_BY_SHAPE = {
    (0, 256, 64, 1, 0): 1073741824 + 89086,
    (0, 256, 64, 1, 1): 1073741824 + 89086,
    (0, 256, 128, 1, 0): 1073741824 + 89086,
    (0, 256, 128, 1, 1): 1073741824 + 89086,
    (0, 256, 256, 1, 0): 1073741824 + 89086,
    (0, 256, 256, 1, 1): 1073741824 + 89086,
    (0, 256, 512, 1, 0): 1073741824 + 89086,
    (0, 256, 512, 1, 1): 1073741824 + 89086,
    (0, 256, 1024, 1, 0): 1073741824 + 89086,
    (0, 256, 1024, 1, 1): 1073741824 + 89086,
    (0, 512, 64, 1, 0): 1073741824 + 89086,
    (0, 512, 64, 1, 1): 1073741824 + 89086,
    (0, 512, 128, 1, 0): 1073741824 + 89086,
    (0, 512, 128, 1, 1): 1073741824 + 89086,
    (0, 512, 256, 1, 0): 1073741824 + 89086,
    (0, 512, 256, 1, 1): 1073741824 + 89086,
    (0, 512, 512, 1, 0): 1073741824 + 89086,
    (0, 512, 512, 1, 1): 1073741824 + 89086,
    (0, 512, 1024, 1, 0): 1073741824 + 89086,
    (0, 512, 1024, 1, 1): 1073741824 + 89086,
    (0, 1024, 64, 1, 0): 1073741824 + 89086,
    (0, 1024, 64, 1, 1): 1073741824 + 89086,
    (0, 1024, 128, 1, 0): 1073741824 + 89086,
    (0, 1024, 128, 1, 1): 1073741824 + 89086,
    (0, 1024, 256, 1, 0): 1073741824 + 89086,
    (0, 1024, 256, 1, 1): 1073741824 + 89086,
    (0, 1024, 512, 1, 0): 1073741824 + 89086,
    (0, 1024, 512, 1, 1): 1073741824 + 89086,
    (0, 1024, 1024, 1, 0): 1073741824 + 89086,
    (0, 1024, 1024, 1, 1): 1073741824 + 89086,
    (1, 256, 8, 1, 0): 1073741824 + 18049183,
    (1, 256, 8, 2, 0): 1073741824 + 9550367,
    (2, 256, 1, 1, 0): 1073741824 + 66559,
    (2, 256, 1, 1, 1): 1073741824 + 66559,
    (2, 256, 1, 2, 0): 1073741824 + 93054,
    (2, 256, 1, 2, 1): 1073741824 + 180382,
    (2, 256, 1, 4, 0): 1073741824 + 1251390,
    (2, 256, 1, 4, 1): 1073741824 + 1269982,
    (2, 1024, 1, 1, 0): 1073741824 + 66559,
    (2, 1024, 1, 1, 1): 1073741824 + 66719,
    (2, 1024, 1, 2, 0): 1073741824 + 88926,
    (2, 1024, 1, 2, 1): 1073741824 + 96958,
    (2, 1024, 1, 4, 0): 1073741824 + 1666270,
    (2, 1024, 1, 4, 1): 1073741824 + 1676574,
    (3, 128, 1, 1, 0): 1073741824 + 69630,
    (3, 128, 1, 1, 1): 1073741824 + 69630,
    (3, 128, 1, 2, 0): 1073741824 + 84990,
    (3, 128, 1, 2, 1): 1073741824 + 84990,
    (3, 256, 1, 1, 0): 1073741824 + 69630,
    (3, 256, 1, 1, 1): 1073741824 + 69630,
    (3, 256, 1, 2, 0): 1073741824 + 84990,
    (3, 256, 1, 2, 1): 1073741824 + 84990,
    (3, 512, 1, 1, 0): 1073741824 + 69630,
    (3, 512, 1, 1, 1): 1073741824 + 69630,
    (3, 512, 1, 2, 0): 1073741824 + 84990,
    (3, 512, 1, 2, 1): 1073741824 + 84990,
    (3, 1024, 1, 1, 0): 1073741824 + 69630,
    (3, 1024, 1, 1, 1): 1073741824 + 69630,
    (3, 1024, 1, 2, 0): 1073741824 + 84990,
    (3, 1024, 1, 2, 1): 1073741824 + 84990,
}

# the kernel each walk of the plain Philox path launches
KERNEL_BY_WALK = {0: "philox_fill_kernel", 1: "philox_blocks_kernel", 2: "philox_chunk_kernel",
                  3: "philox_group_kernel"}


def traffic_for(cfg: dict):
    return TRAFFIC_BY_SHAPE.get((cfg["walk"], cfg["block"], cfg["waves_per_cu"],
                                 cfg["blocks_per_lane"], cfg["nontemporal"]))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--prewarm-s", type=float, default=0.4,
                   help="seconds of headline launches before the warmup steps, so that the "
                        "GPU's clocks reach their steady state under this load")
    p.add_argument("--quick", action="store_true", help="headline only")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    p.add_argument("--shape", default=None,
                   help="walk,block,waves_per_cu,blocks_per_lane,nontemporal: install this "
                        "Philox launch shape instead of autotuning")
    p.add_argument("--no-tune", action="store_true",
                   help="keep the library's default launch shape instead of autotuning it on "
                        "the headline workload before the timed region")
    p.add_argument("--profile", action="store_true",
                   help="for rocprofv3: 5 headline generate launches, then 3 device copies of "
                        "1 GiB (a plain copy kernel of known size for counter calibration)")
    p.add_argument("--profile-cells", action="store_true",
                   help="for rocprofv3 counters: every bulk cell and the substream cell, one "
                        "warm-up and one measured launch each, then the VALU-rate probe "
                        "(known instruction count) for calibration")
    p.add_argument("--profile-batch", action="store_true",
                   help="for rocprofv3: the calorimeter batch, 25 batches in a row")
    p.add_argument("--profile-scenario", default=None,
                   choices=("single_electron", "ttbar", "single_electron_min200k",
                            "single_electron_soa"),
                   help="for rocprofv3: one FastCaloSim-shaped scenario, 25 batches in a "
                        "row, then 5 plain launches of the same total")
    p.add_argument("--batch-shape", default=None,
                   help="block,waves_per_cu,nontemporal: the batch launch shape of "
                        "--profile-batch / --profile-scenario (default: the library's)")
    p.add_argument("--profile-shapes", action="store_true",
                   help="for rocprofv3 counters: the headline workload at every launch shape "
                        "the autotuner can install, two launches each (warm-up, measured), "
                        "then 3 device copies of 1 GiB for counter calibration")
    p.add_argument("--profile-mrg", action="store_true",
                   help="for rocprofv3 counters: MRG32k3a bits and uniform FP64, n = 2^28, "
                        "each into a 16-byte aligned and into a misaligned (one element "
                        "past) output, two launches each, then 3 device copies of 1 GiB for "
                        "counter calibration")
    return p.parse_args()


def copy_calibration(torch, stream, out, n, dev):
    """Three device copies of 1 GiB (1 GiB read, 1 GiB written) after the
    profiled launches: the kernel of known traffic that scales FETCH_SIZE
    and WRITE_SIZE."""
    with torch.cuda.stream(stream):
        src = torch.empty(n, dtype=torch.float32, device=dev)
        src.fill_(0.5)
        dst = out.view(torch.float32)[:n] if out.dtype != torch.float32 else out[:n]
        for _ in range(3):
            dst.copy_(src)
    torch.cuda.synchronize()


def time_region(fn, reps, stream, warm=3):
    """Average duration (ms) of `fn()` in steady state: `warm` untimed calls,
    then `reps` back-to-back calls between two HIP events on `stream`.  (A
    launch that follows an idle gap runs faster while the last-level cache
    absorbs part of its writes; back-to-back calls pay for that.)"""
    import torch
    for _ in range(warm):
        fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    stream.synchronize()
    return a.elapsed_time(b) / reps


def settle(fn, stream, seconds=0.03):
    """Calls `fn()` back to back for at least `seconds` of wall time (a few
    calls at a time, then a sync).  A cell's first tens of milliseconds after
    another workload ran measured a few percent slower (the chip's clocks
    adapt to the new mix), so every cell is timed after this."""
    import time
    t0 = time.perf_counter()
    while True:
        for _ in range(4):
            fn()
        stream.synchronize()
        if time.perf_counter() - t0 >= seconds:
            return


def time_kernel_calls(fn, reps, stream):
    """Average duration (ms) of `fn()` over `reps` calls, each bracketed by
    HIP events recorded on `stream` (the stream the kernels run on)."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    stream.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in evs)
    return sum(ts) / len(ts), ts[len(ts) // 2], ts[int(0.9 * (len(ts) - 1))]


def cpu_baseline(seed, offset, n, cells=None, n_mt=1 << 26, n_st=1 << 22):
    """The oracle over the full headline workload, split into consecutive
    slices over the host's cores (ctypes releases the GIL); and, per bulk
    cell, the oracle on n_mt outputs over all threads and on n_st outputs in
    one thread (MRG slices start from the oracle's own polynomial jump)."""
    import concurrent.futures
    import oracle
    threads = min(16, os.cpu_count() or 1)
    oracle.lib()

    def timed_split(engine, kind, s, o, total, nthreads):
        step = (total + nthreads - 1) // nthreads
        step += step % 2                        # Gaussian pairs stay whole
        start_state = oracle.mrg_skip(oracle.mrg_seed(s), o) if engine == oracle.MRG else None

        def one(first):
            m = min(step, total - first)
            skip = oracle.words_consumed(kind, engine, first)
            if engine == oracle.PHILOX:
                oracle.philox_generate(s, o + skip, kind, m)
            else:
                oracle.mrg_generate(oracle.mrg_skip(start_state, skip), kind, m)
            return m

        t0 = time.perf_counter()
        with concurrent.futures.ThreadPoolExecutor(max_workers=nthreads) as ex:
            done = sum(ex.map(one, range(0, total, step)))
        return done, time.perf_counter() - t0

    done, dt = timed_split(oracle.PHILOX, oracle.UNIFORM_F32, seed, offset, n, threads)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         model)
    except OSError:
        pass
    res = {"value": round(done / dt / 1e9, 4), "unit": "Gsamples/s", "cores": threads,
           "cpu_model": model, "host_cpus": os.cpu_count(),
           "kind": "oracle",
           "sample": f"full headline workload: {n} Philox4x32-10 uniform FP32 samples "
                     f"(seed/offset of the bulk draw), {threads} threads, {dt:.2f} s wall"}
    if cells:
        import synth
        per = {}
        for engine, kind, s, o in cells:
            name = f"{synth.ENGINE_NAME[engine]}/{synth.KIND_NAME[kind]}"
            # the oracle's inverse-CDF quantile is a bisection (about 64 erf
            # evaluations per output): a 64 times smaller sample
            shift = 6 if kind in (synth.GAUSSIAN_ICDF_F32, synth.GAUSSIAN_ICDF_F64) else 0
            d1, t1 = timed_split(engine, kind, s, o, n_mt >> shift, threads)
            d2, t2 = timed_split(engine, kind, s, o, n_st >> shift, 1)
            per[name] = {f"Gsamples_s_{threads}_threads": round(d1 / t1 / 1e9, 4),
                         "Gsamples_s_1_thread": round(d2 / t2 / 1e9, 4)}
        res["cells"] = per
        res["cells_sample"] = (f"each cell's seed/offset: {n_mt} outputs over {threads} "
                               f"threads, {n_st} outputs in 1 thread (64 times fewer for "
                               f"the inverse-CDF Gaussians)")
    return res


def calo_requests(mr, synth, torch, dev):
    """Calorimeter-shaped batch: 20000 events, per event 3h uniform FP32 at
    position 0 and h Gaussians at position 3h on key (42, event id), outputs
    contiguous per event in one device buffer."""
    import numpy as np
    ev = synth.calo_events()
    h = ev.hits.astype(np.uint64)
    sizes = np.stack([3 * h, h], axis=1).reshape(-1)
    total = int(sizes.sum())
    out = torch.empty(total, dtype=torch.float32, device=dev)
    offs = np.concatenate([[0], np.cumsum(sizes * 4)])[:-1].astype(np.uint64)
    seeds = (np.arange(ev.n_events, dtype=np.uint64) << np.uint64(32)) | np.uint64(ev.seed32)
    reqs = mr.make_requests(2 * ev.n_events)
    reqs["engine_type"] = 1
    reqs["kind"] = np.tile([mr.UNIFORM_F32, mr.GAUSSIAN_F32], ev.n_events)
    reqs["p1"] = 1.0
    reqs["seed"] = np.repeat(seeds, 2)
    reqs["offset"] = np.stack([np.zeros_like(h), 3 * h], axis=1).reshape(-1)
    reqs["n"] = sizes
    reqs["out"] = np.uint64(out.data_ptr()) + offs
    return ev, reqs, out, total


def calo_batch_leg(mr, synth, torch, stream, dev, reps=20, tune=True, windows=5, per_window=40):
    """The calorimeter batch in one batched launch per batch.  Reports the
    autotuned shape, pipelined throughput (median of several windows of
    back-to-back batches, wall clock), per-batch GPU time, per-batch latency
    (enqueue to completion) and the plain path on the same mix (one uniform
    and one Gaussian launch of the same totals)."""
    import numpy as np
    ev, reqs, out, total = calo_requests(mr, synth, torch, dev)
    b = mr.Batcher()
    tuned = None
    if tune:
        t0 = time.perf_counter()
        cfg, tms = b.autotune(reqs, stream=stream, prewarm_ms=200, rounds=3, reps=5)
        tuned = {"config": cfg.as_dict(), "ms": round(tms, 4),
                 "tuning_s": round(time.perf_counter() - t0, 3)}
    for _ in range(5):
        b.generate(reqs, stream=stream)
    stream.synchronize()
    wins = []
    for _ in range(windows):
        t0 = time.perf_counter()
        for _ in range(per_window):
            b.generate(reqs, stream=stream)
        stream.synchronize()
        wins.append((time.perf_counter() - t0) * 1e3 / per_window)
    wins.sort()
    ms_pipe = wins[len(wins) // 2]
    gpu_ms = time_region(lambda: b.generate(reqs, stream=stream), reps, stream)
    lat = []
    for _ in range(reps):
        t1 = time.perf_counter()
        b.generate(reqs, stream=stream)
        stream.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat.sort()
    assert np.all(b.statuses(len(reqs)) == 0)
    n_u, n_g = int(3 * ev.hits.sum()), int(ev.hits.sum())

    def plain():
        mr.Engine(mr.PHILOX4X32_10, 42, 0).generate(mr.UNIFORM_F32, n_u, out, stream=stream)
        mr.Engine(mr.PHILOX4X32_10, 43, 0).generate(mr.GAUSSIAN_F32, n_g, out, stream=stream)

    plain()
    plain_ms = time_region(plain, reps, stream)
    return {"events": ev.n_events, "requests": len(reqs), "samples": total,
            "bytes": total * 4, "config": b.config.as_dict(), "autotune": tuned,
            "ms_per_batch_pipelined": round(ms_pipe, 4),
            "pipelined_windows_ms": [round(w, 4) for w in wins],
            "Gsamples_s": round(total / (ms_pipe * 1e-3) / 1e9, 1),
            "gpu_ms_per_batch": round(gpu_ms, 4),
            "latency_ms": {"p50": round(lat[len(lat) // 2], 4),
                           "p99": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 4)},
            "plain_same_mix_ms": round(plain_ms, 4),
            "batch_over_plain_time": round(ms_pipe / plain_ms, 3)}


def scenario_requests(mr, sc, torch, dev):
    """The Philox uniform FP32 requests of scenario `sc` (its own request
    description: per event, or per event and quantity), with outputs in one
    device buffer.  Returns (requests, buffer, total samples)."""
    import numpy as np
    seeds, offsets, sizes, first = sc.requests()
    total = int(sizes.sum())
    out = torch.empty(total, dtype=torch.float32, device=dev)
    reqs = mr.make_requests(sizes.size)
    reqs["engine_type"] = mr.PHILOX4X32_10
    reqs["kind"] = mr.UNIFORM_F32
    reqs["p1"] = 1.0
    reqs["seed"] = seeds
    reqs["offset"] = offsets
    reqs["n"] = sizes
    reqs["out"] = np.uint64(out.data_ptr()) + first * np.uint64(4)
    return reqs, out, total


def scenario_leg(mr, synth, torch, stream, dev):
    """FastCaloSim-shaped event batches (the paper's Sec. 5.2 scenarios):
    single-electron events (10^4 events of 4000-6500 hits) and ttbar events
    (500 events of 600-800 times as many hits), three uniform FP32 per hit,
    one Philox request per event on key (42, event id), outputs contiguous
    per event; and two single-electron variants: at least 200,000 uniforms
    per event, and one request per event and quantity into three arrays
    (SoA).  Each scenario is one batch (launch shape autotuned on it
    first), timed in steady state, against the plain path generating the
    same total in one launch."""
    import numpy as np
    res = {}
    for name, reps in (("single_electron", 20), ("ttbar", 5), ("single_electron_min200k", 10),
                       ("single_electron_soa", 20)):
        sc = synth.calo_scenario(name)
        reqs, out, total = scenario_requests(mr, sc, torch, dev)
        b = mr.Batcher()
        cfg, _ = b.autotune(reqs, stream=stream, prewarm_ms=200, rounds=3, reps=5)
        batch_ms = time_region(lambda: b.generate(reqs, stream=stream), reps, stream)
        assert np.all(b.statuses(reqs.size) == 0)
        e = mr.Engine(mr.PHILOX4X32_10, 42, 0)
        plain_ms = time_region(lambda: e.generate(mr.UNIFORM_F32, total, out, stream=stream),
                               reps, stream)
        res[name] = {"events": sc.n_events, "requests": int(reqs.size), "samples": total,
                     "bytes": total * 4,
                     "batch_config": cfg.as_dict(),
                     "batch_ms": round(batch_ms, 4),
                     "batch_GBs": round(total * 4 / (batch_ms * 1e-3) / 1e9, 1),
                     "plain_ms": round(plain_ms, 4),
                     "batch_over_plain_time": round(batch_ms / plain_ms, 3)}
        b.close()
        del out
    return res


def serve_leg(mr, synth, torch, dev, cells=None, counts=(10500, 20000, 20000), streams=4,
              capacity=32 * 10**9, ring_gib=64, engines_per_type=512):
    """Serving loop under open-loop Poisson arrivals at 1e3, 1e4 and 1e5
    requests/s (`counts` requests each, at least 10 s of arrivals at 1e3/s):
    sizes floor(10^U(3, 8)), engine type and distribution uniform over the
    2 x 4 mix.  Engine states are resident on the device: each server holds
    `engines_per_type` engines of each type (seeds uint64, offsets in
    [0, 2^40)), and every request continues an engine of its type drawn
    uniformly.  Latency runs from each request's scheduled arrival to its
    completion.  Outputs go to a ring of `ring_gib` GiB of device memory
    (placed in arrival order, 256-byte aligned).  Reports completed
    throughput (samples / span), p50/p99 latency overall and by size decade
    and, when the bulk cells were measured, the plain path's rate on the
    same mix."""
    import numpy as np
    ring_bytes = ring_gib << 30
    ring = torch.empty(ring_bytes, dtype=torch.uint8, device=dev)
    base = int(ring.data_ptr())

    def requests(rate, count, k):
        tr = synth.request_trace(rate, count, k=k)
        reqs = mr.make_requests(count)
        reqs["engine_type"] = tr.engine
        reqs["kind"] = tr.kind
        reqs["p1"] = 1.0
        reqs["seed"] = tr.seed
        reqs["offset"] = tr.offset
        reqs["n"] = tr.n
        esz = np.where(tr.kind == mr.UNIFORM_F64, 8, 4).astype(np.int64)
        size = (tr.n * esz + 255) // 256 * 256
        out = np.empty(count, dtype=np.uint64)
        pos = 0
        for i in range(count):
            if pos + int(size[i]) > ring_bytes:
                pos = 0
            out[i] = base + pos
            pos += int(size[i])
        reqs["out"] = out
        return tr, reqs

    def run(rate, count, k):
        tr, reqs = requests(rate, count, k)
        srv = mr.Server(streams=streams, capacity_bytes=capacity, max_batch=65536,
                        max_engines=2 * engines_per_type)
        g = np.random.default_rng(1329 + 500 + k)
        pool = {}
        for et in (mr.PHILOX4X32_10, mr.MRG32K3A):
            seeds = g.integers(0, 2**64, engines_per_type, dtype=np.uint64)
            offs = g.integers(0, 2**40, engines_per_type, dtype=np.uint64)
            pool[et] = np.array([srv.engine_create(et, int(a), int(b))
                                 for a, b in zip(seeds, offs)], dtype=np.uint32)
        pick = g.integers(0, engines_per_type, count)
        eng = np.where(tr.engine == mr.PHILOX4X32_10, pool[mr.PHILOX4X32_10][pick],
                       pool[mr.MRG32K3A][pick]).astype(np.uint32)
        tickets, sub = srv.replay(reqs, tr.arrival_s, engines=eng)
        srv.drain()
        lat = np.array([srv.wait(int(x))[1] for x in tickets])
        st = srv.stats()
        srv.close()
        assert np.all(sub == 0) and st["failed"] == 0
        return tr, st, lat

    def pct(v, q):
        v = np.sort(v)
        return float(v[max(0, int(np.ceil(q * len(v))) - 1)])

    run(1e4, 400, 50)                      # warm-up: tables, staging memory
    res = {}
    for i, (rate, count) in enumerate(zip((1e3, 1e4, 1e5), counts)):
        tr, st, lat = run(rate, count, 51 + i)
        samples = int(tr.n.sum())
        dec = np.floor(np.log10(tr.n)).astype(int)
        by_dec = {f"1e{d}": {"requests": int((dec == d).sum()),
                             "p50": round(pct(lat[dec == d], 0.5), 3),
                             "p99": round(pct(lat[dec == d], 0.99), 3)}
                  for d in range(3, 8) if (dec == d).any()}
        row = {"requests": count, "samples": samples,
               "offered_Gsamples_s": round(samples / max(tr.arrival_s[-1], 1e-9) / 1e9, 1),
               "served_Gsamples_s": round(st["samples"] / st["span_s"] / 1e9, 1),
               "latency_ms": {"p50": round(st["latency_p50_ms"], 3),
                              "p99": round(st["latency_p99_ms"], 3),
                              "max": round(st["latency_max_ms"], 3)},
               "latency_ms_by_size_decade": by_dec,
               "batches": st["batches"], "span_s": round(st["span_s"], 4),
               "max_inflight_GB": round(st["max_inflight_bytes"] / 1e9, 2)}
        if cells:
            t_plain = 0.0
            for e, kd, n in zip(tr.engine, tr.kind, tr.n):
                c = cells[f"{synth.ENGINE_NAME[int(e)]}/{synth.KIND_NAME[int(kd)]}"]
                t_plain += float(n) / (c["Gsamples_s"] * 1e9)
            plain = samples / t_plain / 1e9
            row["plain_same_mix_Gsamples_s"] = round(plain, 1)
            row["served_over_plain"] = round(row["served_Gsamples_s"] / plain, 3)
        res[f"{int(rate)}_per_s"] = row
    del ring
    return {"streams": streams, "capacity_GB": capacity / 1e9,
            "resident_engines": 2 * engines_per_type, "rates": res}


def tts_leg(mr, torch, iters=100, decades=range(0, 9)):
    """The paper's RNG burner on this GPU (Sec. 5.1, Sec. 7): per batch size
    n = 10^0 .. 10^8, `iters` iterations of the whole flow, each timed on
    the host clock: host and device allocation, generator construction and
    seeding, Philox4x32-10 uniform FP32 generation, synchronisation, copy of
    the output to host memory, release.  Run once with this library and once
    with the installed rocRAND (public host API, as a black box), the
    vendor-native side of the paper's comparison.  Also the device-only time
    of the generation call (HIP events).  Reports medians in ms and the
    ratio TTS_rocrand / TTS_mirng (above 1: this library is faster)."""
    import ctypes
    import numpy as np
    hip = ctypes.CDLL("libamdhip64.so")     # the runtime torch has loaded
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipDeviceSynchronize.argtypes = []
    D2H = 2
    lib_path = "/opt/rocm/lib/librocrand.so"
    vendor = ctypes.CDLL(lib_path) if os.path.exists(lib_path) else None
    if vendor is not None:
        vendor.rocrand_create_generator.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
        vendor.rocrand_set_seed.argtypes = [ctypes.c_void_p, ctypes.c_ulonglong]
        vendor.rocrand_generate_uniform.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_size_t]
        vendor.rocrand_destroy_generator.argtypes = [ctypes.c_void_p]
    PHILOX_VENDOR = 404                       # ROCRAND_RNG_PSEUDO_PHILOX4_32_10

    def flow_mirng(n):
        host = np.empty(n, dtype=np.float32)
        d = ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(d), n * 4) == 0
        e = mr.Engine(mr.PHILOX4X32_10, 1234, 0)
        e.generate(mr.UNIFORM_F32, n, d.value)
        assert hip.hipMemcpy(host.ctypes.data, d, n * 4, D2H) == 0
        e.close()
        hip.hipFree(d)
        return host

    def flow_vendor(n):
        host = np.empty(n, dtype=np.float32)
        d = ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(d), n * 4) == 0
        g = ctypes.c_void_p()
        assert vendor.rocrand_create_generator(ctypes.byref(g), PHILOX_VENDOR) == 0
        assert vendor.rocrand_set_seed(g, 1234) == 0
        assert vendor.rocrand_generate_uniform(g, d, n) == 0
        assert hip.hipMemcpy(host.ctypes.data, d, n * 4, D2H) == 0
        vendor.rocrand_destroy_generator(g)
        hip.hipFree(d)
        return host

    def tts(flow, n):
        flow(n)
        ts = []
        for _ in range(iters):
            t0 = time.perf_counter()
            flow(n)
            ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts)), len(ts)

    def device_only(n):
        buf = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        s = torch.cuda.current_stream()
        e = mr.Engine(mr.PHILOX4X32_10, 1234, 0)
        e.generate(mr.UNIFORM_F32, n, buf, stream=s)
        return time_kernel_calls(lambda: e.generate(mr.UNIFORM_F32, n, buf, stream=s), 20, s)[1]

    rows = {}
    eff = []
    for dcd in decades:
        n = 10 ** dcd
        ours, k = tts(flow_mirng, n)
        row = {"tts_ms_mirng": round(ours, 4), "iterations": k,
               "device_ms_mirng": round(device_only(n), 4)}
        if vendor is not None:
            theirs, _ = tts(flow_vendor, n)
            row["tts_ms_rocrand"] = round(theirs, 4)
            row["rocrand_over_mirng"] = round(theirs / ours, 3)
            eff.append(theirs / ours)
        rows[f"1e{dcd}"] = row
    res = {"by_size": rows}
    if eff:
        # one efficiency for this platform: the harmonic mean over the sizes
        # of e(n) = TTS_native / TTS_portable (above 1: this library faster),
        # the form of the paper's performance-portability mean (eq. 1)
        res["efficiency_harmonic_mean"] = round(len(eff) / sum(1.0 / e for e in eff), 3)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path "
              "shards by counter ranges with no exchange, see the design notes", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2109_01329_amd as mr
    import synth

    mr.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream()
    n = synth.BULK_N
    cells = synth.bulk_draws(count=1)
    head = [c for c in cells if c[0] == mr.PHILOX4X32_10 and c[1] == mr.UNIFORM_F32][0]
    _, _, seed, offset = head
    out = torch.empty(n, dtype=torch.float32, device=dev)
    phase = mr.philox_phase(mr.UNIFORM_F32, offset, out)

    def step():
        e = mr.Engine(mr.PHILOX4X32_10, seed, offset)
        e.generate(mr.UNIFORM_F32, n, out, stream=stream)
        return e

    if args.shape:
        walk, blk, wpc, bpl, nt = (int(x) for x in args.shape.split(","))
        mr.set_philox_config(walk=walk, block=blk, waves_per_cu=wpc, blocks_per_lane=bpl,
                             nontemporal=nt)

    if args.profile_cells:
        big = torch.empty(n * 2, dtype=torch.float32, device=dev)
        order = []
        for engine, kind, s, o in cells + synth.extra_draws():
            for _ in range(2):
                mr.Engine(engine, s, o).generate(kind, n, big, stream=stream)
            order.append(f"{synth.ENGINE_NAME[engine]}/{synth.KIND_NAME[kind]}")
        cfg = synth.SUBSTREAMS
        for _ in range(2):
            mr.Engine(mr.MRG32K3A, synth.substream_seed(), 0).generate_substreams(
                mr.UNIFORM_F64, 0, cfg["count"], cfg["per_stream"], big, stream=stream)
        order.append("mrg32k3a/substreams_65536x4096_f64")
        vsink = torch.empty(256 * 4096, dtype=torch.int32, device=dev)
        for _ in range(2):
            mr.bench_valu(4, 256 * 4096, 256, vsink, stream)
        order.append("valu probe fma_f32: 1048576 lanes x 256 iterations x 8 FMAs")
        stream.synchronize()
        print(json.dumps({"profile": "cells, two launches each (warm-up, measured)",
                          "order": order,
                          "config": mr.philox_config(mr.UNIFORM_F32, phase).as_dict()}),
              flush=True)
        return

    def batcher():
        b = mr.Batcher()
        if args.batch_shape:
            blk, wpc, nt = (int(x) for x in args.batch_shape.split(","))
            b.set_config(block=blk, waves_per_cu=wpc, nontemporal=nt)
        return b

    if args.profile_shapes:
        order = []
        for c in mr.philox_candidates():
            mr.set_philox_config(kind=mr.UNIFORM_F32, phase=phase, **c.as_dict())
            for _ in range(2):
                step()
            order.append(c.as_dict())
        copy_calibration(torch, stream, out, n, dev)
        print(json.dumps({"profile": "headline workload at every autotuner shape, two launches "
                                     "each (warm-up, measured), then 1 GiB copy x3",
                          "phase": phase, "order": order}), flush=True)
        return

    if args.profile_mrg:
        big = torch.empty(2 * n + 4, dtype=torch.int32, device=dev)
        e = mr.Engine(mr.MRG32K3A, 0x9E3779B97F4A7C15, 12345)
        for kind, offs in ((mr.BITS_U32, (0, 4)), (mr.UNIFORM_F64, (0, 8))):
            for off in offs:
                for _ in range(2):
                    e.generate(kind, n, int(big.data_ptr()) + off, stream=stream)
        copy_calibration(torch, stream, out, n, dev)
        print(json.dumps({"profile": "MRG32k3a n=2^28: bits aligned x2, 4 bytes past "
                                     "alignment x2, uniform FP64 aligned x2, 8 bytes past x2, "
                                     "then 1 GiB copy x3"}), flush=True)
        return

    if args.profile_batch:
        _, reqs, _, total = calo_requests(mr, synth, torch, dev)
        b = batcher()
        for _ in range(25):
            b.generate(reqs, stream=stream)
        stream.synchronize()
        print(json.dumps({"profile": f"calorimeter batch ({len(reqs)} requests, {total} "
                                     "samples) x25", "config": b.config.as_dict()}), flush=True)
        return

    if args.profile_scenario:
        import numpy as np
        sc = synth.calo_scenario(args.profile_scenario)
        reqs, out, total = scenario_requests(mr, sc, torch, dev)
        b = batcher()
        for _ in range(25):
            b.generate(reqs, stream=stream)
        e = mr.Engine(mr.PHILOX4X32_10, 42, 0)
        for _ in range(5):
            e.generate(mr.UNIFORM_F32, total, out, stream=stream)
        stream.synchronize()
        assert np.all(b.statuses(reqs.size) == 0)
        print(json.dumps({"profile": f"{sc.name} batch ({reqs.size} requests, {total} "
                                     "samples) x25, then plain x5",
                          "config": b.config.as_dict()}), flush=True)
        return

    if args.profile:
        with torch.cuda.stream(stream):
            for _ in range(5):
                step()
            src = torch.empty(n, dtype=torch.float32, device=dev)
            src.fill_(0.5)
            for _ in range(3):
                out.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "philox uniform_f32 n=2^28 x5, then 1 GiB copy x3",
                          "phase": phase,
                          "config": mr.philox_config(mr.UNIFORM_F32, phase).as_dict()}),
              flush=True)
        return

    # launch shape: the library's autotuner on this workload (outside the
    # timed region; only speed depends on the shape)
    tuned = None
    if not args.shape and not args.no_tune:
        t_tune = time.perf_counter()
        cfg, tms = mr.autotune_philox(mr.UNIFORM_F32, n, out, stream=stream, prewarm_ms=300,
                                      rounds=3, reps=30, offset=offset)
        tuned = {"config": cfg.as_dict(), "ms": round(tms, 4),
                 "tuning_s": round(time.perf_counter() - t_tune, 3)}

    # clock ramp: the first ~100 launches of a fresh process run ~15% slower
    t_pre = time.perf_counter()
    launches = 0
    while time.perf_counter() - t_pre < args.prewarm_s:
        step()
        launches += 1
        if launches % 8 == 0:
            stream.synchronize()
    stream.synchronize()
    prewarm = {"seconds": round(time.perf_counter() - t_pre, 3), "launches": launches}

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
        stream.synchronize()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            step()
        ev1.record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = n / (wall / args.steps) / 1e9

    # The step is one launch of the dominant kernel: its average duration is
    # the event time over the timed region on the launch stream / steps.
    avg_ms = ev0.elapsed_time(ev1) / args.steps
    # per-launch brackets (an event pair around every launch) for the spread
    b_avg, b_med, b_p90 = time_kernel_calls(step, 50, stream)
    bytes_per_launch = n * 4
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_for(mr.philox_config(mr.UNIFORM_F32, phase).as_dict()),
                "kernel": (KERNEL_BY_WALK[mr.philox_config(mr.UNIFORM_F32, phase).walk]
                           + "<uniform_f32>"),
                "kernel_ms": {"avg": round(avg_ms, 4),
                              "bracketed_avg": round(b_avg, 4), "bracketed_median": round(b_med, 4),
                              "bracketed_p90": round(b_p90, 4)},
                "algorithmic_bytes_per_launch": bytes_per_launch}

    extra = {}
    if not args.quick:
        # ceilings on the same GPU
        buf = torch.empty(n * 4, dtype=torch.uint8, device=dev)
        st_ms = time_region(lambda: mr.bench_store(buf, n * 4, True, stream), 30, stream)
        st2_ms = time_region(lambda: mr.bench_store(buf, n * 4, False, stream), 30, stream)
        sink = torch.empty(n // 4 // 64 + 64, dtype=torch.int32, device=dev)
        ns_ms = time_kernel_calls(lambda: mr.bench_philox_nostore(n // 4, sink, stream=stream),
                                  20, stream)[0]
        with torch.cuda.stream(stream):
            fill_ms = time_region(lambda: buf.zero_(), 30, stream)
        fill_gbs = n * 4 / (fill_ms * 1e-3) / 1e9
        store_gbs = n * 4 / (min(st_ms, st2_ms) * 1e-3) / 1e9
        extra["ceilings"] = {
            "runtime_fill_GBs": round(fill_gbs, 1),
            "store_only_nt_GBs": round(n * 4 / (st_ms * 1e-3) / 1e9, 1),
            "store_only_GBs": round(n * 4 / (st2_ms * 1e-3) / 1e9, 1),
            "philox_nostore_Gsamples_s": round(n / (ns_ms * 1e-3) / 1e9, 1),
            # the headline kernel against the measured write ceilings
            "headline_frac_of_runtime_fill": round(achieved / fill_gbs, 4),
            "headline_frac_of_store_only": round(achieved / store_gbs, 4),
        }
        vsink = torch.empty(256 * 4096, dtype=torch.int32, device=dev)
        rates = {}
        for op, name in [(0, "mad_u64_u32"), (1, "xor_b32"), (2, "fma_f64"), (3, "floor_f64"),
                         (4, "fma_f32")]:
            threads, iters = 256 * 4096, 256
            ms = time_kernel_calls(lambda: mr.bench_valu(op, threads, iters, vsink, stream), 5,
                                   stream)[0]
            rates[name + "_Gops_s"] = round(threads * iters * 8 / (ms * 1e-3) / 1e9, 1)
        extra["valu_rates"] = rates
        # the VALU probes leave the clocks low for a while: half a second of
        # headline launches before the first cell (measured 0.182-0.190 ms
        # for the uniform FP32 cell right after the probes, against
        # 0.160-0.173 for the same launch in the timed region)
        t_pre = time.perf_counter()
        k = 0
        while time.perf_counter() - t_pre < 0.5:
            step()
            k += 1
            if k % 8 == 0:
                stream.synchronize()
        stream.synchronize()
        # every bulk cell
        res = {}
        big = torch.empty(n * 2, dtype=torch.float32, device=dev)   # 2 GiB
        for engine, kind, s, o in cells + synth.extra_draws():
            name = f"{synth.ENGINE_NAME[engine]}/{synth.KIND_NAME[kind]}"
            if engine == mr.PHILOX4X32_10 and kind != mr.UNIFORM_F32:
                # each Philox kind at its own tuned launch shape (uniform
                # FP32 was tuned on the headline workload above)
                mr.autotune_philox(kind, n, big, stream=stream, prewarm_ms=100, rounds=3,
                                   reps=5, offset=o)

            def gen(engine=engine, kind=kind, s=s, o=o):
                mr.Engine(engine, s, o).generate(kind, n, big, stream=stream)

            settle(gen, stream)
            ms = time_region(gen, 20, stream)
            nbytes = n * synth.ELEM_BYTES[kind]
            res[name] = {"ms": round(ms, 4), "Gsamples_s": round(n / (ms * 1e-3) / 1e9, 1),
                         "GBs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                         "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            if engine == mr.PHILOX4X32_10:
                ph = mr.philox_phase(kind, o, big)
                res[name]["phase"] = ph
                res[name]["config"] = mr.philox_config(kind, ph).as_dict()
        cfg = synth.SUBSTREAMS
        e = mr.Engine(mr.MRG32K3A, synth.substream_seed(), 0)

        def subs():
            e.generate_substreams(mr.UNIFORM_F64, 0, cfg["count"], cfg["per_stream"], big,
                                  stream=stream)

        settle(subs, stream)
        ms = time_region(subs, 20, stream)
        tot = cfg["count"] * cfg["per_stream"]
        res["mrg32k3a/substreams_65536x4096_f64"] = {
            "ms": round(ms, 4), "Gsamples_s": round(tot / (ms * 1e-3) / 1e9, 1),
            "GBs": round(tot * 8 / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(tot * 8 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        extra["cells"] = res
        del big, buf
        extra["batched"] = calo_batch_leg(mr, synth, torch, stream, dev)
        extra["fastcalosim_scenarios"] = scenario_leg(mr, synth, torch, stream, dev)
        extra["serving"] = serve_leg(mr, synth, torch, dev, cells=res)
        extra["burner_tts"] = tts_leg(mr, torch)

    line = {
        "metric": "Gsamples/s + HBM write GB/s (% peak), Philox FP32 uniform n=2^28; batched p99 ms",
        "value": round(value, 2),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "philox4x32_10 uniform_f32 n=2^28, seed/offset from the bulk "
                               "draw (offset uniform in [0, 2^40))",
                   "n": n, "seed": seed, "offset": offset, "phase": phase,
                   "parallelism": "single GPU"},
        "write_GBs": round(n * 4 / (ms_per_step * 1e-3) / 1e9, 1),
        "hbm_write_frac": round(n * 4 / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "prewarm": prewarm,
        "philox_config": mr.philox_config(mr.UNIFORM_F32, phase).as_dict(),
        "autotune": tuned,
    }
    line.update(extra)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(
            seed, offset, n, cells=None if args.quick else cells + synth.extra_draws())
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
