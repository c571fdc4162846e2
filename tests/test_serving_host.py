"""Host-only tests of the serving loop's scheduling policy (admission by
in-flight bytes, arrival-order continuous batching onto free streams, one
batch per stream, completion per stream as soon as its batch is done, a
batch whose launch fails, resident-engine positions assigned in arrival
order, completion statuses and latency statistics), driven by a simulated
executor: the scheduler source is compiled with g++ together with
tests/native/sched_fake.cpp, no HIP involved."""
import json
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2109_01329_amd", "csrc")


@pytest.fixture(scope="module")
def fake(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "sched_fake")
    cmd = ["g++", "-std=c++17", "-O1", "-Wall", "-pthread", f"-I{ROOT}/include", f"-I{CSRC}",
           os.path.join(ROOT, "tests", "native", "sched_fake.cpp"),
           os.path.join(CSRC, "scheduler.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)

    def run(slots=2, capacity=10**6, max_batch=64, ns_per_byte=1.0, base_us=20.0, count=300,
            gap_us=0.0, seed=1, max_n=10**4, mode="random", slot0_factor=1.0, fail_at=()):
        args = [exe, mode, str(slots), str(capacity), str(max_batch), str(ns_per_byte),
                str(base_us), str(count), str(gap_us), str(seed), str(max_n), str(slot0_factor)]
        if fail_at:
            args.append(",".join(str(x) for x in fail_at))
        out = subprocess.run(args, check=True, capture_output=True, text=True, timeout=120)
        return json.loads(out.stdout)
    return run


ELEM = {1: 4, 2: 4, 3: 8, 4: 4, 5: 8, 6: 4, 7: 4, 8: 8}


def _common(d, slots, capacity, max_batch, failed_batches=()):
    ret = np.array(d["ret"])
    bytes_ = np.array(d["bytes"])
    # admission counts n x element size, 0 for requests the kernel refuses
    for k, n, b in zip(d["kind"], d["n"], d["bytes"]):
        assert b == (n * ELEM[k] if k in ELEM and n < 2**32 else 0), (k, n, b)
    acc = np.nonzero(ret == 0)[0]
    # refused exactly when the request alone exceeds the capacity
    assert np.array_equal(ret != 0, bytes_ > capacity)
    assert np.all(ret[ret != 0] == 6)
    # every accepted request completed with the status the kernel gives, or
    # MIRNG_E_LAUNCH exactly when its batch's launch failed
    expect = np.array(d["expect"])
    for b in failed_batches:
        for t in d["batches"][b]:
            expect[acc[t]] = 4
    assert np.array_equal(np.array(d["status"])[acc], expect[acc])
    # batches in arrival order, each request exactly once
    order = [t for b in d["batches"] for t in b]
    assert order == sorted(order) == list(range(len(acc)))
    assert all(1 <= len(b) <= max_batch for b in d["batches"])
    assert not d["double_launch"] and d["max_concurrent"] <= slots
    s = d["stats"]
    assert s["submitted"] == len(acc) and s["completed"] == len(acc)
    assert s["refused"] == int((ret != 0).sum())
    assert s["max_inflight_bytes"] <= capacity
    assert s["failed"] == int((expect[acc] != 0).sum())
    ok = acc[expect[acc] == 0]
    assert s["bytes"] == int(bytes_[ok].sum())
    assert 0.0 <= s["p50"] <= s["p99"] <= s["max"]
    assert d["binds"] == 1 + slots      # dispatcher and one completion thread per slot


@pytest.mark.parametrize("slots,capacity,max_batch", [(1, 10**5, 8), (2, 2 * 10**5, 64),
                                                      (4, 10**6, 1024), (3, 30000, 3)])
def test_policy_invariants(fake, slots, capacity, max_batch):
    d = fake(slots=slots, capacity=capacity, max_batch=max_batch, count=400, seed=slots)
    _common(d, slots, capacity, max_batch)


def test_capacity_bounds_inflight_and_refuses_oversized(fake):
    d = fake(slots=4, capacity=20000, max_batch=64, count=300, max_n=10**4, seed=5)
    _common(d, 4, 20000, 64)
    assert d["stats"]["refused"] > 0
    assert d["stats"]["max_inflight_bytes"] > 0


def test_burst_is_batched_continuously(fake):
    # a slow executor and a burst of arrivals: waiting requests merge into
    # few large batches instead of one launch each
    d = fake(slots=2, capacity=10**9, max_batch=4096, ns_per_byte=2.0, base_us=500.0,
             count=600, max_n=2000, seed=7)
    _common(d, 2, 10**9, 4096)
    assert len(d["batches"]) <= 60


def test_sparse_arrivals_run_alone(fake):
    # arrivals far apart relative to the service time: one request per batch
    d = fake(slots=2, capacity=10**9, max_batch=4096, ns_per_byte=0.01, base_us=5.0,
             count=60, gap_us=2000.0, max_n=1000, seed=9)
    _common(d, 2, 10**9, 4096)
    assert len(d["batches"]) >= 50
    assert d["stats"]["p50"] < 2.0


def test_max_batch_one(fake):
    d = fake(slots=3, capacity=10**9, max_batch=1, count=120, seed=11)
    _common(d, 3, 10**9, 1)
    assert len(d["batches"]) == d["stats"]["submitted"]


def test_slot_completes_independently(fake):
    """Slot 0 runs its batches 200 times slower than slot 1.  Requests that
    go to slot 1 complete (and free their slot) while slot 0's batch is
    still running: completion is per stream, not in launch order."""
    d = fake(slots=2, capacity=10**9, max_batch=1, ns_per_byte=0.0, base_us=1000.0,
             count=12, gap_us=8000.0, max_n=100, slot0_factor=200.0, seed=13)
    _common(d, 2, 10**9, 1)
    fin = np.array(d["finish_us"]) / 1000.0          # ms from the start
    # request 0 takes slot 0 for ~200 ms; requests 1.. arrive 8 ms apart,
    # each finds slot 1 free and finishes ~1 ms later
    assert fin[0] > 150.0
    early = fin[1:12] < fin[0]
    assert early.sum() >= 10, fin
    lat = fin[1:12] - 8.0 * np.arange(1, 12)
    assert np.median(lat) < 20.0, lat


def test_failed_launch_fails_only_its_batch(fake):
    """Launches 1 and 4 fail: exactly their requests report MIRNG_E_LAUNCH,
    the others complete normally, and the server keeps serving."""
    d = fake(slots=2, capacity=10**6, max_batch=16, count=200, seed=17, fail_at=(1, 4))
    assert d["failed_launches"] == [1, 4]
    _common(d, 2, 10**6, 16, failed_batches=(1, 4))
    st = np.array(d["status"])
    failed = {t for b in (1, 4) for t in d["batches"][b]}
    assert len(failed) > 0 and int((st == 4).sum()) == len(failed)


def test_resident_engine_positions_in_arrival_order(fake):
    """Requests on 8 resident engines, batched in any grouping: each request
    starts at the sum of the consumption of the requests admitted before it
    on the same engine (plus a 2^100 + 5 skip of engine 3 half-way), and
    the engine counts equal the totals."""
    d = fake(mode="engines", slots=3, capacity=10**8, max_batch=7, count=300, seed=19,
             max_n=10**5)
    _common(d, 3, 10**8, 7)
    n = np.array(d["n"], dtype=object)
    eng = d["engine"]
    consumed = [0] * 8
    for i in range(len(n)):
        e = eng[i]
        want = consumed[e]
        got = d["skip_lo"][i] + (d["skip_mid"][i] << 64)
        assert d["ref_slot"][i] == e
        assert got == want, (i, e, got, want)
        consumed[e] += int(n[i])
        if i == d["skip_after"]:
            consumed[3] += 2**100 + 5
    for e in range(8):
        assert d["consumed_lo"][e] + (d["consumed_mid"][e] << 64) == consumed[e]
    assert len(d["batches"]) > 20          # the requests were spread over many batches
