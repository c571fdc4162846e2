"""Host-only tests of the serving loop's scheduling policy (admission by
in-flight bytes, arrival-order continuous batching onto free streams, one
batch per stream, completion statuses and latency statistics), driven by a
simulated executor: the scheduler source is compiled with g++ together with
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
            gap_us=0.0, seed=1, max_n=10**4):
        out = subprocess.run([exe, str(slots), str(capacity), str(max_batch), str(ns_per_byte),
                              str(base_us), str(count), str(gap_us), str(seed), str(max_n)],
                             check=True, capture_output=True, text=True, timeout=120)
        return json.loads(out.stdout)
    return run


ELEM = {1: 4, 2: 4, 3: 8, 4: 4, 5: 8, 6: 4, 7: 4, 8: 8}


def _common(d, slots, capacity, max_batch):
    ret = np.array(d["ret"])
    bytes_ = np.array(d["bytes"])
    # admission counts n x element size, 0 for requests the kernel refuses
    for k, n, b in zip(d["kind"], d["n"], d["bytes"]):
        assert b == (n * ELEM[k] if k in ELEM and n < 2**32 else 0), (k, n, b)
    acc = np.nonzero(ret == 0)[0]
    # refused exactly when the request alone exceeds the capacity
    assert np.array_equal(ret != 0, bytes_ > capacity)
    assert np.all(ret[ret != 0] == 6)
    # every accepted request completed with the status the kernel gives
    assert np.array_equal(np.array(d["status"])[acc], np.array(d["expect"])[acc])
    # batches in arrival order, each request exactly once
    order = [t for b in d["batches"] for t in b]
    assert order == sorted(order) == list(range(len(acc)))
    assert all(1 <= len(b) <= max_batch for b in d["batches"])
    assert not d["double_launch"] and d["max_concurrent"] <= slots
    s = d["stats"]
    assert s["submitted"] == len(acc) and s["completed"] == len(acc)
    assert s["refused"] == int((ret != 0).sum())
    assert s["max_inflight_bytes"] <= capacity
    assert s["failed"] == int((np.array(d["expect"])[acc] != 0).sum())
    ok = acc[np.array(d["expect"])[acc] == 0]
    assert s["bytes"] == int(bytes_[ok].sum())
    assert 0.0 <= s["p50"] <= s["p99"] <= s["max"]
    assert d["binds"] == 2      # dispatcher and completion threads


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
