"""GPU parity of the serving loop: requests submitted one at a time (both
engines, every kind, every output alignment) complete with the oracle's
outputs whatever they were batched with; admission keeps the in-flight
output bytes within the capacity; oversized requests are refused; the
native open-loop replay submits on schedule."""
import numpy as np
import pytest

import paper_2109_01329_amd as mr
from tests import gpu_helpers as gh
from tests.test_gpu_batch import FILL, _check_outputs, _mix

pytestmark = pytest.mark.gpu


def _buffer(layout, nbytes, reqs):
    import torch
    buf = gh.device_buffer(nbytes)
    buf.fill_(FILL)
    torch.cuda.synchronize()
    r = reqs.copy()
    r["out"] = [int(buf.data_ptr()) + lay[0] for lay in layout]
    return buf, r


def test_server_mixed_requests_vs_oracle():
    rng = np.random.default_rng(91)
    reqs, layout, nbytes = _mix(rng, 300, max_log10=4.0, mrg_frac=0.5)
    buf, r = _buffer(layout, nbytes, reqs)
    cap = 1 << 18
    srv = mr.Server(streams=3, capacity_bytes=cap, max_batch=64)
    tickets = [srv.submit(x) for x in r]
    res = [srv.wait(t) for t in tickets]
    srv.drain()
    st = srv.stats()
    srv.close()
    statuses = [s for s, _ in res]
    assert all(s == 0 for s in statuses)
    _check_outputs(buf.cpu().numpy(), layout, statuses)
    assert st["completed"] == st["submitted"] == 300 and st["failed"] == 0
    assert 0 < st["max_inflight_bytes"] <= cap
    assert st["batches"] >= 5          # the capacity forces several batches
    assert st["samples"] == int(sum(lay[2] for lay in layout))
    assert all(lat >= 0.0 for _, lat in res)


def test_server_output_independent_of_batching():
    """A request served alone and the same request amid 200 others write the
    same bytes."""
    rng = np.random.default_rng(92)
    reqs, layout, nbytes = _mix(rng, 200, max_log10=3.8, mrg_frac=0.5)
    buf, r = _buffer(layout, nbytes, reqs)
    srv = mr.Server(streams=2, capacity_bytes=1 << 30, max_batch=1 << 16)
    for x in r:
        srv.submit(x)
    srv.drain()
    mixed = buf.cpu().numpy().copy()
    buf.fill_(FILL)
    import torch
    torch.cuda.synchronize()
    chosen = [int(i) for i in rng.choice(len(r), 12, replace=False)]
    for i in chosen:
        s, _ = srv.wait(srv.submit(r[i]))
        assert s == 0
    srv.close()
    alone = buf.cpu().numpy()
    for i in chosen:
        pos, kind, n = layout[i][0], layout[i][1], layout[i][2]
        seg = slice(pos, pos + n * mr.ELEM_BYTES[kind])
        assert np.array_equal(alone[seg], mixed[seg]), i


def test_server_refuses_oversized_and_reports_invalid():
    import torch
    out = torch.empty(4096, dtype=torch.float32, device="cuda")
    srv = mr.Server(streams=1, capacity_bytes=4000, max_batch=16)
    r = mr.make_requests(3)
    r[0] = (1, 0, 2, 0, 0.0, 1.0, 5, 0, 1001, out.data_ptr())     # 4004 bytes > capacity
    r[1] = (2, 0, 9, 0, 0.0, 1.0, 5, 0, 10, out.data_ptr())       # unknown kind
    r[2] = (2, 0, 2, 0, 0.0, 1.0, 5, 0, 1000, out.data_ptr())     # fits exactly
    with pytest.raises(mr.MirngError) as e:
        srv.submit(r[0])
    assert e.value.status == 6
    t1, t2 = srv.submit(r[1]), srv.submit(r[2])
    assert srv.wait(t1)[0] == 2
    assert srv.wait(t2)[0] == 0
    st = srv.stats()
    srv.close()
    assert st["refused"] == 1 and st["failed"] == 1 and st["completed"] == 2
    got = out[:1000].cpu().numpy()
    want = gh.oracle_request(2, 5, 0, mr.UNIFORM_F32, 1000)
    gh.assert_match(mr.UNIFORM_F32, got, want)


def test_server_replay_on_schedule():
    rng = np.random.default_rng(93)
    reqs, layout, nbytes = _mix(rng, 80, max_log10=3.5, mrg_frac=0.5)
    buf, r = _buffer(layout, nbytes, reqs)
    srv = mr.Server(streams=2, capacity_bytes=1 << 30, max_batch=1024)
    arrival = np.cumsum(rng.exponential(200e-6, len(r)))
    import time
    t0 = time.perf_counter()
    tickets, sub = srv.replay(r, arrival)
    dt = time.perf_counter() - t0
    srv.drain()
    st = srv.stats()
    srv.close()
    assert np.all(sub == 0)
    assert dt >= arrival[-1]
    assert st["completed"] == len(r) and st["span_s"] >= arrival[-1] - arrival[0]
    _check_outputs(buf.cpu().numpy(), layout, [0] * len(r))
