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


# ------------------------------------------------------------ resident engines

SEQ_KINDS = [mr.UNIFORM_F32, mr.BITS_U32, mr.GAUSSIAN_F32, mr.UNIFORM_F64, mr.GAUSSIAN_F64,
             mr.UNIFORM_I32, mr.GAUSSIAN_ICDF_F32, mr.GAUSSIAN_ICDF_F64]


def _sequence(rng, count, max_log10=4.0):
    """(kind, n, byte offset) of a request sequence laid out in one buffer."""
    seq, pos = [], 64
    for _ in range(count):
        kind = int(rng.choice(SEQ_KINDS))
        n = int(10 ** rng.uniform(0, max_log10))
        esz = mr.ELEM_BYTES[kind]
        pos = ((pos + 15) // 16) * 16 + int(rng.integers(0, 16 // esz)) * esz
        seq.append((kind, n, pos))
        pos += n * esz + 64
    return seq, pos + 64


def _plain_sequence(engine_type, seed, offset, seq, nbytes, skip=0):
    import torch
    buf = gh.device_buffer(nbytes)
    buf.fill_(FILL)
    e = mr.Engine(engine_type, seed, offset)
    if skip:
        e.skip_ahead(skip)
    base = int(buf.data_ptr())
    for kind, n, pos in seq:
        e.generate(kind, n, base + pos)
    torch.cuda.synchronize()
    return buf.cpu().numpy(), e


@pytest.mark.parametrize("engine_type", [mr.PHILOX4X32_10, mr.MRG32K3A])
def test_resident_engine_equals_plain_engine_alone_and_in_mix(engine_type):
    """A sequence of requests served on one resident engine writes the same
    bytes as the same sequence of generate calls on one plain engine,
    served alone and amid other traffic (another resident engine and
    requests with their own seed and offset), and the server's view of the
    engine state equals the plain engine's."""
    import torch
    rng = np.random.default_rng(94 + engine_type)
    seed, offset = int(rng.integers(0, 2**64, dtype=np.uint64)), 12345 + engine_type
    seq, nbytes = _sequence(rng, 60)
    want, plain = _plain_sequence(engine_type, seed, offset, seq, nbytes)
    others, olayout, onbytes = _mix(rng, 300, max_log10=3.8, mrg_frac=0.5)
    for mixed in (False, True):
        buf = gh.device_buffer(nbytes)
        buf.fill_(FILL)
        obuf, oreqs = _buffer(olayout, onbytes, others)
        sink = torch.empty(1000, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        srv = mr.Server(streams=3, capacity_bytes=1 << 26, max_batch=96, max_engines=16)
        other = srv.engine_create(3 - engine_type, seed ^ 0x5555, 7)
        e = srv.engine_create(engine_type, seed, offset)
        base = int(buf.data_ptr())
        k = 0
        for kind, n, pos in seq:
            if mixed:
                for _ in range(5):
                    srv.submit(oreqs[k])
                    k += 1
                srv.submit_engine(other, mr.UNIFORM_F32, 1000, sink)
            srv.submit_engine(e, kind, n, base + pos)
        srv.drain()
        st, ps = srv.engine_state(e), plain.get_state()
        assert st.engine_type == ps.engine_type and list(st.words) == list(ps.words)
        assert list(st.pos) == list(ps.pos)
        stats = srv.stats()
        srv.close()
        assert stats["failed"] == 0
        got = buf.cpu().numpy()
        assert np.array_equal(got, want), f"mixed={mixed}: {int((got != want).sum())} bytes differ"
        if mixed:
            _check_outputs_prefix(obuf.cpu().numpy(), olayout, k)


def _check_outputs_prefix(host, layout, count):
    for pos, kind, n, seed, offset, p0, p1, engine in layout[:count]:
        got = host[pos: pos + n * mr.ELEM_BYTES[kind]].view(gh.NP_DTYPE[kind])
        gh.assert_match(kind, got, gh.oracle_request(engine, seed, offset, kind, n, p0, p1),
                        p0, p1)


def test_resident_engine_requests_equal_one_generate_of_the_concatenation():
    """40 uniform FP32 requests on one resident engine, written back to back,
    equal one plain generate of their total from the same engine."""
    import torch
    rng = np.random.default_rng(97)
    sizes = [int(10 ** rng.uniform(0, 5)) for _ in range(40)]
    total = sum(sizes)
    out = torch.empty(total, dtype=torch.float32, device="cuda")
    srv = mr.Server(streams=2, capacity_bytes=1 << 30, max_batch=8, max_engines=4)
    e = srv.engine_create(mr.PHILOX4X32_10, 0xC0FFEE, 3)
    pos = 0
    for n in sizes:
        srv.submit_engine(e, mr.UNIFORM_F32, n, out.data_ptr() + 4 * pos)
        pos += n
    srv.drain()
    srv.close()
    ref = torch.empty(total, dtype=torch.float32, device="cuda")
    mr.Engine(mr.PHILOX4X32_10, 0xC0FFEE, 3).generate(mr.UNIFORM_F32, total, ref)
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))


@pytest.mark.parametrize("engine_type,skip", [
    (mr.MRG32K3A, 3 * 2**127 + 5 * 2**76 + 12345),        # stream 3, substream 5
    (mr.PHILOX4X32_10, 2**100 + 2**64 + 3),                # past 64-bit positions
    (mr.PHILOX4X32_10, 2**130 - 7)])                       # across the 2^130 wrap
def test_resident_engine_positions_beyond_64_bits(engine_type, skip):
    """Served requests after a skip past 2^64 words or steps (MRG32k3a
    streams and substreams, Philox positions up to the 2^130 wrap) equal
    the oracle at that position."""
    import torch
    seed, offset = 0x123456789, 77
    seq = [(mr.UNIFORM_F64, 3000), (mr.BITS_U32, 5001), (mr.GAUSSIAN_F32, 777),
           (mr.UNIFORM_F32, 4096)]
    srv = mr.Server(streams=2, capacity_bytes=1 << 28, max_batch=2, max_engines=2)
    e = srv.engine_create(engine_type, seed, offset)
    srv.engine_skip_ahead(e, skip)
    outs = []
    for kind, n in seq:
        out = torch.empty(n * mr.ELEM_BYTES[kind] // 4, dtype=torch.int32, device="cuda")
        srv.submit_engine(e, kind, n, out)
        outs.append(out)
    srv.drain()
    st = srv.engine_state(e)
    srv.close()
    import oracle
    if engine_type == mr.MRG32K3A:
        state = oracle.mrg_skip(oracle.mrg_seed(seed), offset + skip)
    pos = (offset + skip) % 2**130
    for (kind, n), out in zip(seq, outs):
        got = out.cpu().numpy().view(gh.NP_DTYPE[kind])
        if engine_type == mr.MRG32K3A:
            want, state = oracle.mrg_generate(state, kind, n)
        else:
            want = oracle.philox_generate(seed, pos, kind, n)
            pos = (pos + oracle.words_consumed(kind, oracle.PHILOX, n)) % 2**130
        gh.assert_match(kind, got, want)
    if engine_type == mr.MRG32K3A:
        assert list(st.words) == [int(x) for x in state]
    else:
        assert st.pos[0] | (st.pos[1] << 64) | (st.pos[2] << 128) == pos


def test_resident_engine_checkpoint_and_resume():
    """get_state after part of a sequence, more requests, then set_state back
    to the checkpoint: the same requests write the same bytes again."""
    import torch
    srv = mr.Server(streams=2, capacity_bytes=1 << 28, max_batch=4, max_engines=2)
    e = srv.engine_create(mr.MRG32K3A, 99, 5)
    g = torch.empty(333, dtype=torch.float32, device="cuda")
    a = torch.empty(10000, dtype=torch.float32, device="cuda")
    b = torch.empty(10000, dtype=torch.float32, device="cuda")
    # requests in flight together may run in any order: each gets its own
    # output buffer
    srv.submit_engine(e, mr.GAUSSIAN_F32, 333, g)
    ck = srv.engine_state(e)
    srv.submit_engine(e, mr.UNIFORM_F32, 10000, a)
    srv.drain()
    srv.engine_set_state(e, ck)
    srv.submit_engine(e, mr.UNIFORM_F32, 10000, b)
    srv.drain()
    with pytest.raises(mr.MirngError):
        srv.submit_engine(7, mr.UNIFORM_F32, 10, b)          # no such engine
    with pytest.raises(mr.MirngError):
        srv.submit_engine(e, mr.UNIFORM_F32, 10, b, 1.0, 1.0)   # empty range
    assert list(srv.engine_state(e).pos) == [5 + 334 + 10000, 0, 0]
    srv.close()
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
