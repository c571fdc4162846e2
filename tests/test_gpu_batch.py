"""GPU parity of batched generation (Philox4x32-10 and MRG32k3a requests
mixed): every request of a batch equals the oracle (and the plain
single-request path, byte for byte), invalid requests write nothing and
report their status, and outputs do not depend on the request order, the
launch shape or the ring slot and stream used."""
import numpy as np
import pytest

import oracle
import paper_2109_01329_amd as mr
import synth
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

KINDS = [mr.BITS_U32, mr.UNIFORM_F32, mr.UNIFORM_F64, mr.GAUSSIAN_F32, mr.GAUSSIAN_F64,
         mr.UNIFORM_I32, mr.GAUSSIAN_ICDF_F32, mr.GAUSSIAN_ICDF_F64]
GAUSSIANS = (mr.GAUSSIAN_F32, mr.GAUSSIAN_F64, mr.GAUSSIAN_ICDF_F32, mr.GAUSSIAN_ICDF_F64)
FILL = 0xA5


def _mix(rng, count, max_log10=4.3, mrg_frac=0.3):
    """Random requests laid out in one buffer with 64-byte guard gaps and
    every output alignment the element size allows; a fraction `mrg_frac`
    of them on MRG32k3a."""
    reqs = mr.make_requests(count)
    layout = []
    pos = 64
    for i in range(count):
        kind = int(rng.choice(KINDS))
        esz = mr.ELEM_BYTES[kind]
        n = int(rng.choice([0, 1, 2, 3, 5])) if rng.random() < 0.15 else \
            int(10 ** rng.uniform(0, max_log10))
        mis = int(rng.integers(0, 16 // esz)) * esz
        pos = ((pos + 15) // 16) * 16 + mis
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        offset = int(rng.integers(0, 2**64, dtype=np.uint64)) if rng.random() < 0.3 else \
            int(rng.integers(0, 2**40, dtype=np.uint64))
        if kind in (mr.UNIFORM_F32, mr.UNIFORM_F64) and rng.random() < 0.3:
            p0, p1 = -2.0, 3.5
        elif kind in GAUSSIANS and rng.random() < 0.3:
            p0, p1 = 1.5, 0.25
        elif kind == mr.UNIFORM_I32:
            lo = int(rng.integers(-2**31, 2**31 - 1))
            p0, p1 = float(lo), float(rng.integers(lo + 1, 2**31 + 1))
        else:
            p0, p1 = 0.0, 1.0
        engine = mr.MRG32K3A if rng.random() < mrg_frac else mr.PHILOX4X32_10
        reqs[i] = (engine, 0, kind, 0, p0, p1, seed, offset, n, 0)
        layout.append((pos, kind, n, seed, offset, p0, p1, engine))
        pos += n * esz + 64
    return reqs, layout, pos + 64


def _run(reqs, layout, nbytes, batcher=None, stream=None):
    import torch
    buf = gh.device_buffer(nbytes)
    buf.fill_(FILL)
    base = int(buf.data_ptr())
    r = reqs.copy()
    r["out"] = [base + lay[0] for lay in layout]
    b = batcher or mr.Batcher()
    b.generate(r, stream=stream)
    torch.cuda.synchronize()
    return buf.cpu().numpy(), b.statuses(len(r))


def _check_outputs(host, layout, statuses):
    covered = np.zeros(host.size, dtype=bool)
    for (pos, kind, n, seed, offset, p0, p1, engine), st in zip(layout, statuses):
        esz = mr.ELEM_BYTES[kind]
        if st != 0:
            continue
        got = host[pos: pos + n * esz].view(gh.NP_DTYPE[kind])
        want = gh.oracle_request(engine, seed, offset, kind, n, p0, p1)
        gh.assert_match(kind, got, want, p0, p1)
        covered[pos: pos + n * esz] = True
    assert np.all(host[~covered] == FILL), "bytes outside the requests were written"


def test_batch_mixed_requests_vs_oracle():
    rng = np.random.default_rng(71)
    reqs, layout, nbytes = _mix(rng, 400)
    host, st = _run(reqs, layout, nbytes)
    assert np.all(st == 0)
    _check_outputs(host, layout, st)


@pytest.mark.parametrize("count", [65536, 70001])
def test_batch_many_small_requests(count):
    """Batches of exactly 64 chunks of 1024 requests (every wave keeps the
    chunk prefix in registers) and of more (the scan kernel's prefixes)."""
    rng = np.random.default_rng(count)
    reqs, layout, nbytes = _mix(rng, count, max_log10=1.6)
    host, st = _run(reqs, layout, nbytes)
    assert np.all(st == 0)
    _check_outputs(host, layout, st)


def test_batch_counter_carries():
    """Philox requests whose blocks cross a carry out of the counter's low
    word part-way through (a request's 64-bit offset reaches no higher
    carry), and requests at the top of the offset range."""
    positions = [((1 << 32) - 3000) * 4 + 1, ((1 << 32) - 2) * 4, 5 * (1 << 34) - 4 * 2000 + 3,
                 (1 << 64) - 4 * 3000 + 2]
    reqs = mr.make_requests(len(positions) * len(KINDS))
    layout = []
    pos = 64
    i = 0
    for kind in KINDS:
        esz = mr.ELEM_BYTES[kind]
        for j, off in enumerate(positions):
            n = 20001 + 7 * j
            pos = ((pos + 15) // 16) * 16 + (j % (16 // esz)) * esz
            reqs[i] = (mr.PHILOX4X32_10, 0, kind, 0, 0.0, 1.0, 1234 + i, off, n, 0)
            layout.append((pos, kind, n, 1234 + i, off, 0.0, 1.0, mr.PHILOX4X32_10))
            pos += n * esz + 64
            i += 1
    host, st = _run(reqs, layout, pos + 64)
    assert np.all(st == 0)
    _check_outputs(host, layout, st)


def test_batch_follows_earlier_work_on_its_stream():
    """A mixed batch (its MRG kernel runs beside the Philox kernel on an
    internal stream) starts after the work enqueued before it on the
    caller's stream: a long fill of the same buffers enqueued first never
    overwrites the batch's outputs."""
    import torch
    stream = torch.cuda.Stream()
    big = torch.empty(1 << 29, dtype=torch.float32, device="cuda")   # 2 GiB
    n = 50000
    reqs = mr.make_requests(2)
    reqs[0] = (mr.PHILOX4X32_10, 0, mr.UNIFORM_F32, 0, 0.0, 1.0, 11, 0, n, 0)
    reqs[1] = (mr.MRG32K3A, 0, mr.UNIFORM_F32, 0, 0.0, 1.0, 12, 0, n, 0)
    reqs["out"] = [int(big.data_ptr()), int(big.data_ptr()) + 4 * n + 256]
    b = mr.Batcher()
    for _ in range(3):
        with torch.cuda.stream(stream):
            big.fill_(-1.0)
        b.generate(reqs, stream=stream)
        stream.synchronize()
        host = big[: 2 * n + 64].cpu().numpy()
        gh.assert_match(mr.UNIFORM_F32, host[:n], gh.oracle_request(mr.PHILOX4X32_10, 11, 0,
                                                                      mr.UNIFORM_F32, n))
        gh.assert_match(mr.UNIFORM_F32, host[n + 64: 2 * n + 64],
                        gh.oracle_request(mr.MRG32K3A, 12, 0, mr.UNIFORM_F32, n))


def test_batch_equals_plain_path_bytes():
    import torch
    rng = np.random.default_rng(72)
    reqs, layout, nbytes = _mix(rng, 120)
    host, st = _run(reqs, layout, nbytes)
    for pos, kind, n, seed, offset, p0, p1, engine in layout:
        if n == 0:
            continue
        e = mr.Engine(engine, seed, offset)
        got, _ = gh.generate(e, kind, n, pos % 16, p0, p1)
        esz = mr.ELEM_BYTES[kind]
        assert np.array_equal(got.view(np.uint8), host[pos: pos + n * esz])


def test_batch_invariant_to_order_and_launch_shape():
    rng = np.random.default_rng(73)
    reqs, layout, nbytes = _mix(rng, 300)
    ref, _ = _run(reqs, layout, nbytes)
    perm = rng.permutation(len(reqs))
    b = mr.Batcher()
    for cfg in (dict(block=64, waves_per_cu=1, nontemporal=0),
                dict(block=256, waves_per_cu=7, nontemporal=1),
                dict(block=1024, waves_per_cu=4096, nontemporal=0)):
        b.set_config(**cfg)
        host, st = _run(reqs[perm], [layout[i] for i in perm], nbytes, batcher=b)
        assert np.array_equal(host, ref), cfg


def test_batch_invalid_requests_report_and_write_nothing():
    rng = np.random.default_rng(74)
    reqs, layout, nbytes = _mix(rng, 60, max_log10=3)
    bad = {}
    def setbad(i, field, value, code):
        reqs[i][field] = value
        bad[i] = code
    # pick requests with n > 0 to corrupt
    idx = [i for i, lay in enumerate(layout) if lay[2] > 4]
    setbad(idx[0], "kind", 9, 2)                       # unknown distribution
    setbad(idx[1], "engine_type", 7, 2)                # unknown engine
    setbad(idx[2], "engine_type", 0, 2)                # no engine
    setbad(idx[3], "reserved", 1, 1)
    setbad(idx[4], "dist_reserved", 3, 1)
    if layout[idx[5]][1] in (mr.UNIFORM_F32, mr.UNIFORM_F64):
        reqs[idx[5]]["p0"], reqs[idx[5]]["p1"] = 1.0, 1.0
    else:
        reqs[idx[5]]["kind"] = mr.GAUSSIAN_F32
        reqs[idx[5]]["p1"] = -1.0
    bad[idx[5]] = 1
    reqs[idx[6]]["p0"] = float("nan")
    reqs[idx[6]]["kind"] = mr.UNIFORM_F32
    bad[idx[6]] = 1
    reqs[idx[7]]["n"] = 1 << 32
    bad[idx[7]] = 6
    host, st = _run(reqs, layout, nbytes)
    for i, code in bad.items():
        assert st[i] == code, (i, st[i], code)
    good = [i for i in range(len(layout)) if i not in bad]
    assert np.all(st[good] == 0)
    lay2 = list(layout)
    _check_outputs(host, lay2, [st[i] for i in range(len(layout))])


def test_batch_mrg_chunk_edges():
    """MRG requests whose sizes straddle chunk and pass boundaries (16384
    outputs per chunk for 4-byte kinds, 8192 for FP64), at every alignment
    and with offsets across the 64-bit range."""
    rng = np.random.default_rng(77)
    reqs = mr.make_requests(0)
    sizes = [1, 31, 32, 33, 63, 64, 65, 8191, 8192, 8193, 16383, 16384, 16385, 40000]
    recs, layout, pos = [], [], 64
    for n in sizes:
        for kind in KINDS:
            esz = mr.ELEM_BYTES[kind]
            mis = int(rng.integers(0, 16 // esz)) * esz
            pos = ((pos + 15) // 16) * 16 + mis
            seed = int(rng.integers(0, 2**64, dtype=np.uint64))
            offset = int(rng.integers(0, 2**64, dtype=np.uint64))
            recs.append((mr.MRG32K3A, 0, kind, 0, 0.0, 1.0, seed, offset, n, 0))
            layout.append((pos, kind, n, seed, offset, 0.0, 1.0, mr.MRG32K3A))
            pos += n * esz + 64
    reqs = np.array(recs, dtype=mr.request_dtype())
    host, st = _run(reqs, layout, pos + 64)
    assert np.all(st == 0)
    _check_outputs(host, layout, st)


def test_batch_calorimeter_shape():
    """Event-shaped batch: per event a uniform FP32 request of 3h outputs at
    position 0 and a Gaussian request of h outputs at position 3h on key
    (seed32, event id); outputs contiguous per event."""
    import torch
    ev = synth.calo_events(n_events=2000)
    h = ev.hits
    reqs = mr.make_requests(2 * ev.n_events)
    sizes = np.stack([3 * h, h], axis=1).reshape(-1)
    offs = np.concatenate([[0], np.cumsum(sizes * 4)])[:-1]
    out = torch.empty(int(sizes.sum()), dtype=torch.float32, device="cuda")
    base = int(out.data_ptr())
    seeds = (np.arange(ev.n_events, dtype=np.uint64) << np.uint64(32)) | np.uint64(ev.seed32)
    reqs["engine_type"] = 1
    reqs["kind"] = np.tile([mr.UNIFORM_F32, mr.GAUSSIAN_F32], ev.n_events)
    reqs["p0"] = 0.0
    reqs["p1"] = 1.0
    reqs["seed"] = np.repeat(seeds, 2)
    reqs["offset"] = np.stack([np.zeros_like(h), 3 * h], axis=1).reshape(-1)
    reqs["n"] = sizes
    reqs["out"] = base + offs
    b = mr.Batcher()
    b.generate(reqs)
    torch.cuda.synchronize()
    assert np.all(b.statuses(len(reqs)) == 0)
    host = out.cpu().numpy()
    rng = np.random.default_rng(75)
    for e in rng.choice(ev.n_events, 150, replace=False):
        seed = int(seeds[e])
        o = int(offs[2 * e]) // 4
        gh.assert_match(mr.UNIFORM_F32, host[o: o + 3 * h[e]],
                        gh.oracle_philox(seed, 0, mr.UNIFORM_F32, int(3 * h[e])))
        g = host[o + 3 * h[e]: o + 4 * h[e]]
        gh.assert_match(mr.GAUSSIAN_F32, g,
                        gh.oracle_philox(seed, int(3 * h[e]), mr.GAUSSIAN_F32, int(h[e])))


def test_batch_staged_ring_two_streams():
    import torch
    rng = np.random.default_rng(76)
    b = mr.Batcher()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    jobs = []
    for k in range(7):                 # more batches than ring slots
        reqs, layout, nbytes = _mix(rng, 50 + 13 * k, max_log10=3.5)
        buf = gh.device_buffer(nbytes)
        buf.fill_(FILL)
        torch.cuda.synchronize()
        staged = b.stage(len(reqs))
        staged[:] = reqs
        staged["out"] = [int(buf.data_ptr()) + lay[0] for lay in layout]
        b.generate(staged, stream=streams[k % 2])
        jobs.append((buf, layout))
    torch.cuda.synchronize()
    for buf, layout in jobs:
        host = buf.cpu().numpy()
        _check_outputs(host, layout, [0] * len(layout))


def test_batch_large_requests_among_small():
    """Two large requests (one per engine, misaligned, odd phase) among many
    small ones: the generation waves and groups whose ranges start inside a
    large request find it by search."""
    rng = np.random.default_rng(78)
    reqs, layout, nbytes = _mix(rng, 300, max_log10=3.0)
    big = [(mr.PHILOX4X32_10, mr.UNIFORM_F32, (1 << 22) + 13, 4, 2**40 + 3),
           (mr.MRG32K3A, mr.UNIFORM_F64, (1 << 21) + 5, 8, 2**50 + 7),
           (mr.PHILOX4X32_10, mr.GAUSSIAN_F32, (1 << 20) + 1, 12, 2**33 + 1)]
    recs = list(reqs)
    lay = list(layout)
    pos = nbytes
    for engine, kind, n, mis, offset in big:
        pos = ((pos + 15) // 16) * 16 + mis
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        at = int(rng.integers(0, len(recs) + 1))
        recs.insert(at, (engine, 0, kind, 0, 0.0, 1.0, seed, offset, n, 0))
        lay.insert(at, (pos, kind, n, seed, offset, 0.0, 1.0, engine))
        pos += n * mr.ELEM_BYTES[kind] + 64
    r = np.array(recs, dtype=mr.request_dtype())
    host, st = _run(r, lay, pos + 64)
    assert np.all(st == 0)
    _check_outputs(host, lay, st)


@pytest.mark.parametrize("name,events", [("single_electron", 400), ("ttbar", 3),
                                         ("single_electron_min200k", 40),
                                         ("single_electron_soa", 300)])
def test_batch_fastcalosim_scenarios(name, events):
    """The paper's FastCaloSim scenarios as one batch each: three uniform
    FP32 per hit on key (42, event id); the variants draw at least 200,000
    per event, or one request per quantity into three arrays.  Requests of
    up to 200,000 outputs are checked whole; ttbar events (tens of millions
    of samples each) at their head, middle and tail."""
    import torch
    sc = synth.calo_scenario(name, n_events=events)
    seeds, offsets, sizes, first = sc.requests()
    total = int(sizes.sum())
    out = torch.empty(total, dtype=torch.float32, device="cuda")
    reqs = mr.make_requests(sizes.size)
    reqs["engine_type"] = mr.PHILOX4X32_10
    reqs["kind"] = mr.UNIFORM_F32
    reqs["p1"] = 1.0
    reqs["seed"] = seeds
    reqs["offset"] = offsets
    reqs["n"] = sizes
    reqs["out"] = np.uint64(out.data_ptr()) + first * np.uint64(4)
    b = mr.Batcher()
    b.generate(reqs)
    torch.cuda.synchronize()
    assert np.all(b.statuses(sizes.size) == 0)
    host = out.cpu().numpy()
    covered = 0
    for r in range(sizes.size):
        n, o, f = int(sizes[r]), int(offsets[r]), int(first[r])
        wins = [(0, n)] if n <= 200000 else [(0, 4096), (n // 2 - 2048, 4096), (n - 4096, 4096)]
        for s, m in wins:
            gh.assert_match(mr.UNIFORM_F32, host[f + s: f + s + m],
                            gh.oracle_philox(int(seeds[r]), o + s, mr.UNIFORM_F32, m))
        covered += n
    assert covered == total
    if sc.layout == "soa":
        # quantity q of event e is the event's stream from word q h_e on
        e, h = 1, int(sc.hits[1])
        place = int(sc.hits[:1].sum())
        allw = gh.oracle_philox(int(seeds[3]), 0, mr.UNIFORM_F32, 3 * h)
        for q in range(3):
            start = q * int(sc.hits.sum()) + place
            gh.assert_match(mr.UNIFORM_F32, host[start: start + h], allw[q * h:(q + 1) * h])
