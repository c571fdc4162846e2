"""GPU parity at the bulk size n = 2^28 for every engine x output cell, with
the seeds and offsets of the bulk workload, in the launch configuration the
benchmark times.  Philox uniform FP32 (the headline cell) is compared in
full; the other cells over three 2^20 windows (head, a random middle, tail)
and 4096 random single elements that the oracle computes one by one."""
import concurrent.futures
import os

import numpy as np
import pytest

import oracle
import paper_2109_01329_amd as mr
import synth
from tests import gpu_helpers as gh

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = synth.BULK_N
WIN = 1 << 20


def _philox_parallel(seed, pos, kind, n, parts=16):
    """The oracle on `parts` consecutive slices, in threads (ctypes releases
    the GIL); slices start at even outputs so Gaussian pairs stay whole."""
    step = ((n + parts - 1) // parts + 1) & ~1
    starts = list(range(0, n, step))

    def one(s):
        m = min(step, n - s)
        return gh.oracle_philox(seed, pos + mr.words_consumed(1, kind, s), kind, m)

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        return np.concatenate(list(ex.map(one, starts)))


def _cells():
    cells = synth.bulk_draws(count=1)
    return [pytest.param(*c, id=f"{synth.ENGINE_NAME[c[0]]}-{synth.KIND_NAME[c[1]]}")
            for c in cells]


def _expect_window(engine, kind, seed, offset, start, m):
    if engine == mr.PHILOX4X32_10:
        return gh.oracle_philox(seed, offset + mr.words_consumed(1, kind, start), kind, m)
    st = oracle.mrg_skip(oracle.mrg_seed(seed), offset + start)
    return gh.oracle_mrg(st, kind, m)


@pytest.mark.parametrize("engine,kind,seed,offset", _cells())
def test_bulk_cell(engine, kind, seed, offset):
    import torch
    dt = {mr.BITS_U32: torch.int32, mr.UNIFORM_F32: torch.float32,
          mr.UNIFORM_F64: torch.float64, mr.GAUSSIAN_F32: torch.float32}[kind]
    out = torch.empty(N, dtype=dt, device="cuda")
    e = mr.Engine(engine, seed, offset)
    e.generate(kind, N, out)
    torch.cuda.synchronize()
    npdt = gh.NP_DTYPE[kind]
    if engine == mr.PHILOX4X32_10 and kind == mr.UNIFORM_F32:
        got = out.cpu().numpy().view(npdt)
        gh.assert_match(kind, got, _philox_parallel(seed, offset, kind, N))
        return
    g = np.random.default_rng(seed & 0xFFFF)
    mid = int(g.integers(WIN, N - 2 * WIN)) & ~1
    for start in (0, mid, N - WIN):
        got = out[start:start + WIN].cpu().numpy().view(npdt)
        gh.assert_match(kind, got, _expect_window(engine, kind, seed, offset, start, WIN))
    idx = np.unique(g.integers(0, N, 4096))
    got = out[torch.from_numpy(idx).cuda()].cpu().numpy().view(npdt)
    want = []
    for i in idx:
        i = int(i)
        if kind == mr.GAUSSIAN_F32:
            pair = _expect_window(engine, kind, seed, offset, i & ~1, 2)
            want.append(pair[i & 1])
        else:
            want.append(_expect_window(engine, kind, seed, offset, i, 1)[0])
    gh.assert_match(kind, got, np.array(want, dtype=gh.oracle.OUT_DTYPE[kind]
                                        if kind == mr.GAUSSIAN_F32 else npdt))
    # properties over the whole array, computed on the device
    if kind in (mr.UNIFORM_F32, mr.UNIFORM_F64):
        assert float(out.min()) >= 0.0 and float(out.max()) < 1.0
        assert abs(float(out.double().mean()) - 0.5) < 6 * (1 / (12 * N)) ** 0.5
    if kind == mr.GAUSSIAN_F32:
        assert abs(float(out.double().mean())) < 6 / N**0.5
        assert abs(float(out.double().var()) - 1.0) < 6 * (2 / N) ** 0.5


@pytest.mark.parametrize("engine,kind,seed,offset", [
    (mr.PHILOX4X32_10, mr.UNIFORM_F32, 0x0123456789ABCDEF, 2**40 + 1),
    (mr.PHILOX4X32_10, mr.GAUSSIAN_F32, 77, 3),
    (mr.MRG32K3A, mr.BITS_U32, 0xFEDCBA9876543210, 12345)])
def test_beyond_2p32_outputs(engine, kind, seed, offset):
    """One generate of 2^32 + 2^20 + 7 outputs (beyond a single Philox launch
    of 2^32, and 17 GB): windows at the head, across 2^32 and at the tail
    equal the oracle, and the engine advanced by the words consumed."""
    import torch
    n = (1 << 32) + (1 << 20) + 7
    esz = mr.ELEM_BYTES[kind]
    buf = torch.empty(n * esz // 4 + 64, dtype=torch.int32, device="cuda")
    e = mr.Engine(engine, seed, offset)
    e.generate(kind, n, buf)
    torch.cuda.synchronize()
    raw = buf.view(torch.uint8)
    for start in (0, (1 << 32) - 4098, n - 4096):
        start -= start % 2
        m = min(8192, n - start)
        got = raw[start * esz: (start + m) * esz].cpu().numpy().view(gh.NP_DTYPE[kind])
        gh.assert_match(kind, got, _expect_window(engine, kind, seed, offset, start, m))
    assert e.position == offset + mr.words_consumed(engine, kind, n)
    del buf, raw
    torch.cuda.empty_cache()
