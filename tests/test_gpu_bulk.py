"""GPU parity at the bulk size n = 2^28 for every engine x output cell, with
the seeds and offsets of the bulk workload (three draws per cell, plus the
draw the benchmark times), in the launch configuration the benchmark uses:
the whole 2^28-element array of every cell is compared with the oracle,
which runs in threads over consecutive slices (each slice starts from the
engine position of its first output)."""
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
CHUNK = 1 << 24          # outputs compared per round (host memory stays small)
THREADS = min(16, os.cpu_count() or 4)


def _expect_window(engine, kind, seed, offset, start, m):
    """Oracle outputs start .. start + m - 1 of the engine (seed, offset);
    start is even, so Gaussian pairs stay whole."""
    if engine == mr.PHILOX4X32_10:
        return gh.oracle_philox(seed, offset + oracle.words_consumed(kind, engine, start), kind, m)
    st = oracle.mrg_skip(oracle.mrg_seed(seed),
                         offset + oracle.words_consumed(kind, engine, start))
    return gh.oracle_mrg(st, kind, m)


def _expect_parallel(engine, kind, seed, offset, start, m, ex):
    step = ((m + THREADS - 1) // THREADS + 1) & ~1
    parts = list(range(0, m, step))
    res = ex.map(lambda s: _expect_window(engine, kind, seed, offset, start + s,
                                          min(step, m - s)), parts)
    return np.concatenate(list(res))


def _cells():
    seen, cells = set(), []
    for c in synth.bulk_draws(count=3) + synth.bulk_draws(count=1):
        if c not in seen:
            seen.add(c)
            cells.append(c)
    return [pytest.param(*c, id=f"{synth.ENGINE_NAME[c[0]]}-{synth.KIND_NAME[c[1]]}-"
                                f"{c[2]:016x}") for c in cells]


@pytest.mark.parametrize("engine,kind,seed,offset", _cells())
def test_bulk_cell(engine, kind, seed, offset):
    import torch
    dt = {mr.BITS_U32: torch.int32, mr.UNIFORM_F32: torch.float32,
          mr.UNIFORM_F64: torch.float64, mr.GAUSSIAN_F32: torch.float32}[kind]
    out = torch.empty(N, dtype=dt, device="cuda")
    e = mr.Engine(engine, seed, offset)
    print(f"bulk cell {synth.ENGINE_NAME[engine]}/{synth.KIND_NAME[kind]} seed {seed:#x} "
          f"offset {offset:#x}", flush=True)
    e.generate(kind, N, out)
    torch.cuda.synchronize()
    assert e.position == offset + mr.words_consumed(engine, kind, N)
    npdt = gh.NP_DTYPE[kind]
    worst = 0.0
    with concurrent.futures.ThreadPoolExecutor(max_workers=THREADS) as ex:
        for start in range(0, N, CHUNK):
            got = out[start:start + CHUNK].cpu().numpy().view(npdt)
            want = _expect_parallel(engine, kind, seed, offset, start, CHUNK, ex)
            worst = max(worst, gh.assert_match(kind, got, want))
    if kind == mr.GAUSSIAN_F32:
        print(f"  worst Gaussian error over 2^28 outputs: {2 * worst:.4f} ulp", flush=True)
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
