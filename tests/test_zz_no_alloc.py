"""GPU parity of the allocation-free batched entry point
(mirng_generate_batch_noalloc): on the same requests it gives the batcher's
outputs byte for byte and the same per-request statuses, over two calls in a
row (the second smaller, so stale tables of the first call would show), and
its outputs match the oracle.  Collected last, so that it also runs after
every other GPU test in one process."""
import ctypes

import numpy as np
import pytest

import paper_2109_01329_amd as mr
from tests import gpu_helpers as gh
from tests.test_gpu_batch import FILL, _check_outputs, _mix

pytestmark = pytest.mark.gpu


def _with_out(reqs, layout, base):
    r = reqs.copy()
    r["out"] = [base + lay[0] for lay in layout]
    return r


def _both(reqs, layout, nbytes, cfg=None):
    """(batcher bytes, batcher statuses, no-alloc bytes, no-alloc statuses)."""
    import torch
    a = gh.device_buffer(nbytes)
    b = gh.device_buffer(nbytes)
    a.fill_(FILL)
    b.fill_(FILL)
    st = torch.full((max(len(reqs), 1),), -1, dtype=torch.int32, device="cuda")
    bt = mr.Batcher()
    if cfg is not None:
        bt.set_config(cfg)
    bt.generate(_with_out(reqs, layout, int(a.data_ptr())))
    mr.generate_batch_noalloc(_with_out(reqs, layout, int(b.data_ptr())), st, config=cfg)
    torch.cuda.synchronize()
    want_st = bt.statuses(len(reqs))
    bt.close()
    return a.cpu().numpy(), want_st, b.cpu().numpy(), st.cpu().numpy()[:len(reqs)]


def _bad_request(reqs, layout):
    """Make request 3 invalid (uniform with a >= b): it must report
    INVALID_ARG on both paths and write nothing."""
    reqs[3]["kind"] = mr.UNIFORM_F32
    reqs[3]["p0"] = 2.0
    reqs[3]["p1"] = 1.0
    pos, _, n, seed, off, _, _, eng = layout[3]
    layout[3] = (pos, mr.UNIFORM_F32, n, seed, off, 2.0, 1.0, eng)


def test_noalloc_matches_batcher_two_calls():
    mr.device_init()
    rng = np.random.default_rng(907)
    # first call: a large mixed batch (several planning chunks, both
    # engines, every kind, wide kinds included)
    print("no-alloc call 1: 5000 requests", flush=True)
    reqs, layout, nbytes = _mix(rng, 5000, max_log10=4.0, mrg_frac=0.35)
    _bad_request(reqs, layout)
    want, want_st, got, got_st = _both(reqs, layout, nbytes)
    assert np.array_equal(got_st, want_st)
    assert got_st[3] == 1 and np.sum(got_st != 0) == 1
    assert np.array_equal(got, want)
    _check_outputs(got, layout, got_st)
    # second call: smaller, through the same scratch array
    print("no-alloc call 2: 300 requests", flush=True)
    reqs, layout, nbytes = _mix(rng, 300, max_log10=3.5, mrg_frac=0.5)
    want, want_st, got, got_st = _both(reqs, layout, nbytes,
                                       cfg=mr.BatchConfig(256, 64, 1, 0))
    assert np.array_equal(got_st, want_st) and np.all(got_st == 0)
    assert np.array_equal(got, want)
    _check_outputs(got, layout, got_st)


def test_noalloc_limits_and_arguments():
    import torch
    mr.device_init()
    L = mr.lib()
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    reqs = mr.make_requests(4)
    ptr = reqs.ctypes.data
    assert L.mirng_generate_batch_noalloc(ptr, 0, None, None, None) == 0
    assert L.mirng_generate_batch_noalloc(None, 4, st.data_ptr(), None, None) == 1
    assert L.mirng_generate_batch_noalloc(ptr, 4, None, None, None) == 1
    assert L.mirng_generate_batch_noalloc(ptr, 4, st.data_ptr() + 2, None, None) == 1
    bad = mr.BatchConfig(100, 64, 0, 0)
    assert L.mirng_generate_batch_noalloc(ptr, 4, st.data_ptr(), ctypes.byref(bad), None) == 1
    big = mr.make_requests(mr.NOALLOC_MAX_REQUESTS + 1)
    big_st = torch.zeros(len(big), dtype=torch.int32, device="cuda")
    assert L.mirng_generate_batch_noalloc(big.ctypes.data, len(big), big_st.data_ptr(),
                                          None, None) == 6
    torch.cuda.synchronize()


def test_noalloc_at_the_request_limit():
    """A batch of exactly MIRNG_NOALLOC_MAX_REQUESTS small requests."""
    rng = np.random.default_rng(5)
    reqs, layout, nbytes = _mix(rng, mr.NOALLOC_MAX_REQUESTS, max_log10=1.5)
    want, want_st, got, got_st = _both(reqs, layout, nbytes)
    assert np.array_equal(got_st, want_st) and np.all(got_st == 0)
    assert np.array_equal(got, want)
