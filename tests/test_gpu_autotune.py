"""The autotuner picks a launch shape by timing candidates on the caller's
workload; the chosen shape is installed and outputs generated with it still
equal the oracle (a launch shape changes speed only)."""
import numpy as np
import pytest

import paper_2109_01329_amd as mr
from tests import gpu_helpers as gh
from tests.test_gpu_batch import _mix, _run, _check_outputs

pytestmark = pytest.mark.gpu


def test_autotune_philox_installs_a_valid_shape():
    import torch
    n = (1 << 20) + 37
    prev = mr.philox_config()
    try:
        buf = torch.empty(n, dtype=torch.float32, device="cuda")
        cfg, ms = mr.autotune_philox(mr.UNIFORM_F32, n, buf, prewarm_ms=50, rounds=2, reps=3,
                                     offset=12345)
        torch.cuda.synchronize()
        assert ms > 0.0
        # installed for the tuned kind at the tuned phase only (12345 mod 4)
        assert mr.philox_config(mr.UNIFORM_F32, 1).as_dict() == cfg.as_dict()
        assert mr.philox_config().as_dict() == prev.as_dict()
        assert mr.philox_config(mr.BITS_U32, 1).as_dict() == prev.as_dict()
        for ph in (0, 2, 3):
            assert mr.philox_config(mr.UNIFORM_F32, ph).as_dict() == prev.as_dict()
        e = mr.Engine(mr.PHILOX4X32_10, 0xFEEDFACE12345678, 12345)
        got, out = gh.generate(e, mr.UNIFORM_F32, n, 0)
        assert gh.guards_intact(out, 0, n * 4)
        gh.assert_match(mr.UNIFORM_F32, got, gh.oracle_philox(0xFEEDFACE12345678, 12345,
                                                               mr.UNIFORM_F32, n))
    finally:
        mr.set_philox_config(prev)


def test_phase_keyed_shapes_differ_and_match_the_oracle():
    """Shapes installed for phase 0 and phase 1 of a kind differ (one each
    by the autotuner's phase keying, set here explicitly so that they surely
    differ), each launch uses its phase's shape, and both give the
    oracle's values; the autotuner run at a phase-0 and at a phase-1
    position installs its results at those phases only."""
    import torch
    prev = mr.philox_config()
    n = (1 << 20) + 9
    try:
        mr.set_philox_config(kind=mr.UNIFORM_F32, phase=0, walk=2, block=256,
                             blocks_per_lane=1, nontemporal=0)
        mr.set_philox_config(kind=mr.UNIFORM_F32, phase=1, walk=0, block=1024,
                             waves_per_cu=256, nontemporal=1)
        assert mr.philox_config(mr.UNIFORM_F32, 0).walk == 2
        assert mr.philox_config(mr.UNIFORM_F32, 1).walk == 0
        for pos in (2**40, 2**40 + 1, 2**40 + 2):
            e = mr.Engine(mr.PHILOX4X32_10, 31337, pos)
            got, buf = gh.generate(e, mr.UNIFORM_F32, n, 0)
            gh.assert_match(mr.UNIFORM_F32, got,
                            gh.oracle_philox(31337, pos, mr.UNIFORM_F32, n))
            assert gh.guards_intact(buf, 0, n * 4)
        buf = torch.empty(n, dtype=torch.float32, device="cuda")
        c0, _ = mr.autotune_philox(mr.BITS_U32, n, buf, prewarm_ms=20, rounds=1, reps=2,
                                   offset=8)
        c1, _ = mr.autotune_philox(mr.BITS_U32, n, buf, prewarm_ms=20, rounds=1, reps=2,
                                   offset=9)
        assert mr.philox_config(mr.BITS_U32, 0).as_dict() == c0.as_dict()
        assert mr.philox_config(mr.BITS_U32, 1).as_dict() == c1.as_dict()
        for pos in (8, 9):
            e = mr.Engine(mr.PHILOX4X32_10, 5, pos)
            got, _ = gh.generate(e, mr.BITS_U32, n, 0)
            gh.assert_match(mr.BITS_U32, got, gh.oracle_philox(5, pos, mr.BITS_U32, n))
    finally:
        mr.set_philox_config(prev)


def test_autotune_batch_keeps_outputs():
    rng = np.random.default_rng(81)
    reqs, layout, nbytes = _mix(rng, 200, max_log10=3.5)
    b = mr.Batcher()
    import torch
    buf = gh.device_buffer(nbytes)
    r = reqs.copy()
    r["out"] = [int(buf.data_ptr()) + lay[0] for lay in layout]
    cfg, ms = b.autotune(r, prewarm_ms=50, rounds=2, reps=3)
    torch.cuda.synchronize()
    assert ms > 0.0
    assert b.config.as_dict() == cfg.as_dict()
    host, st = _run(reqs, layout, nbytes, batcher=b)
    assert np.all(st == 0)
    _check_outputs(host, layout, st)


def test_autotune_cache_hit_installs_stored_shape(tmp_path):
    import time
    import torch
    n = 1 << 20
    prev = mr.philox_config()
    try:
        cache = mr.TuningCache(str(tmp_path / "tune.json"))
        buf = torch.empty(n, dtype=torch.float32, device="cuda")
        cfg, ms = mr.autotune_philox(mr.UNIFORM_F32, n, buf, prewarm_ms=20, rounds=1, reps=2,
                                     cache=cache)
        mr.set_philox_config(walk=1, block=256, waves_per_cu=8, blocks_per_lane=1,
                             nontemporal=0)
        t0 = time.perf_counter()
        cfg2, ms2 = mr.autotune_philox(mr.UNIFORM_F32, n, buf, cache=mr.TuningCache(cache.path))
        assert time.perf_counter() - t0 < 0.2          # no timing loop ran
        assert cfg2.as_dict() == cfg.as_dict() == mr.philox_config(mr.UNIFORM_F32, 1).as_dict()
        assert ms2 == ms
    finally:
        mr.set_philox_config(prev)


def test_per_kind_shapes_apply_to_their_kind_only():
    """A kind's own shape serves that kind; the others follow the
    process-wide shape; both give the oracle's values; the process-wide set
    drops every kind's own shape."""
    prev = mr.philox_config()
    try:
        mr.set_philox_config(walk=3, block=256, waves_per_cu=1, blocks_per_lane=2, nontemporal=0)
        mr.set_philox_config(kind=mr.UNIFORM_F32, walk=0, block=1024, waves_per_cu=256,
                             blocks_per_lane=1, nontemporal=1)
        assert mr.philox_config(mr.UNIFORM_F32).walk == 0
        assert mr.philox_config(mr.GAUSSIAN_F32).walk == 3
        n = 300007
        for kind in (mr.UNIFORM_F32, mr.GAUSSIAN_F32, mr.UNIFORM_I32):
            e = mr.Engine(mr.PHILOX4X32_10, 12, 0)
            e.skip_ahead(2**40 + 1)
            got, buf = gh.generate(e, kind, n, 4)
            gh.assert_match(kind, got, gh.oracle_philox(12, 2**40 + 1, kind, n))
            assert gh.guards_intact(buf, 4, n * 4)
        mr.clear_philox_config(mr.UNIFORM_F32)
        assert mr.philox_config(mr.UNIFORM_F32).walk == 3
        mr.set_philox_config(kind=mr.BITS_U32, walk=2)
        mr.set_philox_config(walk=3)
        assert mr.philox_config(mr.BITS_U32).walk == 3
    finally:
        mr.set_philox_config(prev)
