"""Host-side tests of libmirng.so that launch nothing: every symbol the
headers declare is exported, engine state and skip-ahead (the library's
matrix-power jumps) agree with the oracle's polynomial jumps, and argument
validation returns the documented status without touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2109_01329_amd as mr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
M1, M2 = 2**32 - 209, 2**32 - 22853


@pytest.fixture(scope="module")
def L():
    return mr.lib()


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(mirng_\w+)\s*\(", src))
    return names


def test_exports_every_declared_symbol(L):
    names = _declared_symbols()
    assert "mirng_generate" in names and "mirng_engine_create" in names
    for n in sorted(names):
        assert hasattr(L, n), n


def test_abi_version_and_status_strings(L):
    assert L.mirng_abi_version() == 2
    for s in range(7):
        assert L.mirng_status_string(s)
    assert L.mirng_status_string(99) == b"unknown status"


def test_philox_state_from_seed_and_offset():
    e = mr.Engine(mr.PHILOX4X32_10, 0x1122334455667788, 12345)
    s = e.get_state()
    assert (s.words[0], s.words[1]) == (0x55667788, 0x11223344)
    assert e.position == 12345
    e.skip_ahead(2**64 + 7)
    assert e.position == 12345 + 2**64 + 7
    e.skip_ahead(2**130 - 1)          # wraps modulo 2^130
    assert e.position == 12345 + 2**64 + 6


def test_mrg_create_matches_oracle_jump(orc):
    g = np.random.default_rng(41)
    for _ in range(20):
        seed = int(g.integers(0, 2**64, dtype=np.uint64))
        off = int(g.integers(0, 2**40, dtype=np.uint64))
        e = mr.Engine(mr.MRG32K3A, seed, off)
        s = e.get_state()
        want = orc.mrg_skip(orc.mrg_seed(seed), off)
        assert [int(x) for x in s.words] == [int(x) for x in want]
        assert e.position == off


@pytest.mark.parametrize("n", [1, 2**63 + 5, 2**76, 3 * 2**76 + 1, 2**127, 2**191 + 99])
def test_mrg_skip_multi_matches_oracle(orc, n):
    e = mr.Engine(mr.MRG32K3A, 7, 0)
    e.skip_ahead(n)
    want = orc.mrg_skip(orc.mrg_seed(7), n)
    assert [int(x) for x in e.get_state().words] == [int(x) for x in want]


def test_state_round_trip_and_validation():
    e = mr.Engine(mr.MRG32K3A, 99, 5)
    s = e.get_state()
    f = mr.Engine(mr.MRG32K3A, 1, 0)
    f.set_state(s)
    assert list(f.get_state().words) == list(s.words)
    bad = mr.State.from_buffer_copy(s)
    bad.words[0] = M1
    with pytest.raises(mr.MirngError):
        f.set_state(bad)
    zero = mr.State.from_buffer_copy(s)
    zero.words[0] = zero.words[1] = zero.words[2] = 0
    with pytest.raises(mr.MirngError):
        f.set_state(zero)
    p = mr.Engine(mr.PHILOX4X32_10, 3, 0)
    with pytest.raises(mr.MirngError):
        p.set_state(s)                    # engine type mismatch
    ps = p.get_state()
    ps.pos[2] = 4
    with pytest.raises(mr.MirngError):
        p.set_state(ps)


def test_words_consumed():
    assert mr.words_consumed(1, mr.UNIFORM_F64, 5) == 10
    assert mr.words_consumed(2, mr.UNIFORM_F64, 5) == 5
    assert mr.words_consumed(1, mr.GAUSSIAN_F32, 5) == 6
    assert mr.words_consumed(2, mr.BITS_U32, 5) == 5
    assert mr.words_consumed(1, mr.GAUSSIAN_F64, 5) == 12
    assert mr.words_consumed(2, mr.GAUSSIAN_F64, 5) == 6
    assert mr.words_consumed(1, mr.UNIFORM_I32, 5) == 5
    assert mr.words_consumed(1, mr.GAUSSIAN_ICDF_F32, 5) == 5
    assert mr.words_consumed(1, mr.GAUSSIAN_ICDF_F64, 5) == 10
    assert mr.words_consumed(2, mr.GAUSSIAN_ICDF_F64, 5) == 5
    import oracle
    for kind in (1, 2, 3, 4, 5, 6, 7, 8):
        for engine in (1, 2):
            for n in (0, 1, 2, 7, 2**40 + 1):
                assert mr.words_consumed(engine, kind, n) == oracle.words_consumed(kind, engine, n)
    assert mr.words_consumed(1, 77, 5) == 0


def _gen(L, e, kind, n, out, p0=0.0, p1=1.0, reserved=0):
    d = mr.Distribution(kind, reserved, p0, p1)
    return L.mirng_generate(e.handle, ctypes.byref(d), n, out, None)


def test_generate_validation_without_device(L):
    """Validation happens before any device call and leaves the engine as
    it was."""
    e = mr.Engine(mr.PHILOX4X32_10, 1, 10)
    fake = 0x10000
    assert _gen(L, e, mr.UNIFORM_F32, 0, None) == 0               # n == 0: no-op
    assert _gen(L, e, mr.UNIFORM_F32, 8, None) == 1               # NULL out
    assert _gen(L, e, mr.UNIFORM_F32, 8, fake + 2) == 1           # misaligned F32
    assert _gen(L, e, mr.UNIFORM_F64, 8, fake + 4) == 1           # misaligned F64
    assert _gen(L, e, mr.UNIFORM_F32, 8, fake, 1.0, 1.0) == 1     # a >= b
    assert _gen(L, e, mr.UNIFORM_F32, 8, fake, float("nan"), 1.0) == 1
    assert _gen(L, e, mr.UNIFORM_F64, 8, fake, 0.0, float("inf")) == 1
    assert _gen(L, e, mr.GAUSSIAN_F32, 8, fake, 0.0, 0.0) == 1    # stddev <= 0
    assert _gen(L, e, mr.GAUSSIAN_F32, 8, fake, 0.0, -1.0) == 1
    assert _gen(L, e, mr.GAUSSIAN_F64, 8, fake + 4) == 1         # misaligned FP64
    assert _gen(L, e, mr.GAUSSIAN_F64, 8, fake, 0.0, 0.0) == 1
    assert _gen(L, e, mr.GAUSSIAN_F64, 8, fake, float("inf"), 1.0) == 1
    # uniform int32: integers with -2^31 <= a < b <= 2^31
    i32 = mr.UNIFORM_I32
    assert _gen(L, e, i32, 8, fake + 2, 0.0, 10.0) == 1            # misaligned int32
    assert _gen(L, e, i32, 8, fake, 0.5, 10.0) == 1                # not an integer
    assert _gen(L, e, i32, 8, fake, 0.0, 10.25) == 1
    assert _gen(L, e, i32, 8, fake, 5.0, 5.0) == 1                 # a >= b
    assert _gen(L, e, i32, 8, fake, -2.0**31 - 1, 0.0) == 1        # below int32
    assert _gen(L, e, i32, 8, fake, 0.0, 2.0**31 + 1) == 1         # above int32 + 1
    assert _gen(L, e, i32, 8, fake, float("nan"), 1.0) == 1
    # inverse-CDF Gaussians: stddev > 0, finite
    assert _gen(L, e, mr.GAUSSIAN_ICDF_F32, 8, fake, 0.0, 0.0) == 1
    assert _gen(L, e, mr.GAUSSIAN_ICDF_F64, 8, fake, float("inf"), 1.0) == 1
    assert _gen(L, e, mr.GAUSSIAN_ICDF_F64, 8, fake + 4) == 1     # misaligned FP64
    assert _gen(L, e, mr.UNIFORM_F32, 8, fake, reserved=1) == 1
    assert _gen(L, e, 9, 8, fake) == 2                            # unknown kind
    assert _gen(L, e, 0, 8, fake) == 2
    d = mr.Distribution(mr.UNIFORM_F32, 0, 0.0, 1.0)
    assert L.mirng_generate(None, ctypes.byref(d), 8, fake, None) == 1
    assert L.mirng_generate(e.handle, None, 8, fake, None) == 1
    assert e.position == 10


def test_engine_create_validation(L):
    h = ctypes.c_void_p()
    assert L.mirng_engine_create(3, 1, 0, ctypes.byref(h)) == 2
    assert L.mirng_engine_create(1, 1, 0, None) == 1
    assert L.mirng_engine_destroy(None) == 0
    lim = (ctypes.c_uint64 * 4)(1, 2, 3, 4)
    e = mr.Engine(mr.MRG32K3A, 1, 0)
    before = list(e.get_state().words)
    assert L.mirng_skip_ahead_multi(e.handle, lim, 4) == 1
    assert L.mirng_skip_ahead_multi(e.handle, None, 2) == 1
    assert list(e.get_state().words) == before
    # the binding refuses offsets its 64-bit argument would truncate
    for bad in (-1, 2**64, 2**66 + 3):
        with pytest.raises(ValueError):
            mr.Engine(mr.PHILOX4X32_10, 1, bad)


def test_substream_validation(L):
    d = mr.Distribution(mr.UNIFORM_F64, 0, 0.0, 1.0)
    p = mr.Engine(mr.PHILOX4X32_10, 1, 0)
    assert L.mirng_generate_substreams(p.handle, ctypes.byref(d), 0, 4, 16, 0x10000, None) == 2
    m = mr.Engine(mr.MRG32K3A, 1, 0)
    assert L.mirng_generate_substreams(m.handle, ctypes.byref(d), 0, 4, 16, None, None) == 1
    assert L.mirng_generate_substreams(m.handle, ctypes.byref(d), 2**30, 1, 16, 0x10000,
                                       None) == 1
    assert L.mirng_generate_substreams(m.handle, ctypes.byref(d), 0, 0, 16, None, None) == 0
    assert L.mirng_generate_streams(p.handle, ctypes.byref(d), 0, 4, 16, 0x10000, None) == 2
    assert L.mirng_generate_streams(m.handle, ctypes.byref(d), 0, 4, 16, None, None) == 1
    assert L.mirng_generate_streams(m.handle, ctypes.byref(d), 2**30 - 1, 2, 16, 0x10000,
                                    None) == 1
    assert L.mirng_generate_streams(m.handle, ctypes.byref(d), 0, 4, 16, 0x10004, None) == 1


def test_philox_config_validation():
    c = mr.philox_config()
    assert c.block in (64, 128, 256, 512, 1024)
    for bad in (dict(block=100), dict(waves_per_cu=0), dict(walk=1, waves_per_cu=4097),
                dict(walk=0, waves_per_cu=4097), dict(walk=4), dict(walk=-1),
                dict(blocks_per_lane=3),
                dict(nontemporal=2), dict(reserved=1)):
        with pytest.raises(mr.MirngError):
            mr.set_philox_config(**bad)
    assert mr.philox_config().as_dict() == c.as_dict()
    prev = mr.set_philox_config(block=512, waves_per_cu=8)
    assert mr.philox_config().block == 512
    mr.set_philox_config(prev)
    assert mr.philox_config().as_dict() == c.as_dict()


def test_per_kind_philox_config_validation():
    """Per-kind, per-phase shapes: unknown kinds are UNSUPPORTED, bad shapes
    or phases INVALID_ARG (nothing changes), NULL drops the kind's own
    shape, a shape set at one phase serves that phase only, and the
    process-wide set drops them all (no device needed)."""
    import ctypes
    L = mr.lib()
    c = mr.philox_config()
    out = mr.PhiloxConfig()
    assert L.mirng_philox_config_get_kind(0, 0, ctypes.byref(out)) == 2      # UNSUPPORTED
    assert L.mirng_philox_config_get_kind(9, 0, ctypes.byref(out)) == 2
    assert L.mirng_philox_config_get_kind(mr.UNIFORM_F32, 0, None) == 1      # INVALID_ARG
    assert L.mirng_philox_config_get_kind(mr.UNIFORM_F32, 4, ctypes.byref(out)) == 1
    assert L.mirng_philox_config_get_kind(mr.UNIFORM_F32, -1, ctypes.byref(out)) == 1
    assert L.mirng_philox_config_set_kind(9, -1, None) == 2
    assert L.mirng_philox_config_set_kind(mr.UNIFORM_F32, -2, None) == 1
    bad = mr.PhiloxConfig.from_buffer_copy(c)
    bad.block = 100
    assert L.mirng_philox_config_set_kind(mr.UNIFORM_F32, -1, ctypes.byref(bad)) == 1
    assert mr.philox_config(mr.UNIFORM_F32).as_dict() == c.as_dict()
    try:
        mr.set_philox_config(kind=mr.GAUSSIAN_F32, walk=0, block=512, waves_per_cu=64)
        for ph in range(4):
            assert mr.philox_config(mr.GAUSSIAN_F32, ph).block == 512
        assert mr.philox_config().as_dict() == c.as_dict()
        assert mr.philox_config(mr.UNIFORM_F32).as_dict() == c.as_dict()
        mr.clear_philox_config(mr.GAUSSIAN_F32)
        assert mr.philox_config(mr.GAUSSIAN_F32).as_dict() == c.as_dict()
        # one phase only
        mr.set_philox_config(kind=mr.BITS_U32, phase=2, walk=2, waves_per_cu=1)
        assert mr.philox_config(mr.BITS_U32, 2).walk == 2
        for ph in (0, 1, 3):
            assert mr.philox_config(mr.BITS_U32, ph).as_dict() == c.as_dict()
        mr.clear_philox_config(mr.BITS_U32, 2)
        assert mr.philox_config(mr.BITS_U32, 2).as_dict() == c.as_dict()
        mr.set_philox_config(kind=mr.BITS_U32, walk=2, waves_per_cu=1)
        mr.set_philox_config(c)
        assert mr.philox_config(mr.BITS_U32).as_dict() == c.as_dict()
    finally:
        mr.set_philox_config(c)


def test_philox_phase_of_position_and_output():
    """Phase = (position - head * words per element) mod 4, head = elements
    before the output on the 16-byte grid; Gaussian pairs that would
    straddle the grid start at the output itself (head 0)."""
    for kind, esz, wpe in ((mr.UNIFORM_F32, 4, 1), (mr.BITS_U32, 4, 1), (mr.UNIFORM_F64, 8, 2),
                           (mr.GAUSSIAN_F32, 4, 1), (mr.GAUSSIAN_F64, 8, 2)):
        for pos in (0, 1, 2, 3, 2**40 + 1, 2**64 - 1):
            for mis in range(0, 16, esz):
                head = mis // esz
                if kind in (mr.GAUSSIAN_F32, mr.GAUSSIAN_F64) and head % 2:
                    head = 0
                want = (pos - head * wpe) % 4
                assert mr.philox_phase(kind, pos, 0x10000 + mis) == want, (kind, pos, mis)


def test_request_record_layout():
    import ctypes as ct
    dt = mr.request_dtype()
    assert dt.itemsize == 64
    for name, field in (("engine_type", "engine_type"), ("seed", "seed"), ("offset", "offset"),
                        ("n", "n"), ("out", "out")):
        assert dt.fields[name][1] == getattr(mr.Request, field).offset
    assert dt.fields["kind"][1] == mr.Request.dist.offset
    assert dt.fields["p0"][1] == mr.Request.dist.offset + mr.Distribution.p0.offset


def test_batcher_host_validation(L):
    b = mr.Batcher()
    c = b.config
    assert c.block in (64, 128, 256, 512, 1024)
    for bad in (dict(block=3), dict(waves_per_cu=0), dict(nontemporal=5), dict(reserved=1)):
        with pytest.raises(mr.MirngError):
            b.set_config(**bad)
    assert b.config.as_dict() == c.as_dict()
    reqs = mr.make_requests(3)
    # NULL table, empty batch, oversize count: rejected or accepted without a device
    assert L.mirng_generate_batch(b._h, None, 3, None) == 1
    assert L.mirng_generate_batch(b._h, reqs.ctypes.data, 0, None) == 0
    assert L.mirng_generate_batch(b._h, reqs.ctypes.data, 2**31, None) == 1
    assert L.mirng_batcher_statuses(b._h, None, 0) == 0
    assert L.mirng_batcher_statuses(b._h, reqs.ctypes.data, 1) == 1   # no batch yet
    assert L.mirng_batcher_destroy(None) == 0
    b.close()


def test_autotune_argument_validation(L):
    c = mr.PhiloxConfig()
    ms = ctypes.c_float()
    fake = ctypes.c_void_p(0x10000)
    assert L.mirng_autotune_philox(9, 1, 16, fake, None, 0, 1, 1, ctypes.byref(c),
                                   ctypes.byref(ms)) == 2
    assert L.mirng_autotune_philox(2, 1, 0, fake, None, 0, 1, 1, None, None) == 1
    assert L.mirng_autotune_philox(2, 1, 16, None, None, 0, 1, 1, None, None) == 1
    assert L.mirng_autotune_philox(2, 1, 16, fake, None, -1, 1, 1, None, None) == 1
    assert L.mirng_autotune_philox(2, 1, 16, fake, None, 0, 0, 1, None, None) == 1
    assert L.mirng_autotune_philox(2, 1, 16, fake, None, 0, 1, 0, None, None) == 1
    assert L.mirng_autotune_philox(3, 1, 16, ctypes.c_void_p(0x10004), None, 0, 1, 1,
                                   None, None) == 1
    b = mr.Batcher()
    reqs = mr.make_requests(2)
    bc = mr.BatchConfig()
    assert L.mirng_autotune_batch(None, reqs.ctypes.data, 2, None, 0, 1, 1, None, None) == 1
    assert L.mirng_autotune_batch(b._h, None, 2, None, 0, 1, 1, None, None) == 1
    assert L.mirng_autotune_batch(b._h, reqs.ctypes.data, 0, None, 0, 1, 1, None, None) == 1
    assert L.mirng_autotune_batch(b._h, reqs.ctypes.data, 2, None, 0, 65, 1,
                                  ctypes.byref(bc), None) == 1


def test_tuning_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    c = mr.TuningCache(path)
    assert c.get("gfx950/philox4x32_10/2/29") is None
    c.put("gfx950/philox4x32_10/2/29", {"config": {"walk": 0, "block": 1024}, "ms": 0.17})
    c2 = mr.TuningCache(path)
    assert c2.get("gfx950/philox4x32_10/2/29")["ms"] == 0.17
    assert mr.size_class(1 << 28) == 29 and mr.size_class(1) == 1
