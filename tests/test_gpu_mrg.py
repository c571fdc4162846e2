"""GPU parity of the MRG32k3a path against the oracle's sequential stepping,
through the C ABI: plain generate at ragged sizes and output alignments (off
the 16-byte and the 128-byte grid, where the thread ranges start at the first
line boundary and the head is written separately), continuity, and
substreams 2^76 apart."""
import numpy as np
import pytest

import oracle
import paper_2109_01329_amd as mr
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

KINDS = [mr.BITS_U32, mr.UNIFORM_F32, mr.UNIFORM_F64, mr.GAUSSIAN_F32, mr.GAUSSIAN_F64,
         mr.UNIFORM_I32, mr.GAUSSIAN_ICDF_F32, mr.GAUSSIAN_ICDF_F64]
SIZES = [1, 3, 16, 31, 33, 1000, 8191, 8193, 65537, (1 << 20) + 3]


@pytest.mark.parametrize("kind", KINDS)
def test_plain_sizes_and_alignments(kind):
    esz = mr.ELEM_BYTES[kind]
    g = np.random.default_rng(61 + kind)
    for n in SIZES:
        for off in ([0, 4, 8, 12, 16, 72] if esz == 4 else [0, 8, 16, 72]):
            seed = int(g.integers(0, 2**64, dtype=np.uint64))
            offset = int(g.integers(0, 2**40, dtype=np.uint64))
            e = mr.Engine(mr.MRG32K3A, seed, offset)
            st = oracle.mrg_skip(oracle.mrg_seed(seed), offset)
            got, buf = gh.generate(e, kind, n, off)
            gh.assert_match(kind, got, gh.oracle_mrg(st, kind, n))
            assert gh.guards_intact(buf, off, n * esz), (n, off)
            # the engine advanced by the consumed steps
            want = oracle.mrg_skip(st, mr.words_consumed(2, kind, n))
            assert [int(x) for x in e.get_state().words] == [int(x) for x in want]


@pytest.mark.parametrize("kind", KINDS)
def test_continuity(kind):
    e = mr.Engine(mr.MRG32K3A, 1234, 99)
    a, _ = gh.generate(e, kind, 5000)
    b, _ = gh.generate(e, kind, 777)
    st = oracle.mrg_skip(oracle.mrg_seed(1234), 99)
    gh.assert_match(kind, np.concatenate([a, b]), gh.oracle_mrg(st, kind, 5777))


def test_range_parameters():
    for kind, p0, p1 in [(mr.UNIFORM_F32, -2.0, 7.0), (mr.UNIFORM_F64, 10.0, 10.5),
                         (mr.GAUSSIAN_F32, 1.0, 2.0), (mr.GAUSSIAN_F64, -4.0, 0.25),
                         (mr.UNIFORM_I32, -7.0, 1000.0), (mr.UNIFORM_I32, -2.0**31, 2.0**31),
                         (mr.GAUSSIAN_ICDF_F32, 1.0, 2.0), (mr.GAUSSIAN_ICDF_F64, -4.0, 0.25)]:
        e = mr.Engine(mr.MRG32K3A, 5, 5)
        got, _ = gh.generate(e, kind, 40001, 0, p0, p1)
        st = oracle.mrg_skip(oracle.mrg_seed(5), 5)
        gh.assert_match(kind, got, gh.oracle_mrg(st, kind, 40001, p0, p1), p0, p1)


def test_bits_range():
    e = mr.Engine(mr.MRG32K3A, 0, 0)
    got, _ = gh.generate(e, mr.BITS_U32, 1 << 20)
    assert got.min() >= 1 and got.max() <= 2**32 - 209


def test_substreams_vs_sequential_stepping():
    """65536 substreams x 4096 uniform FP64 in one launch; substreams
    {0,1,2,3,4095,32768,65534,65535} x first 1024 values equal sequential
    stepping from the oracle's jump by s * 2^76."""
    import synth
    import torch
    seed = synth.substream_seed()
    cfg = synth.SUBSTREAMS
    count, per = cfg["count"], cfg["per_stream"]
    e = mr.Engine(mr.MRG32K3A, seed, 0)
    out = torch.empty(count * per, dtype=torch.float64, device="cuda")
    e.generate_substreams(mr.UNIFORM_F64, 0, count, per, out)
    torch.cuda.synchronize()
    s0 = oracle.mrg_seed(seed)
    for s in cfg["check_streams"]:
        st = oracle.mrg_skip(s0, s << 76)
        want = gh.oracle_mrg(st, mr.UNIFORM_F64, cfg["check_len"])
        got = out[s * per: s * per + cfg["check_len"]].cpu().numpy()
        gh.assert_match(mr.UNIFORM_F64, got, want)
    # whole substream 65535 and the engine itself did not move
    st = oracle.mrg_skip(s0, 65535 << 76)
    gh.assert_match(mr.UNIFORM_F64, out[65535 * per:].cpu().numpy(),
                    gh.oracle_mrg(st, mr.UNIFORM_F64, per))
    assert [int(x) for x in e.get_state().words] == [int(x) for x in s0]


@pytest.mark.parametrize("kind,first,count,n_each,off", [
    (mr.UNIFORM_F32, 5, 7, 1000, 0), (mr.BITS_U32, 123456, 3, 70001, 4),
    (mr.GAUSSIAN_F32, 2**29, 4, 333, 8), (mr.UNIFORM_F64, 0, 2, 300000, 8)])
def test_substreams_ragged(kind, first, count, n_each, off):
    esz = mr.ELEM_BYTES[kind]
    e = mr.Engine(mr.MRG32K3A, 8, 1000)
    buf = gh.device_buffer(count * n_each * esz + off + 64)
    buf.fill_(0xA5)
    e.generate_substreams(kind, first, count, n_each, int(buf.data_ptr()) + off)
    got = gh.fetch(buf, off, kind, count * n_each)
    st0 = oracle.mrg_skip(oracle.mrg_seed(8), 1000)
    for i in range(count):
        st = oracle.mrg_skip(st0, (first + i) << 76)
        gh.assert_match(kind, got[i * n_each:(i + 1) * n_each], gh.oracle_mrg(st, kind, n_each))
    assert gh.guards_intact(buf, off, count * n_each * esz)


@pytest.mark.parametrize("kind,first,count,n_each", [
    (mr.UNIFORM_F32, 3, 7, 2048), (mr.GAUSSIAN_F32, 10, 6, 4096), (mr.UNIFORM_F64, 0, 5, 4096),
    (mr.GAUSSIAN_F64, 100, 4, 2048), (mr.BITS_U32, 2**30 - 1026, 1026, 16384),
    (mr.GAUSSIAN_ICDF_F32, 77, 4, 8192), (mr.UNIFORM_I32, 5000, 3, 64 * 32)])
def test_substreams_four_per_group(kind, first, count, n_each):
    """Short line-aligned substreams run four to a workgroup (64 threads
    each, 32 to 256 steps per thread here); counts that are not a multiple
    of four leave the last group partly empty.  Each substream checked
    (all of them, or 9 spread over the 1026) equals the oracle's jump by
    s * 2^76 followed by sequential stepping."""
    esz = mr.ELEM_BYTES[kind]
    e = mr.Engine(mr.MRG32K3A, 0x5EED, 77)
    buf = gh.device_buffer(count * n_each * esz + 256)
    buf.fill_(0xA5)
    e.generate_substreams(kind, first, count, n_each, int(buf.data_ptr()) + 128)
    got = gh.fetch(buf, 128, kind, count * n_each)
    st0 = oracle.mrg_skip(oracle.mrg_seed(0x5EED), 77)
    check = range(count) if count <= 16 else [0, 1, 2, 3, 4, 511, 1023, 1024, 1025]
    for i in check:
        st = oracle.mrg_skip(st0, (first + i) << 76)
        gh.assert_match(kind, got[i * n_each:(i + 1) * n_each], gh.oracle_mrg(st, kind, n_each))
    assert gh.guards_intact(buf, 128, count * n_each * esz)


@pytest.mark.parametrize("kind,first,count,n_each,off", [
    (mr.UNIFORM_F64, 0, 5, 4097, 8), (mr.BITS_U32, 2**30 - 3, 3, 1000, 4),
    (mr.GAUSSIAN_F32, 77, 2, 12345, 0)])
def test_streams_2p127(kind, first, count, n_each, off):
    """Streams 2^127 steps apart equal the oracle's jump by s * 2^127 (its
    polynomial method, a different algorithm from the library's tables);
    substream j of stream s is reached by a further jump of 2^76 j."""
    esz = mr.ELEM_BYTES[kind]
    e = mr.Engine(mr.MRG32K3A, 0xDEADBEEF12345678, 31)
    buf = gh.device_buffer(count * n_each * esz + off + 64)
    buf.fill_(0xA5)
    e.generate_streams(kind, first, count, n_each, int(buf.data_ptr()) + off)
    got = gh.fetch(buf, off, kind, count * n_each)
    st0 = oracle.mrg_skip(oracle.mrg_seed(0xDEADBEEF12345678), 31)
    for i in range(count):
        st = oracle.mrg_skip(st0, (first + i) << 127)
        gh.assert_match(kind, got[i * n_each:(i + 1) * n_each], gh.oracle_mrg(st, kind, n_each))
    assert gh.guards_intact(buf, off, count * n_each * esz)
    # substream 3 of stream `first`: skip 2^127 first + 2^76 3, then plain
    e2 = mr.Engine(mr.MRG32K3A, 0xDEADBEEF12345678, 31)
    e2.skip_ahead((first << 127) + (3 << 76))
    got2, _ = gh.generate(e2, kind, 999)
    gh.assert_match(kind, got2, gh.oracle_mrg(oracle.mrg_skip(st0, (first << 127) + (3 << 76)),
                                              kind, 999))
