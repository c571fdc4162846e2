"""GPU parity of the Philox4x32-10 path against the oracle, through the C ABI:
bit-exact bits and uniforms, Gaussians within 2 ulp of the FP64 transform,
at every engine-position phase, output alignment, ragged size, counter
carry and the 2^130 wrap."""
import numpy as np
import pytest

import oracle
import paper_2109_01329_amd as mr
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

KINDS = [mr.BITS_U32, mr.UNIFORM_F32, mr.UNIFORM_F64, mr.GAUSSIAN_F32, mr.GAUSSIAN_F64,
         mr.UNIFORM_I32, mr.GAUSSIAN_ICDF_F32, mr.GAUSSIAN_ICDF_F64]


def test_small_case_seed42():
    """Seed 42, offset 0: 2^20 uniform FP32 and 2^20 bits from engines at the
    same position, and one engine producing uniforms then bits."""
    n = 1 << 20
    e = mr.Engine(mr.PHILOX4X32_10, 42, 0)
    u, _ = gh.generate(e, mr.UNIFORM_F32, n)
    gh.assert_match(mr.UNIFORM_F32, u, gh.oracle_philox(42, 0, mr.UNIFORM_F32, n))
    b_same_engine, _ = gh.generate(e, mr.BITS_U32, n)
    gh.assert_match(mr.BITS_U32, b_same_engine, gh.oracle_philox(42, n, mr.BITS_U32, n))
    f = mr.Engine(mr.PHILOX4X32_10, 42, 0)
    b, _ = gh.generate(f, mr.BITS_U32, n)
    gh.assert_match(mr.BITS_U32, b, gh.oracle_philox(42, 0, mr.BITS_U32, n))
    assert e.position == 2 * n


# Counter carries: out of the low word ((1 << 34) - 5, and mid-run at
# block 2^32 - 3000), out of the low half ((1 << 66) - 3, and mid-run), out
# of the third word, and the 2^130 wrap.
CARRY_POSITIONS = [((1 << 32) - 3000) * 4 + 1, (1 << 66) - 4 * 3000 + 2]
POSITIONS = [0, 1, 2, 3, 12345, (1 << 34) - 5, (1 << 66) - 3, (1 << 98) - 1,
             (1 << 130) - 7] + CARRY_POSITIONS
SIZES = [1, 2, 3, 5, 17, 255, 4097, 70001]


@pytest.mark.parametrize("kind", KINDS)
def test_phases_alignments_sizes(kind):
    esz = mr.ELEM_BYTES[kind]
    offsets = [0, 4, 8, 12] if esz == 4 else [0, 8]
    seed = 0x0123456789ABCDEF
    for pos in POSITIONS:
        for off in offsets:
            for n in SIZES:
                e = mr.Engine(mr.PHILOX4X32_10, seed, 0)
                e.skip_ahead(pos)
                got, buf = gh.generate(e, kind, n, off)
                want = gh.oracle_philox(seed, pos, kind, n)
                gh.assert_match(kind, got, want)
                assert gh.guards_intact(buf, off, n * esz), (pos, off, n)
                assert e.position == (pos + mr.words_consumed(1, kind, n)) % (1 << 130)


@pytest.mark.parametrize("kind", KINDS)
def test_continuity_across_calls(kind):
    g = np.random.default_rng(51)
    for _ in range(6):
        seed = int(g.integers(0, 2**64, dtype=np.uint64))
        off = int(g.integers(0, 2**40, dtype=np.uint64))
        paired = kind in (mr.GAUSSIAN_F32, mr.GAUSSIAN_F64)
        n1 = int(g.integers(1, 5000)) * (2 if paired else 1)
        n2 = int(g.integers(1, 5000))
        e = mr.Engine(mr.PHILOX4X32_10, seed, off)
        a, _ = gh.generate(e, kind, n1)
        b, _ = gh.generate(e, kind, n2)
        f = mr.Engine(mr.PHILOX4X32_10, seed, off)
        c, _ = gh.generate(f, kind, n1 + n2)
        gh.assert_match(kind, np.concatenate([a, b]), gh.oracle_philox(seed, off, kind, n1 + n2))
        if kind != mr.GAUSSIAN_F32:
            assert np.array_equal(np.concatenate([a, b]).view(np.uint8), c.view(np.uint8))


@pytest.mark.parametrize("kind,p0,p1", [
    (mr.UNIFORM_F32, -3.0, 5.0), (mr.UNIFORM_F32, 1e-3, 2e-3), (mr.UNIFORM_F32, 100.0, 101.5),
    (mr.UNIFORM_F64, -1.0, 0.0), (mr.UNIFORM_F64, 1e-3, 2e-3),
    (mr.GAUSSIAN_F32, 2.5, 0.5), (mr.GAUSSIAN_F32, -1.0, 3.0),
    (mr.GAUSSIAN_F64, 2.5, 0.5), (mr.GAUSSIAN_F64, -1e3, 1e-3),
    (mr.UNIFORM_I32, -5.0, 7.0), (mr.UNIFORM_I32, -2.0**31, 2.0**31), (mr.UNIFORM_I32, 0.0, 1.0),
    (mr.UNIFORM_I32, 1000.0, 2.0**31), (mr.UNIFORM_I32, -2.0**31, -2.0**31 + 3),
    (mr.GAUSSIAN_ICDF_F32, 2.5, 0.5), (mr.GAUSSIAN_ICDF_F32, -1.0, 3.0),
    (mr.GAUSSIAN_ICDF_F64, 2.5, 0.5), (mr.GAUSSIAN_ICDF_F64, -1e3, 1e-3)])
def test_range_and_moments_parameters(kind, p0, p1):
    n = 100003
    for off in (0, 4 if mr.ELEM_BYTES[kind] == 4 else 8):
        e = mr.Engine(mr.PHILOX4X32_10, 77, 3)
        got, _ = gh.generate(e, kind, n, off, p0, p1)
        gh.assert_match(kind, got, gh.oracle_philox(77, 3, kind, n, p0, p1), p0, p1)


def test_gaussian_odd_offset_pairs_path():
    """Output 4 mod 8 bytes: the pair kernel; odd n drops the last z1."""
    for pos in (0, 1, 2, 3, (1 << 66) - 1):
        for n in (1, 2, 7, 1000, 65537):
            e = mr.Engine(mr.PHILOX4X32_10, 5, 0)
            e.skip_ahead(pos)
            got, buf = gh.generate(e, mr.GAUSSIAN_F32, n, 4)
            gh.assert_match(mr.GAUSSIAN_F32, got, gh.oracle_philox(5, pos, mr.GAUSSIAN_F32, n))
            assert gh.guards_intact(buf, 4, 4 * n)


def test_gaussian64_misaligned_pairs_path():
    """FP64 Gaussians at an output 8 mod 16 bytes (the pair would straddle
    the 16-byte grid): slots anchored at the output; odd n drops the last
    z1; every word phase."""
    for pos in (0, 1, 2, 3, (1 << 66) - 1):
        for n in (1, 2, 7, 1000, 65537):
            e = mr.Engine(mr.PHILOX4X32_10, 6, 0)
            e.skip_ahead(pos)
            got, buf = gh.generate(e, mr.GAUSSIAN_F64, n, 8)
            gh.assert_match(mr.GAUSSIAN_F64, got, gh.oracle_philox(6, pos, mr.GAUSSIAN_F64, n))
            assert gh.guards_intact(buf, 8, 8 * n)


def test_gaussian64_error_distribution():
    """Worst error of 2^20 FP64 Gaussians in units of the tolerance."""
    n = 1 << 20
    e = mr.Engine(mr.PHILOX4X32_10, 2025, 0)
    got, _ = gh.generate(e, mr.GAUSSIAN_F64, n)
    worst = gh.assert_match(mr.GAUSSIAN_F64, got, gh.oracle_philox(2025, 0, mr.GAUSSIAN_F64, n))
    print(f"worst FP64 Gaussian error: {worst:.3f} of the tolerance")


def test_many_seeds_bits():
    g = np.random.default_rng(52)
    for _ in range(40):
        seed = int(g.integers(0, 2**64, dtype=np.uint64))
        pos = int(g.integers(0, 2**62, dtype=np.uint64)) << int(g.integers(0, 66))
        n = int(g.integers(1, 20000))
        e = mr.Engine(mr.PHILOX4X32_10, seed, 0)
        e.skip_ahead(pos)
        got, _ = gh.generate(e, mr.BITS_U32, n, 4 * int(g.integers(0, 4)))
        gh.assert_match(mr.BITS_U32, got, gh.oracle_philox(seed, pos, mr.BITS_U32, n))


@pytest.mark.parametrize("kind", [mr.GAUSSIAN_ICDF_F32, mr.GAUSSIAN_ICDF_F64])
def test_icdf_error_distribution(kind):
    """Worst error of 2^18 inverse-CDF Gaussians against the oracle's
    quantile, in units of the tolerance (FP32: 2 ulp of the FP64 quantile;
    FP64: 8 ulp64)."""
    n = 1 << 18
    e = mr.Engine(mr.PHILOX4X32_10, 2026, 0)
    got, _ = gh.generate(e, kind, n)
    worst = gh.assert_match(kind, got, gh.oracle_philox(2026, 0, kind, n))
    print(f"worst inverse-CDF error (kind {kind}): {worst:.3f} of the tolerance")


def test_gaussian_error_distribution():
    """Worst error of 2^22 Gaussians in ulp of the FP64 transform."""
    n = 1 << 22
    e = mr.Engine(mr.PHILOX4X32_10, 2024, 0)
    got, _ = gh.generate(e, mr.GAUSSIAN_F32, n)
    want = gh.oracle_philox(2024, 0, mr.GAUSSIAN_F32, n)
    worst = gh.assert_match(mr.GAUSSIAN_F32, got, want)
    print(f"worst FP32 Gaussian error: {2.0 * worst:.4f} ulp")
    # in tolerance units (2 ulp): the kernel rounds once an FP64 value within
    # about 2^-28 relative of the transform (at most 0.56 ulp)
    assert worst <= 0.5 * 1.02


CONFIGS = [
    dict(walk=1, block=256, waves_per_cu=4, blocks_per_lane=1, nontemporal=0),
    dict(walk=1, block=64, waves_per_cu=1, blocks_per_lane=4, nontemporal=1),
    dict(walk=1, block=1024, waves_per_cu=64, blocks_per_lane=2, nontemporal=0),
    dict(walk=0, block=128, waves_per_cu=3, blocks_per_lane=2, nontemporal=1),
    dict(walk=0, block=64, waves_per_cu=1, blocks_per_lane=1, nontemporal=0),
    dict(walk=0, block=1024, waves_per_cu=4096, blocks_per_lane=1, nontemporal=1),
    dict(walk=1, block=512, waves_per_cu=5, blocks_per_lane=4, nontemporal=1),
    dict(walk=2, block=256, waves_per_cu=1, blocks_per_lane=1, nontemporal=0),
    dict(walk=2, block=64, waves_per_cu=1, blocks_per_lane=2, nontemporal=1),
    dict(walk=2, block=1024, waves_per_cu=1, blocks_per_lane=4, nontemporal=0),
    dict(walk=3, block=64, waves_per_cu=1, blocks_per_lane=1, nontemporal=0),
    dict(walk=3, block=256, waves_per_cu=1, blocks_per_lane=1, nontemporal=1),
    dict(walk=3, block=1024, waves_per_cu=1, blocks_per_lane=1, nontemporal=0),
    dict(walk=3, block=64, waves_per_cu=1, blocks_per_lane=2, nontemporal=0),
    dict(walk=3, block=256, waves_per_cu=1, blocks_per_lane=2, nontemporal=1),
    dict(walk=3, block=1024, waves_per_cu=1, blocks_per_lane=4, nontemporal=0),
    dict(walk=3, block=512, waves_per_cu=1, blocks_per_lane=4, nontemporal=1),
]


_ORACLE_CACHE = {}


def _oracle_cached(seed, pos, kind, n):
    """The oracle's outputs, computed once per (seed, pos, kind, n) across
    the launch shapes (they do not depend on it)."""
    key = (seed, pos, kind, n)
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = gh.oracle_philox(seed, pos, kind, n)
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("cfg", CONFIGS)
def test_outputs_invariant_under_launch_shape(cfg):
    """Every launch shape gives the oracle's values, on both walks (the
    grid-stride walk hands FP64 and Gaussian at odd positions to the
    contiguous walk)."""
    prev = mr.set_philox_config(**cfg)
    try:
        for kind in KINDS:
            for pos in (0, 1, 2, 3, 2**40 + 5, *CARRY_POSITIONS):
                for off in (0, 4 if mr.ELEM_BYTES[kind] == 4 else 8):
                    n = 100003
                    e = mr.Engine(mr.PHILOX4X32_10, 99, 0)
                    e.skip_ahead(pos)
                    got, buf = gh.generate(e, kind, n, off)
                    gh.assert_match(kind, got, _oracle_cached(99, pos, kind, n))
                    assert gh.guards_intact(buf, off, n * mr.ELEM_BYTES[kind])
    finally:
        mr.set_philox_config(prev)


@pytest.mark.parametrize("cfg", [dict(walk=3, block=b, waves_per_cu=1, blocks_per_lane=c,
                                      nontemporal=0) for b, c in ((64, 1), (256, 2), (1024, 4))])
def test_group_walk_short_runs(cfg):
    """Runs shorter than one group's tile (up to 64 x 1024 / 64 x 4 slots):
    most waves store nothing but still take part in the head exchange and
    reach the barrier; every phase, a carry, both alignments."""
    prev = mr.set_philox_config(**cfg)
    try:
        for kind in KINDS:
            for pos in (0, 1, 2, 3, CARRY_POSITIONS[0]):
                for n in (1, 5, 63, 65, 257, 4097):
                    for off in (0, 4 if mr.ELEM_BYTES[kind] == 4 else 8):
                        e = mr.Engine(mr.PHILOX4X32_10, 31, 0)
                        e.skip_ahead(pos)
                        got, buf = gh.generate(e, kind, n, off)
                        gh.assert_match(kind, got, gh.oracle_philox(31, pos, kind, n))
                        assert gh.guards_intact(buf, off, n * mr.ELEM_BYTES[kind])
    finally:
        mr.set_philox_config(prev)


AUTOTUNE_CANDIDATES = (
    [dict(walk=0, block=b, waves_per_cu=w, blocks_per_lane=1, nontemporal=nt)
     for b in (256, 512, 1024) for w in (64, 128, 256, 512, 1024) for nt in (0, 1)]
    + [dict(walk=1, block=256, waves_per_cu=8, blocks_per_lane=bpl, nontemporal=0)
       for bpl in (1, 2)]
    + [dict(walk=2, block=b, waves_per_cu=1, blocks_per_lane=i, nontemporal=nt)
       for b in (256, 1024) for i in (1, 2, 4) for nt in (0, 1)]
    + [dict(walk=3, block=b, waves_per_cu=1, blocks_per_lane=c, nontemporal=nt)
       for b in (128, 256, 512, 1024) for c in (1, 2) for nt in (0, 1)])


def test_outputs_invariant_under_every_autotuner_candidate():
    """The autotuner may install any of its candidate shapes: each gives the
    oracle's values (uniform FP32 at an odd phase and Gaussians at an even
    one, misaligned outputs)."""
    n = 65537
    want_u = gh.oracle_philox(7, 2**33 + 1, mr.UNIFORM_F32, n)
    want_g = gh.oracle_philox(7, 2, mr.GAUSSIAN_F32, n)
    prev = mr.philox_config()
    try:
        for cfg in AUTOTUNE_CANDIDATES:
            mr.set_philox_config(**cfg)
            got, _ = gh.generate(mr.Engine(mr.PHILOX4X32_10, 7, 2**33 + 1), mr.UNIFORM_F32, n, 4)
            gh.assert_match(mr.UNIFORM_F32, got, want_u)
            got, _ = gh.generate(mr.Engine(mr.PHILOX4X32_10, 7, 2), mr.GAUSSIAN_F32, n, 8)
            gh.assert_match(mr.GAUSSIAN_F32, got, want_g)
    finally:
        mr.set_philox_config(prev)
