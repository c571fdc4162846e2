"""Pins of the oracle's Philox4x32-10 engine ([S11]) and its word-position
arithmetic (readings R2-R5), each against something other than the oracle:
an independent library implementation, closed forms, or Python integers."""
import math

import mpmath
import numpy as np
import pytest

from oracle import tiny_ref

MASK64 = (1 << 64) - 1


def _ctr_add(ctr, k):
    v = sum(int(x) << (64 * i) for i, x in enumerate(ctr)) + k
    v %= 1 << 256
    return np.array([(v >> (64 * i)) & MASK64 for i in range(4)], dtype=np.uint64)


def test_round_structure_matches_numpy_philox4x64(orc):
    """The round body is shared by the W=32 and W=64 instances; the W=64
    instance must reproduce numpy's Philox4x64-10 bit for bit.  numpy
    increments its counter before each block, so its block j uses c+1+j."""
    g = np.random.default_rng(11)
    for _ in range(200):
        key = g.integers(0, 2**64, 2, dtype=np.uint64)
        ctr = g.integers(0, 2**64, 4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        raw = bg.random_raw(12)
        ours = np.concatenate([orc.philox4x64(_ctr_add(ctr, 1 + j), key) for j in range(3)])
        assert np.array_equal(ours, raw)


def test_round_structure_carry_cases_vs_numpy(orc):
    """Counters that carry across all 64-bit limbs."""
    key = np.array([0, MASK64], dtype=np.uint64)
    for ctr in ([MASK64, 0, 0, 0], [MASK64, MASK64, MASK64, MASK64 - 1],
                [MASK64] * 4, [0, 0, 0, 0]):
        ctr = np.array(ctr, dtype=np.uint64)
        raw = np.random.Philox(key=key, counter=ctr).random_raw(8)
        ours = np.concatenate([orc.philox4x64(_ctr_add(ctr, 1 + j), key) for j in range(2)])
        assert np.array_equal(ours, raw)


def _frac_bits(x, bits):
    mpmath.mp.dps = 60
    return int(mpmath.floor(mpmath.frac(x) * mpmath.mpf(2) ** bits))


def test_weyl_constants_closed_form(orc):
    """Key increments are the leading bits of frac(golden ratio) and of
    sqrt(3) - 1 ([S11])."""
    mpmath.mp.dps = 60
    phi = (1 + mpmath.sqrt(5)) / 2
    s3 = mpmath.sqrt(3) - 1
    c = orc.philox_constants()
    assert c["W32"] == (_frac_bits(phi, 32), _frac_bits(s3, 32))
    assert c["W64"] == (_frac_bits(phi, 64), _frac_bits(s3, 64))


def test_c_oracle_equals_python_integers(orc):
    g = np.random.default_rng(12)
    for _ in range(300):
        ctr = [int(v) for v in g.integers(0, 2**32, 4, dtype=np.uint64)]
        key = [int(v) for v in g.integers(0, 2**32, 2, dtype=np.uint64)]
        assert list(orc.philox4x32(ctr, key)) == tiny_ref.philox(ctr, key)


def test_bijection_distinct_outputs(orc):
    """A bijection of the counter: consecutive counters give distinct
    128-bit outputs, and one output bit flips about half the bits."""
    key = [0x01234567, 0x89ABCDEF]
    flips = []
    g = np.random.default_rng(13)
    for _ in range(2000):
        ctr = [int(v) for v in g.integers(0, 2**32, 4, dtype=np.uint64)]
        bit = int(g.integers(0, 128))
        ctr2 = list(ctr)
        ctr2[bit // 32] ^= 1 << (bit % 32)
        a = orc.philox4x32(ctr, key)
        b = orc.philox4x32(ctr2, key)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    m = float(np.mean(flips))
    # binomial(128, 1/2): mean 64, sd of the mean 5.66/sqrt(2000) = 0.13
    assert abs(m - 64.0) < 0.6


@pytest.mark.parametrize("seed,pos,n", [
    (42, 0, 37), (0xFFFFFFFFFFFFFFFF, 3, 21), (7, (1 << 34) - 8, 24),
    (7, (1 << 66) - 9, 24), (7, (1 << 98) - 7, 24), (9, (1 << 130) - 6, 16),
])
def test_word_positions_vs_python_integers(orc, seed, pos, n):
    """Counter layout, word order and carries at 2^34 (c0 -> c1), 2^66,
    2^98 and the wrap at 2^130, against big-integer arithmetic."""
    assert list(orc.philox_words(seed, pos, n)) == tiny_ref.philox_words(seed, pos, n)


def test_wrap_at_2_130(orc):
    a = orc.philox_words(5, (1 << 130) - 2, 6)
    b = orc.philox_words(5, 0, 4)
    assert np.array_equal(a[2:], b)


def test_continuity_and_skip(orc):
    """words(p, n1) ++ words(p+n1, n2) == words(p, n1+n2); dropping k words
    equals starting k later."""
    g = np.random.default_rng(14)
    for _ in range(50):
        seed = int(g.integers(0, 2**64, dtype=np.uint64))
        p = int(g.integers(0, 2**62, dtype=np.uint64)) << int(g.integers(0, 60))
        n1, n2 = int(g.integers(0, 33)), int(g.integers(0, 33))
        whole = orc.philox_words(seed, p, n1 + n2)
        assert np.array_equal(whole[:n1], orc.philox_words(seed, p, n1))
        assert np.array_equal(whole[n1:], orc.philox_words(seed, p + n1, n2))


def test_key_from_seed(orc):
    """R2: key = (lo32(seed), hi32(seed)); word 4b+j is word j of block b."""
    seed = 0x1122334455667788
    blk = orc.philox4x32([5, 0, 0, 0], [0x55667788, 0x11223344])
    assert np.array_equal(orc.philox_words(seed, 20, 4), blk)


def test_small_case_runs_under_a_second(orc):
    """2^20 uniform FP32 plus 2^20 bits from seed 42, one core, < 1 s."""
    import time
    t0 = time.perf_counter()
    u = orc.philox_generate(42, 0, orc.UNIFORM_F32, 1 << 20)
    b = orc.philox_generate(42, 0, orc.BITS_U32, 1 << 20)
    dt = time.perf_counter() - t0
    assert dt < 1.0
    assert u.dtype == np.float32 and b.dtype == np.uint32
    # same engine position: uniforms are the bits' top 24 bits
    assert np.array_equal(u * np.float32(2**24), (b >> 8).astype(np.float32))
