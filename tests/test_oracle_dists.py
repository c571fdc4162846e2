"""Pins of the oracle's output transforms (readings R10-R16): exactness of
the integer-to-float maps over all of their inputs, the range transform of
the paper (Sec. 4.3), and the FP64 Box-Muller ([BM58]) against mpmath at
50 digits, its special cases and its moments."""
import math

import mpmath
import numpy as np
import pytest

M1 = 2**32 - 209


def test_u01_f32_exhaustive(orc):
    """u = (w >> 8) 2^-24 for all 2^24 distinct values: exact, in
    [0, 1 - 2^-24], increasing, mean 1/2 - 2^-25 exactly."""
    k = np.arange(1 << 24, dtype=np.uint32)
    w = (k << 8) | np.uint32(0xA5)
    u = orc.apply(orc.UNIFORM_F32, orc.PHILOX, w, w.size, 0.0, 1.0)
    assert np.array_equal(u.astype(np.float64) * 2.0**24, k.astype(np.float64))
    assert u[0] == 0.0 and u[-1] == np.float32(1 - 2.0**-24) and u.max() < 1.0
    assert np.all(np.diff(u) > 0)
    assert math.fsum(u.astype(np.float64)) / u.size == 0.5 - 2.0**-25


def test_u01_f64_words(orc):
    g = np.random.default_rng(31)
    w = g.integers(0, 2**32, 2 * 4096, dtype=np.uint64).astype(np.uint32)
    u = orc.apply(orc.UNIFORM_F64, orc.PHILOX, w, 4096, 0.0, 1.0)
    v = (w[1::2].astype(np.uint64) << np.uint64(32)) | w[0::2].astype(np.uint64)
    for ui, vi in zip(u, v):
        assert int(ui * 2.0**53) == int(vi) >> 11
    ext = np.array([0, 0, 0xFFFFFFFF, 0xFFFFFFFF], dtype=np.uint32)
    e = orc.apply(orc.UNIFORM_F64, orc.PHILOX, ext, 2, 0.0, 1.0)
    assert e[0] == 0.0 and e[1] == 1.0 - 2.0**-53


def test_u01_f64_mrg(orc):
    """u = y / (m1 + 1) rounded once; strictly inside (0, 1)."""
    mpmath.mp.dps = 40
    for y in (1, 2, 12345, M1 // 2, M1 - 1, M1):
        u = orc.u01_f64_mrg(y)
        exact = mpmath.mpf(y) / (M1 + 1)
        # y * RN(1/(m1+1)) rounded: within 1 ulp of the exact quotient
        assert abs(mpmath.mpf(u) - exact) <= mpmath.mpf(2) ** -52 * exact
        assert 0.0 < u < 1.0


def test_mrg_f32_below_one(orc):
    u = orc.apply(orc.UNIFORM_F32, orc.MRG, np.array([M1, 1], dtype=np.uint32), 2, 0.0, 1.0)
    assert u[0] == np.float32(1 - 2.0**-24) and u[1] == 0.0


@pytest.mark.parametrize("a,b", [(0.0, 1.0), (-3.0, 5.0), (1e-3, 2e-3), (-1.0, 0.0),
                                 (100.0, 101.5)])
def test_range_transform_fma(orc, a, b):
    """r = fma(u, RN32(b - a), RN32(a)) computed once; checked against exact
    rational arithmetic rounded to float32 by numpy."""
    g = np.random.default_rng(32)
    w = g.integers(0, 2**32, 1000, dtype=np.uint64).astype(np.uint32)
    r = orc.apply(orc.UNIFORM_F32, orc.PHILOX, w, 1000, a, b)
    d = np.float32(b - a)
    a32 = np.float32(a)
    from fractions import Fraction
    for wi, ri in zip(w, r):
        u = Fraction(int(wi) >> 8, 1 << 24)
        exact = u * Fraction(float(d)) + Fraction(float(a32))
        assert float(ri) == float(np.float32(_round_to_f32(exact)))


def _round_to_f32(fr):
    """Round a Fraction to the nearest float32 (ties to even)."""
    x = float(fr)                         # nearest double
    f = np.float32(x)
    # correct a possible double rounding: compare the two float32 neighbours
    cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]
    from fractions import Fraction
    best = min(cands, key=lambda c: (abs(Fraction(float(c)) - fr),
                                     int(np.float32(c).view(np.uint32)) & 1))
    return best


def _bm_mp(wa, wb):
    mpmath.mp.dps = 50
    u1 = mpmath.mpf((wa >> 8) + 1) / 2**24
    u2 = mpmath.mpf(wb >> 8) / 2**24
    r = mpmath.sqrt(-2 * mpmath.log(u1))
    return r * mpmath.cospi(2 * u2), r * mpmath.sinpi(2 * u2)


def _ulp32(x):
    x = abs(float(x))
    if x == 0.0:
        return 2.0**-149
    return 2.0 ** (math.floor(math.log2(x)) - 23)


def test_box_muller_vs_mpmath(orc):
    """The FP64 transform must be far inside the 2-ulp FP32 band: error
    below 1e-4 ulp32 of the exact value on random and edge pairs."""
    g = np.random.default_rng(33)
    pairs = [(int(a), int(b)) for a, b in g.integers(0, 2**32, (3000, 2), dtype=np.uint64)]
    edges = [0, 0xFF, 0x100, 0x7FFFFFFF, 0x80000000, 0xFFFFFEFF, 0xFFFFFFFF,
             0x40000000, 0xC0000000, 0x3FFFFF00, 0x20000000, 0xBFFFFF00]
    pairs += [(a, b) for a in edges for b in edges]
    worst = 0.0
    for wa, wb in pairs:
        z0, z1 = orc.box_muller(wa, wb)
        e0, e1 = _bm_mp(wa, wb)
        for z, e in ((z0, e0), (z1, e1)):
            if e == 0:
                assert z == 0.0
                continue
            worst = max(worst, float(abs(mpmath.mpf(z) - e)) / _ulp32(e))
    assert worst < 1e-4


def test_box_muller_special_cases(orc):
    """u1 = 1 gives +-0; u2 in {0, 1/4, 1/2, 3/4} gives exact axis values."""
    top = 0xFFFFFFFF  # (w >> 8) + 1 = 2^24 -> u1 = 1
    for wb in (0, 0x40000000, 0x80000000, 0xC0000000, 0x12345678):
        z0, z1 = orc.box_muller(top, wb)
        assert z0 == 0.0 and z1 == 0.0
    wa = 0x12345600
    r = math.sqrt(-2.0 * math.log(((wa >> 8) + 1) * 2.0**-24))
    assert orc.box_muller(wa, 0) == (r, 0.0)
    assert orc.box_muller(wa, 0x40000000) == (0.0, r)
    assert orc.box_muller(wa, 0x80000000) == (-r, 0.0)
    assert orc.box_muller(wa, 0xC0000000) == (0.0, -r)


def test_box_muller_bound(orc):
    """|z| <= sqrt(-2 ln 2^-24) = sqrt(48 ln 2)."""
    z0, z1 = orc.box_muller(0, 0)
    assert z0 == math.sqrt(48 * math.log(2)) and z1 == 0.0


def test_gaussian_moments(orc):
    n = 1 << 20
    z = orc.philox_generate(2024, 0, orc.GAUSSIAN_F32, n)
    m = z.mean(); v = z.var()
    s = ((z - m) ** 3).mean() / v**1.5
    k = ((z - m) ** 4).mean() / v**2
    se = 1 / math.sqrt(n)
    assert abs(m) < 5 * se
    assert abs(v - 1) < 5 * math.sqrt(2) * se
    assert abs(s) < 5 * math.sqrt(6) * se
    assert abs(k - 3) < 5 * math.sqrt(24) * se
    assert np.abs(z).max() <= math.sqrt(48 * math.log(2))


def test_uniform_moments(orc):
    n = 1 << 20
    u = orc.philox_generate(7, 12345, orc.UNIFORM_F32, n).astype(np.float64)
    bound = 6 * math.sqrt(1 / (12 * n))
    assert abs(u.mean() - (0.5 - 2.0**-25)) < bound
    assert abs(u.var() - 1 / 12) < 6 * math.sqrt(1 / (180 * n))
    st = orc.mrg_seed(7)
    um, _ = orc.mrg_generate(st, orc.UNIFORM_F64, n)
    assert abs(um.mean() - 0.5) < bound


def test_gaussian_odd_n_and_consumption(orc):
    """R14: odd n uses 2*ceil(n/2) words and drops the last z1."""
    assert orc.words_consumed(orc.GAUSSIAN_F32, orc.PHILOX, 5) == 6
    assert orc.words_consumed(orc.UNIFORM_F64, orc.PHILOX, 5) == 10
    assert orc.words_consumed(orc.UNIFORM_F64, orc.MRG, 5) == 5
    z5 = orc.philox_generate(3, 1, orc.GAUSSIAN_F32, 5)
    z6 = orc.philox_generate(3, 1, orc.GAUSSIAN_F32, 6)
    assert np.array_equal(z5, z6[:5])


def test_gaussian_mean_sd(orc):
    z = orc.philox_generate(3, 0, orc.GAUSSIAN_F32, 64)
    y = orc.philox_generate(3, 0, orc.GAUSSIAN_F32, 64, 2.5, 0.5)
    assert np.array_equal(y, z * 0.5 + 2.5)


# ---------------------------------------------------------------- Gaussian FP64 (R21)

def _ulp64(x):
    x = abs(float(x))
    if x == 0.0:
        return 2.0**-1074
    return 2.0 ** (math.floor(math.log2(x)) - 52)


def _bm64_mp(u1, u2):
    mpmath.mp.dps = 50
    r = mpmath.sqrt(-2 * mpmath.log(mpmath.mpf(u1)))
    return r * mpmath.cospi(2 * mpmath.mpf(u2)), r * mpmath.sinpi(2 * mpmath.mpf(u2))


def test_box_muller64_vs_mpmath(orc):
    """The FP64 Gaussian transform is within 4 ulp64 of the exact value of the
    same two FP64 uniforms (libm log, sqrt and sin/cos after the exact
    quarter-turn reduction), on random and edge pairs."""
    g = np.random.default_rng(34)
    us = [(float(a), float(b)) for a, b in g.random((2000, 2))]
    us = [(1.0 - a if a < 1.0 else 1.0, b) for a, b in us]     # u1 in (0, 1]
    edges1 = [2.0**-53, 2.0**-30, 0.5, 1.0 - 2.0**-53, 1.0 - 2.0**-30, 0.3, 0.999]
    edges2 = [0.0, 2.0**-53, 0.125, 0.25 - 2.0**-53, 0.375, 0.5, 0.75, 1.0 - 2.0**-53]
    us += [(a, b) for a in edges1 for b in edges2]
    worst = 0.0
    for u1, u2 in us:
        z0, z1 = orc.box_muller64(u1, u2)
        e0, e1 = _bm64_mp(u1, u2)
        for z, e in ((z0, e0), (z1, e1)):
            if e == 0:
                assert z == 0.0
                continue
            worst = max(worst, float(abs(mpmath.mpf(z) - e)) / _ulp64(e))
    assert worst <= 4.0, worst


def test_gauss64_uniforms_from_words(orc):
    """Philox: u1 = (v_a + 1) 2^-53 from words (w0, w1), u2 = v_b 2^-53 from
    (w2, w3), first word low; MRG: y / (m1 + 1) for each output."""
    M1 = 2**32 - 209
    g = np.random.default_rng(35)
    for w in g.integers(0, 2**32, (200, 4), dtype=np.uint64):
        w = [int(x) for x in w]
        va = ((w[1] << 32) | w[0]) >> 11
        vb = ((w[3] << 32) | w[2]) >> 11
        assert orc.gauss64_uniforms(orc.PHILOX, w) == ((va + 1) / 2**53, vb / 2**53)
        y = [1 + x % M1 for x in w[:2]]
        u1, u2 = orc.gauss64_uniforms(orc.MRG, y)
        for u, yy in ((u1, y[0]), (u2, y[1])):
            mpmath.mp.dps = 40
            assert abs(mpmath.mpf(u) - mpmath.mpf(yy) / (M1 + 1)) <= mpmath.mpf(2)**-52 * u
    assert orc.gauss64_uniforms(orc.PHILOX, [0] * 4) == (2.0**-53, 0.0)
    assert orc.gauss64_uniforms(orc.PHILOX, [0xFFFFFFFF] * 4) == (1.0, 1.0 - 2.0**-53)


def test_gaussian64_words_per_pair_and_consumption(orc):
    """Pair j of a Philox Gaussian FP64 stream uses words 4j .. 4j + 3; MRG
    outputs 2j, 2j + 1; odd n drops the last z1 (R21)."""
    assert orc.words_consumed(orc.GAUSSIAN_F64, orc.PHILOX, 5) == 12
    assert orc.words_consumed(orc.GAUSSIAN_F64, orc.MRG, 5) == 6
    w = orc.philox_words(11, 6, 16)
    z = orc.philox_generate(11, 6, orc.GAUSSIAN_F64, 7)
    for j in range(4):
        u1, u2 = orc.gauss64_uniforms(orc.PHILOX, w[4 * j: 4 * j + 4])
        z0, z1 = orc.box_muller64(u1, u2)
        assert z[2 * j] == z0
        if 2 * j + 1 < 7:
            assert z[2 * j + 1] == z1
    st = orc.mrg_seed(11)
    y, _ = orc.mrg_words(st, 8)
    zm, _ = orc.mrg_generate(st, orc.GAUSSIAN_F64, 8)
    for j in range(4):
        assert tuple(zm[2 * j: 2 * j + 2]) == orc.box_muller64(
            *orc.gauss64_uniforms(orc.MRG, y[2 * j: 2 * j + 2]))
    z8 = orc.philox_generate(11, 6, orc.GAUSSIAN_F64, 8)
    assert np.array_equal(z, z8[:7])


def test_gaussian64_distribution(orc):
    """2^20 Philox and 2^19 MRG Gaussian FP64 outputs pass a
    Kolmogorov-Smirnov test against the standard normal (scipy) at the 0.1%
    level, with the moments of N(0, 1)."""
    from scipy import stats
    for z in (orc.philox_generate(2025, 0, orc.GAUSSIAN_F64, 1 << 20),
              orc.mrg_generate(orc.mrg_seed(2025), orc.GAUSSIAN_F64, 1 << 19)[0]):
        n = z.size
        assert stats.kstest(z, "norm").pvalue > 1e-3
        se = 1 / math.sqrt(n)
        assert abs(z.mean()) < 5 * se
        assert abs(z.var() - 1) < 5 * math.sqrt(2) * se


def test_gaussian64_special_cases(orc):
    """u1 = 1 gives +-0; u2 on the axes gives exact axis values; the largest
    radius is sqrt(-2 ln 2^-53)."""
    for u2 in (0.0, 0.25, 0.5, 0.75, 0.3):
        z0, z1 = orc.box_muller64(1.0, u2)
        assert z0 == 0.0 and z1 == 0.0
    r = math.sqrt(-2.0 * math.log(0.3))
    assert orc.box_muller64(0.3, 0.0) == (r, 0.0)
    assert orc.box_muller64(0.3, 0.25) == (0.0, r)
    assert orc.box_muller64(0.3, 0.5) == (-r, 0.0)
    assert orc.box_muller64(0.3, 0.75) == (0.0, -r)
    z0, _ = orc.box_muller64(2.0**-53, 0.0)
    assert z0 == math.sqrt(-2.0 * math.log(2.0**-53))
