"""Pins of the oracle's uniform int32 (reading R23) and inverse-CDF Gaussians
(reading R24, the oneMKL "icdf" method of the paper's Sec. 4.1).

The integer map is checked against its definition in rational arithmetic,
its boundary words and its monotonicity.  The normal quantile (a bisection
on libm's erf / erfc) is checked against mpmath's erfinv at 50 digits,
scipy's ndtri, known quantiles and its exact symmetry; the uniforms behind
it against exact fractions."""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.special as sp

M1 = 2**32 - 209


def _ulp64(x: float) -> float:
    return math.ulp(abs(x)) if x != 0.0 else 2.0**-1074


# ---------------------------------------------------------------- uniform int32

RANGES = [(0, 1), (-5, 7), (0, 3), (0, 1000), (-2**31, 2**31), (10, 2**31),
          (-2**31, -2**31 + 1), (-(2**31) + 5, 2**31 - 7), (0, 2**31), (123456, 123459)]


@pytest.mark.parametrize("a,b", RANGES)
def test_uniform_i32_is_floor_of_the_scaled_fraction(orc, a, b):
    """x = a + floor((w / 2^32) (b - a)), in exact rationals."""
    g = np.random.default_rng(a & 0xFFFF)
    words = [0, 1, 2**31 - 1, 2**31, 2**32 - 2, 2**32 - 1] + \
        [int(v) for v in g.integers(0, 2**32, 2000, dtype=np.uint64)]
    for w in words:
        want = a + math.floor(Fraction(w, 2**32) * (b - a))
        assert orc.uniform_i32(w, float(a), float(b)) == want, (w, a, b)


@pytest.mark.parametrize("a,b", RANGES)
def test_uniform_i32_boundaries_and_order(orc, a, b):
    """Word 0 gives a, word 2^32 - 1 gives b - 1; the value k first appears at
    word ceil(k 2^32 / r) (so each value gets floor or ceil of 2^32 / r
    words); the map never decreases."""
    r = b - a
    assert orc.uniform_i32(0, float(a), float(b)) == a
    assert orc.uniform_i32(2**32 - 1, float(a), float(b)) == b - 1
    g = np.random.default_rng(7)
    for k in sorted({1, r - 1, r // 2, *[int(x) for x in g.integers(1, max(r, 2), 50)]}):
        if not 1 <= k < r:
            continue
        first = -(-(k << 32) // r)
        assert orc.uniform_i32(first, float(a), float(b)) == a + k
        assert orc.uniform_i32(first - 1, float(a), float(b)) == a + k - 1
    w = np.sort(g.integers(0, 2**32, 4000, dtype=np.uint64))
    x = [orc.uniform_i32(int(v), float(a), float(b)) for v in w]
    assert all(p <= q for p, q in zip(x, x[1:]))


def test_uniform_i32_full_range_is_the_word(orc):
    """[-2^31, 2^31): x = w - 2^31, i.e. the word with its top bit flipped."""
    g = np.random.default_rng(8)
    w = g.integers(0, 2**32, 4096, dtype=np.uint64).astype(np.uint32)
    x = orc.apply(orc.UNIFORM_I32, orc.PHILOX, w, w.size, -2.0**31, 2.0**31)
    assert np.array_equal(x.view(np.uint32), w ^ np.uint32(0x80000000))


def test_uniform_i32_stream_and_consumption(orc):
    """One word per output for both engines; the stream is the words'."""
    assert orc.words_consumed(orc.UNIFORM_I32, orc.PHILOX, 7) == 7
    assert orc.words_consumed(orc.UNIFORM_I32, orc.MRG, 7) == 7
    words = orc.philox_words(99, 5, 64)
    x = orc.philox_generate(99, 5, orc.UNIFORM_I32, 64, -3.0, 9.0)
    assert [int(v) for v in x] == [orc.uniform_i32(int(w), -3.0, 9.0) for w in words]
    st = orc.mrg_seed(4)
    ys, _ = orc.mrg_words(st, 64)
    xm, _ = orc.mrg_generate(orc.mrg_seed(4), orc.UNIFORM_I32, 64, 0.0, 1000.0)
    assert [int(v) for v in xm] == [orc.uniform_i32(int(y), 0.0, 1000.0) for y in ys]


# ---------------------------------------------------------------- normal quantile

def _quantile_points():
    g = np.random.default_rng(24)
    pts = [0.5 + 2.0**-25, 0.5 - 2.0**-25, 0.5 + 2.0**-53, 2.0**-25, 2.0**-53, 1 - 2.0**-25,
           0.25, 0.75, 0.25 + 2.0**-40, 0.075, 0.925, 1e-300, 1e-10]
    pts += [float(x) for x in g.random(120)]
    pts += [float(10.0 ** -x) for x in g.uniform(1, 16, 40)]
    pts += [float(0.5 + (x - 0.5) * 1e-7) for x in g.random(20)]
    return pts


def test_normal_quantile_vs_mpmath(orc):
    """Within 2 ulp of sqrt(2) erfinv(2u - 1) at 50 digits."""
    mpmath.mp.dps = 50
    worst = 0.0
    for u in _quantile_points():
        z = orc.normal_quantile(u)
        exact = mpmath.sqrt(2) * mpmath.erfinv(2 * mpmath.mpf(u) - 1)
        worst = max(worst, float(abs(mpmath.mpf(z) - exact)) / _ulp64(float(exact)))
    assert worst <= 2.0, worst


def test_normal_quantile_vs_scipy(orc):
    """Within 4 ulp of scipy's ndtri (a separate implementation) over
    20000 uniforms."""
    g = np.random.default_rng(25)
    u = np.concatenate([g.random(15000), 10.0 ** -g.uniform(0, 15, 5000)])
    z = np.array([orc.normal_quantile(float(x)) for x in u])
    r = sp.ndtri(u)
    assert np.all(np.abs(z - r) <= 4 * np.spacing(np.abs(r)))


def test_normal_quantile_known_values_and_symmetry(orc):
    assert abs(orc.normal_quantile(0.975) - 1.959963984540054) <= 2 * _ulp64(1.96)
    assert abs(orc.normal_quantile(0.8413447460685429) - 1.0) <= 4 * _ulp64(1.0)
    assert abs(orc.normal_quantile(0.0013498980316300946) + 3.0) <= 8 * _ulp64(3.0)
    assert orc.normal_quantile(0.5) == 0.0
    # 1 - u is exact on the 2^-24 grid: the two ends are exact negatives
    for m in (0, 1, 5, 1000, 2**23 - 1, 2**23, 2**24 - 1):
        u = (m + 0.5) * 2.0**-24
        assert orc.normal_quantile(1.0 - u) == -orc.normal_quantile(u)
    # small |z|: z ~ sqrt(2 pi) (u - 1/2)
    z = orc.normal_quantile(0.5 + 2.0**-25)
    assert abs(z - math.sqrt(2 * math.pi) * 2.0**-25) <= 1e-12 * z
    zs = [orc.normal_quantile(x) for x in np.linspace(1e-6, 1 - 1e-6, 2001)]
    assert all(p < q for p, q in zip(zs, zs[1:]))


def test_icdf_uniforms_are_exact_midpoints(orc):
    """FP32 kind: u = ((w >> 8) + 1/2) 2^-24; FP64 kind, Philox:
    u = (floor(v / 2) + 1/2) 2^-52 from the 53-bit v of two words; MRG:
    y / (m1 + 1) rounded once; all strictly inside (0, 1)."""
    g = np.random.default_rng(26)
    for w in [0, 255, 256, 2**32 - 1] + [int(x) for x in g.integers(0, 2**32, 500,
                                                                      dtype=np.uint64)]:
        u = orc.icdf_uniform(orc.GAUSSIAN_ICDF_F32, orc.PHILOX, [w])
        assert Fraction(u) == (Fraction(w >> 8) + Fraction(1, 2)) / 2**24
        assert 0.0 < u < 1.0
        # the complement word gives the complement uniform
        assert u + orc.icdf_uniform(orc.GAUSSIAN_ICDF_F32, orc.PHILOX, [w ^ 0xFFFFFFFF]) == 1.0
    for lo, hi in [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF)] + \
            [tuple(int(x) for x in g.integers(0, 2**32, 2, dtype=np.uint64)) for _ in range(500)]:
        u = orc.icdf_uniform(orc.GAUSSIAN_ICDF_F64, orc.PHILOX, [lo, hi])
        v = ((hi << 32) | lo) >> 11
        assert Fraction(u) == (Fraction(v >> 1) + Fraction(1, 2)) / 2**52
        assert 0.0 < u < 1.0
    mpmath.mp.dps = 40
    for y in (1, 2, M1 - 1, M1, 12345):
        u = orc.icdf_uniform(orc.GAUSSIAN_ICDF_F64, orc.MRG, [y])
        assert u == orc.u01_f64_mrg(y) and 0.0 < u < 1.0


def test_icdf_apply_structure_and_consumption(orc):
    """Output i is Phi^-1 of the uniform of word i (FP32 kind, both
    engines; FP64 kind on MRG) or of words (2i, 2i + 1) (FP64 kind on
    Philox), times sd plus mean in FP64."""
    assert orc.words_consumed(orc.GAUSSIAN_ICDF_F32, orc.PHILOX, 5) == 5
    assert orc.words_consumed(orc.GAUSSIAN_ICDF_F64, orc.PHILOX, 5) == 10
    assert orc.words_consumed(orc.GAUSSIAN_ICDF_F64, orc.MRG, 5) == 5
    words = orc.philox_words(7, 3, 40)
    z = orc.philox_generate(7, 3, orc.GAUSSIAN_ICDF_F32, 40, 2.0, 0.5)
    for i in range(40):
        u = orc.icdf_uniform(orc.GAUSSIAN_ICDF_F32, orc.PHILOX, [int(words[i])])
        assert z[i] == orc.normal_quantile(u) * 0.5 + 2.0
    z64 = orc.philox_generate(7, 3, orc.GAUSSIAN_ICDF_F64, 20)
    for i in range(20):
        u = orc.icdf_uniform(orc.GAUSSIAN_ICDF_F64, orc.PHILOX,
                             [int(words[2 * i]), int(words[2 * i + 1])])
        assert z64[i] == orc.normal_quantile(u)
    ys, _ = orc.mrg_words(orc.mrg_seed(9), 20)
    zm, _ = orc.mrg_generate(orc.mrg_seed(9), orc.GAUSSIAN_ICDF_F64, 20)
    for i in range(20):
        assert zm[i] == orc.normal_quantile(orc.u01_f64_mrg(int(ys[i])))


def test_icdf_moments(orc):
    """2^15 inverse-CDF Gaussians: mean 0 and variance 1 within 5 sigma,
    and the 1% / 99% empirical quantiles near -+2.326."""
    for z in (orc.philox_generate(2025, 0, orc.GAUSSIAN_ICDF_F32, 1 << 15),
              orc.mrg_generate(orc.mrg_seed(2025), orc.GAUSSIAN_ICDF_F64, 1 << 15)[0]):
        n = z.size
        assert abs(z.mean()) < 5 / math.sqrt(n)
        assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
        lo, hi = np.quantile(z, [0.01, 0.99])
        assert abs(lo + 2.326) < 0.06 and abs(hi - 2.326) < 0.06
