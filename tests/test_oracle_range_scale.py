"""Pins of three oracle steps against exact arithmetic (no GPU):

* the range transform of the paper (Sec. 4.3, r = u (b - a) + a) in FP64,
  read as one rounding of u RN(b - a) + a (R12), checked with exact
  rationals rounded to the nearest double;
* the MRG32k3a FP64 output scale y / (m1 + 1) of [L99], read as
  RN(y RN(1 / (m1 + 1))) (R11), bit for bit over edge and random outputs;
* the (mean, stddev) step of every Gaussian kind (the oneMKL distributions
  with a mean and a standard deviation, Sec. 4.1), against the exact
  transform of the same uniforms from mpmath at 50 digits.

A dropped or swapped parameter, a wrong sign or a missing rounding in any of
these fails one of the checks."""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

M1 = 2**32 - 209


def _rn(fr: Fraction) -> float:
    """The nearest double to a rational (Python's int / int true division
    is correctly rounded, ties to even)."""
    return fr.numerator / fr.denominator


RANGES64 = [(-1.0, 0.0), (1e-3, 2e-3), (10.0, 10.5), (-3.0, 5.0)]


@pytest.mark.parametrize("a,b", RANGES64)
def test_range_f64_philox_exact(orc, a, b):
    g = np.random.default_rng(4101)
    w = g.integers(0, 2**32, 2 * 3000, dtype=np.uint64).astype(np.uint32)
    edge = np.array([0, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0x800, 0, 0, 0x80000000], dtype=np.uint32)
    w = np.concatenate([edge, w])
    n = w.size // 2
    r = orc.apply(orc.UNIFORM_F64, orc.PHILOX, w, n, a, b)
    d = Fraction(b - a)                      # (b - a) rounded once in FP64
    for i in range(n):
        v = ((int(w[2 * i + 1]) << 32) | int(w[2 * i])) >> 11
        u = Fraction(v, 1 << 53)
        assert r[i] == _rn(u * d + Fraction(a)), (i, a, b)


@pytest.mark.parametrize("a,b", RANGES64)
def test_range_f64_mrg_exact(orc, a, b):
    g = np.random.default_rng(4102)
    y = np.concatenate([np.array([1, 2, M1 // 2, M1 - 1, M1], dtype=np.uint64),
                        g.integers(1, M1 + 1, 3000, dtype=np.uint64)]).astype(np.uint32)
    r = orc.apply(orc.UNIFORM_F64, orc.MRG, y, y.size, a, b)
    norm = Fraction(_rn(Fraction(1, M1 + 1)))
    d = Fraction(b - a)
    for yi, ri in zip(y, r):
        u = Fraction(_rn(int(yi) * norm))
        assert ri == _rn(u * d + Fraction(a))


def test_range_f64_unit_range_is_identity(orc):
    w = np.random.default_rng(4103).integers(0, 2**32, 2000, dtype=np.uint64).astype(np.uint32)
    u = orc.apply(orc.UNIFORM_F64, orc.PHILOX, w, 1000, 0.0, 1.0)
    for i in range(1000):
        v = ((int(w[2 * i + 1]) << 32) | int(w[2 * i])) >> 11
        assert u[i] == v / 2**53


def test_mrg_f64_scale_bit_exact(orc):
    """u = RN(y * RN(1 / (m1 + 1))) for every y tried: the edges of [1, m1],
    powers of two, values around the binade changes of u, and random y."""
    norm = _rn(Fraction(1, M1 + 1))
    assert norm == 1.0 / (M1 + 1)
    g = np.random.default_rng(4104)
    ys = [1, 2, 3, M1 - 1, M1, 2**31, 2**31 - 1, 2**31 + 1, 2**30, 2**32 - 210]
    ys += [2**k + d for k in range(1, 32) for d in (-1, 0, 1) if 1 <= 2**k + d <= M1]
    ys += [int(x) for x in g.integers(1, M1 + 1, 20000, dtype=np.uint64)]
    arr = np.array(ys, dtype=np.uint32)
    u = orc.apply(orc.UNIFORM_F64, orc.MRG, arr, arr.size, 0.0, 1.0)
    for yi, ui in zip(ys, u):
        assert ui == _rn(yi * Fraction(norm)), yi
        assert orc.u01_f64_mrg(yi) == ui
    assert 0.0 < u.min() and u.max() < 1.0


# ------------------------------------------------------------ Gaussian (mean, sd)

def _z_exact_bm32(wa, wb):
    u1 = mpmath.mpf((wa >> 8) + 1) / 2**24
    u2 = mpmath.mpf(wb >> 8) / 2**24
    r = mpmath.sqrt(-2 * mpmath.log(u1))
    return r * mpmath.cospi(2 * u2), r * mpmath.sinpi(2 * u2)


def _z_exact_bm64(u1, u2):
    r = mpmath.sqrt(-2 * mpmath.log(mpmath.mpf(u1)))
    return r * mpmath.cospi(2 * mpmath.mpf(u2)), r * mpmath.sinpi(2 * mpmath.mpf(u2))


def _quantile(u):
    return mpmath.sqrt(2) * mpmath.erfinv(2 * mpmath.mpf(u) - 1)


def _ulp64(x):
    x = abs(float(x))
    return 2.0**-1074 if x == 0.0 else float(mpmath.mpf(2) ** (mpmath.floor(mpmath.log(x, 2)) - 52))


@pytest.mark.parametrize("engine", ["philox", "mrg"])
@pytest.mark.parametrize("mean,sd", [(1.5, 0.25), (-3.0, 7.5), (1000.0, 1e-3)])
def test_gaussian_mean_sd_vs_mpmath(orc, engine, mean, sd):
    """o = RN(RN(z sd) + mean) with z the oracle's FP64 transform (within
    4 ulp64 for Box-Muller, 2 ulp64 for the quantile): |o - (z_exact sd +
    mean)| <= 4 ulp64(z) |sd| + ulp64(z sd)/2 + ulp64(o)/2, for all four
    Gaussian kinds."""
    mpmath.mp.dps = 50
    eng = orc.PHILOX if engine == "philox" else orc.MRG
    n = 64
    for kind in (orc.GAUSSIAN_F32, orc.GAUSSIAN_F64, orc.GAUSSIAN_ICDF_F32,
                 orc.GAUSSIAN_ICDF_F64):
        nw = orc.words_consumed(kind, eng, n)
        if eng == orc.PHILOX:
            w = orc.philox_words(977 + kind, 5, nw)
            o = orc.philox_generate(977 + kind, 5, kind, n, mean, sd)
        else:
            st = orc.mrg_skip(orc.mrg_seed(977 + kind), 5)
            w, _ = orc.mrg_words(st, nw)
            o, _ = orc.mrg_generate(st, kind, n, mean, sd)
        exact = []
        if kind == orc.GAUSSIAN_F32:
            for j in range(0, n, 2):
                exact += list(_z_exact_bm32(int(w[j]), int(w[j + 1])))
        elif kind == orc.GAUSSIAN_F64:
            per = 2 if eng == orc.MRG else 4
            for j in range(n // 2):
                u1, u2 = orc.gauss64_uniforms(eng, w[per * j: per * j + per])
                exact += list(_z_exact_bm64(u1, u2))
        else:
            per = 2 if (kind == orc.GAUSSIAN_ICDF_F64 and eng == orc.PHILOX) else 1
            for j in range(n):
                exact.append(_quantile(orc.icdf_uniform(kind, eng, w[per * j: per * j + per])))
        for oi, ze in zip(o, exact):
            want = ze * mpmath.mpf(sd) + mpmath.mpf(mean)
            zs = float(ze * sd)
            bound = 4 * _ulp64(ze) * sd + _ulp64(zs) / 2 + _ulp64(oi) / 2
            assert abs(mpmath.mpf(float(oi)) - want) <= bound, (kind, float(oi), float(want))


def test_gaussian_mean_sd_order_matters(orc):
    """Swapping mean and sd (or dropping either) changes the outputs: the
    check above would see such a mistake."""
    a = orc.philox_generate(5, 0, orc.GAUSSIAN_F64, 16, 1.5, 0.25)
    b = orc.philox_generate(5, 0, orc.GAUSSIAN_F64, 16, 0.25, 1.5)
    z = orc.philox_generate(5, 0, orc.GAUSSIAN_F64, 16)
    assert not np.array_equal(a, b) and not np.array_equal(a, z + 1.5)
    assert not np.array_equal(a, z * 0.25)
