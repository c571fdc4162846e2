"""Pins of the oracle's MRG32k3a engine ([L99]) and its polynomial jump:
primitivity of both characteristic polynomials (the full period m^3 - 1 that
[L99] states for each component), brute-force stepping, and agreement with
plain matrix powers computed over Python integers."""
import numpy as np
import pytest
import sympy

from oracle import tiny_ref

M1 = 2**32 - 209
M2 = 2**32 - 22853


def test_moduli_and_constants(orc):
    c = orc.mrg_constants()
    assert c["m1"] == M1 and c["m2"] == M2
    assert sympy.isprime(M1) and sympy.isprime(M2)


def _component(st, comp):
    return [int(v) for v in (st[:3] if comp == 0 else st[3:])]


@pytest.mark.parametrize("comp,m", [(0, M1), (1, M2)])
def test_full_period_group_order(orc, comp, m):
    """A^(m^3 - 1) = I and A^((m^3 - 1)/q) != I for each prime q | m^3 - 1:
    the characteristic polynomial is primitive, so the component has the
    maximal period m^3 - 1."""
    order = m**3 - 1
    g = np.random.default_rng(21 + comp)
    st = [int(v) for v in g.integers(1, M2, 6, dtype=np.uint64)]
    assert _component(orc.mrg_skip(st, order), comp) == _component(st, comp)
    for q in sympy.factorint(order):
        jumped = _component(orc.mrg_skip(st, order // q), comp)
        assert jumped != _component(st, comp), q


def test_skip_equals_stepping_bruteforce(orc):
    st0 = orc.mrg_seed(0xDEADBEEF12345678)
    ys, _ = orc.mrg_words(st0, 4096)
    st = np.array(st0)
    for n in range(0, 4097):
        if n:
            _, st = orc.mrg_words(st, 1)
        if n % 97 == 0 or n < 64 or n == 4096:
            assert np.array_equal(orc.mrg_skip(st0, n), st), n
    g = np.random.default_rng(22)
    for n in g.integers(0, 10**6, 20):
        _, st_n = orc.mrg_words(st0, int(n))
        assert np.array_equal(orc.mrg_skip(st0, int(n)), st_n)


def test_c_stepping_equals_python_integers(orc):
    for seed in (0, 1, 12345, 0xFFFFFFFFFFFFFFFF, 0x00000000FFFFFF00):
        st = orc.mrg_seed(seed)
        assert [int(v) for v in st] == tiny_ref.mrg_seed(seed)
        ys, st2 = orc.mrg_words(st, 500)
        ys_ref, st2_ref = tiny_ref.mrg_words(tiny_ref.mrg_seed(seed), 500)
        assert [int(v) for v in ys] == ys_ref
        assert [int(v) for v in st2] == st2_ref


@pytest.mark.parametrize("n", [1, 2, 3, 1000, 2**40 + 17, 2**76, 3 * 2**76,
                               2**127, 2**191 + 12345, 2**192 - 1])
def test_polynomial_jump_equals_matrix_power(orc, n):
    st = [int(v) for v in np.random.default_rng(n % 1000).integers(0, M2, 6, dtype=np.uint64)]
    assert [int(v) for v in orc.mrg_skip(st, n)] == tiny_ref.mrg_skip(st, n)


def test_jump_additivity(orc):
    st = orc.mrg_seed(99)
    a, b = 2**76 * 5, 2**127 + 3
    assert np.array_equal(orc.mrg_skip(orc.mrg_skip(st, a), b), orc.mrg_skip(st, a + b))


def test_output_range_and_state_bounds(orc):
    g = np.random.default_rng(23)
    for seed in g.integers(0, 2**64, 20, dtype=np.uint64):
        ys, st = orc.mrg_words(orc.mrg_seed(int(seed)), 2000)
        assert ys.min() >= 1 and ys.max() <= M1
        assert all(int(v) < M1 for v in st[:3]) and all(int(v) < M2 for v in st[3:])


def test_output_equal_components_gives_m1(orc):
    """R9: when x1 == x2 the combined output is m1, never 0."""
    # a state whose next x1 and x2 are both 0: x1[n] = 1403580 s1 - 810728 s0
    st = [0, 0, 5, 0, 7, 0]
    y, _ = tiny_ref.mrg_step(st)
    ys, _ = orc.mrg_words(st, 1)
    assert int(ys[0]) == y == M1


def test_seed_never_all_zero(orc):
    for seed in (0, M1, M1 | (M2 << 32)):
        st = orc.mrg_seed(seed)
        assert any(int(v) for v in st[:3]) and any(int(v) for v in st[3:])
