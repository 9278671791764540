"""Pins of the int8-slice product oracle (oracle/slices.py) against exact
arithmetic: Python integers and fractions, brute force on tiny inputs."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import slices


def exact_product(L, R):
    """L^T R in exact rational arithmetic."""
    k, m = L.shape
    _, n = R.shape
    return [[sum(Fraction(float(L[q, i])) * Fraction(float(R[q, j])) for q in range(k))
             for j in range(n)] for i in range(m)]


def wide_range(rng, shape, lo=-6, hi=3):
    """Random signs, magnitudes log-uniform over 10^lo .. 10^hi."""
    mag = 10.0 ** rng.uniform(lo, hi, size=shape)
    return np.where(rng.random(shape) < 0.5, -mag, mag)


def test_row_exponents_bracket_the_row_maximum():
    X = np.array([[0.5, -0.25], [1.0, 3.0], [0.0, 0.0], [-1e-300, 7e-301]])
    e = slices.row_exponents(X)
    assert list(e) == [0, 2, 0, -996]
    for i in (0, 1, 3):
        m = np.abs(X[i]).max()
        assert 2.0 ** (e[i] - 1) <= m < 2.0 ** e[i]


def test_digits_stay_in_int8_range_and_round_to_nearest():
    rng = np.random.default_rng(1)
    X = wide_range(rng, (30, 50))
    X[3, :] = np.ldexp(255.0 / 256.0, 4)  # 2^7 y = 127.5 exactly: rounds to even (128), clamps
    d, e = slices.split_rows(X, 8)
    assert np.abs(d).max() <= 127
    assert (d[0, 3] == 127).all() and (d[1, 3] == 64).all()  # remainder 0.5 -> 64 next digit


def test_dyadic_inputs_reconstruct_exactly():
    rng = np.random.default_rng(2)
    m = rng.integers(-(2 ** 40), 2 ** 40, size=(20, 33))
    X = np.ldexp(m.astype(np.float64), -40)
    d, e = slices.split_rows(X, 8)
    assert np.array_equal(slices.join_rows(d, e), X)


@pytest.mark.parametrize("s", [1, 3, 5, 8])
def test_reconstruction_error_is_below_the_last_digit(s):
    rng = np.random.default_rng(3)
    X = wide_range(rng, (25, 40))
    d, e = slices.split_rows(X, s)
    # exact remainder, in fractions: |x - sum_t d_t 2^(e - beta t)| <= 2^(e - beta s)
    for i in range(X.shape[0]):
        for j in range(0, X.shape[1], 7):
            rec = sum(Fraction(int(d[t, i, j])) * Fraction(2) ** (int(e[i]) - 7 * (t + 1))
                      for t in range(s))
            assert abs(Fraction(float(X[i, j])) - rec) <= Fraction(2) ** (int(e[i]) - 7 * s)


def test_level_sums_match_brute_force():
    rng = np.random.default_rng(4)
    L = wide_range(rng, (6, 4))
    R = wide_range(rng, (6, 3))
    s = 4
    levels, el, er = slices.level_sums(L, R, s)
    a, _ = slices.split_rows(L.T, s)
    b, _ = slices.split_rows(R.T, s)
    for g in range(2, s + 2):
        for i in range(4):
            for j in range(3):
                want = 0
                for t in range(1, s + 1):
                    for u in range(1, s + 1):
                        if t + u == g:
                            want += sum(int(a[t - 1, i, q]) * int(b[u - 1, j, q]) for q in range(6))
                assert int(levels[g][i, j]) == want


@pytest.mark.parametrize("s", [1, 8])
def test_small_integer_products_are_exact(s):
    rng = np.random.default_rng(5)
    L = rng.integers(-100, 101, size=(64, 17))
    R = rng.integers(-100, 101, size=(64, 11))
    D = slices.product(L.astype(np.float64), R.astype(np.float64), s)
    assert np.array_equal(D, (L.T @ R).astype(np.float64))


def test_two_digit_inputs_lose_nothing_but_the_final_roundings():
    rng = np.random.default_rng(6)
    L = np.ldexp(rng.integers(-(2 ** 13), 2 ** 13, size=(24, 9)).astype(np.float64), -13)
    R = np.ldexp(rng.integers(-(2 ** 13), 2 ** 13, size=(24, 8)).astype(np.float64), -13)
    D = slices.product(L, R, 8)
    ex = exact_product(L, R)
    absLR = np.abs(L).T @ np.abs(R)
    for i in range(9):
        for j in range(8):
            assert abs(Fraction(float(D[i, j])) - ex[i][j]) <= Fraction(2.0 * 8 * 2.0 ** -53 * absLR[i, j])


@pytest.mark.parametrize("s", [2, 4, 6, 8, 9])
def test_random_products_stay_within_the_error_bound(s):
    rng = np.random.default_rng(7 + s)
    L = wide_range(rng, (15, 9))
    R = wide_range(rng, (15, 7))
    D = slices.product(L, R, s)
    ex = exact_product(L, R)
    bound = slices.error_bound(L, R, s)
    worst = 0.0
    for i in range(9):
        for j in range(7):
            err = abs(Fraction(float(D[i, j])) - ex[i][j])
            assert err <= Fraction(float(bound[i, j]))
            worst = max(worst, float(err) / float(bound[i, j]))
    # the bound is not vacuous: a few slices leave an error of its order
    if s <= 4:
        assert worst > 1e-3


def test_more_slices_approach_the_float64_product():
    rng = np.random.default_rng(8)
    L = rng.standard_normal((200, 60))
    R = rng.standard_normal((200, 50))
    # x87 extended precision (64-bit significand) as the reference
    ref = L.astype(np.longdouble).T @ R.astype(np.longdouble)
    errs = [float(np.abs(slices.product(L, R, s) - ref).max()) for s in (4, 6, 8, 9)]
    assert errs[0] > errs[1] > errs[2] >= errs[3]
    assert errs[3] < 1e-15 * float(np.abs(ref).max())
    # each slice is worth about beta = 7 bits until float64 rounding takes over
    assert errs[0] / errs[1] > 2 ** 12
