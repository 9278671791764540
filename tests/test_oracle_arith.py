"""Pins of the all-arithmetic oracle (oracle/arith.py): every operation of the
coupled iteration rounded to a custom float or fixed-point type (Section IV,
"all involved calculations"; Section IV-C, Figs. 2a and 3a)."""
import math

import numpy as np
import pytest

import workloads as w
from oracle import arith, storage
from oracle import iteration as it


def rnd_float(x: float, bits: int) -> float:
    """Nearest value with `bits` stored mantissa bits (ties to even), written
    with Python scalars: frexp gives x = m 2^e, 0.5 <= |m| < 1, so m 2^(bits+1)
    holds the leading bit and `bits` more; round() is ties-to-even."""
    if x == 0.0:
        return 0.0
    m, e = math.frexp(x)
    return math.ldexp(round(m * 2.0 ** (bits + 1)), e - bits - 1)


def rnd_fixed(x: float, bits: int) -> float:
    return round(x * 2.0 ** bits) / 2.0 ** bits


@pytest.mark.parametrize("fmt,bits", [("float", 6), ("float", 11), ("fixed", 9)])
def test_product_equals_brute_force_loops(fmt, bits):
    # every product and partial sum rounded, k ascending, mirrored triangle
    r = rnd_float if fmt == "float" else rnd_fixed
    rng = np.random.default_rng(bits)
    n = 5
    x = np.vectorize(lambda v: r(v, bits))(rng.standard_normal((n, n)))
    y = np.vectorize(lambda v: r(v, bits))(rng.standard_normal((n, n)))
    got = arith.product(x, y, fmt, bits)
    for i in range(n):
        for j in range(n):
            a, b = (i, j) if i <= j else (j, i)
            acc = 0.0
            for k in range(n):
                acc = r(acc + r(float(x[k, a]) * float(y[k, b]), bits), bits)
            assert got[i, j] == acc


def test_rounding_rule_ties_to_even_and_grid():
    # 1 + 2^-11 lies halfway between 1 and 1 + 2^-10 (10 stored bits): to 1;
    # 1 + 3 2^-11 halfway between 1 + 2^-10 and 1 + 2^-9: to 1 + 2^-9
    assert arith.rnd(1.0 + 2.0 ** -11, "float", 10) == 1.0
    assert arith.rnd(1.0 + 3 * 2.0 ** -11, "float", 10) == 1.0 + 2.0 ** -9
    assert arith.rnd(-2.5 / 16, "fixed", 3) == -2.0 / 16        # -2.5 -> -2 units of 1/8
    x = np.random.default_rng(0).standard_normal(1000)
    assert np.array_equal(arith.rnd(x, "float", 7), np.vectorize(lambda v: rnd_float(v, 7))(x))


@pytest.mark.parametrize("fmt,bits,p", [("float", 10, 2), ("float", 16, 3), ("fixed", 18, 2)])
def test_diagonal_matrix_is_the_rounded_scalar_recursion(fmt, bits, p):
    # on diagonal A every product reduces to one rounded multiplication per
    # diagonal entry, so the dense iteration is the scalar recursion with
    # each operation rounded: n = rnd(1 + rnd(rnd(1 - m)/p)), c <- rnd(c n),
    # m <- rnd(n rnd(n ... m)) (p times)
    r = (lambda v: rnd_float(v, bits)) if fmt == "float" else (lambda v: rnd_fixed(v, bits))
    lam = np.array([0.013, 0.2, 0.51, 0.77, 1.0])
    a = np.diag(lam)
    iters = 8
    c_dense, errs, _ = arith.coupled_arith(a, p, iters, fmt, bits)
    sigma = math.sqrt(it.norm_1(a) * it.norm_inf(a))
    c0 = r(sigma ** (-1.0 / p))
    cp = r(c0 ** p)
    for i, l in enumerate(lam):
        c, m = c0, r(cp * r(float(l)))
        for _ in range(iters):
            nn = r(1.0 + r(r(1.0 - m) / p))
            c = r(c * nn)
            for _ in range(p):
                m = r(nn * m)
        assert c_dense[i, i] == c
    assert np.count_nonzero(c_dense - np.diag(np.diag(c_dense))) == 0
    # and the error falls towards the type's floor
    assert errs[-1] < 0.1 * errs[0]


def test_fifty_two_bits_is_the_float64_iteration():
    # with 52 stored bits rounding changes nothing: the trajectory is the
    # plain float64 coupled iteration's (which sums in another order and
    # averages instead of mirroring): the same up to float64 rounding
    a, lam, _ = w.spd_log_spectrum(40, 1e2, seed=3)
    _, e_ar, r_ar = arith.coupled_arith(a, 2, 12, "float", 52)
    _, e_64, r_64 = storage.coupled_stored(a, 2, 12, None)
    for x, y in zip(e_ar, e_64):
        assert abs(x - y) <= 1e-12
    assert e_ar[-1] < 1e-12 and r_ar[-1] < 1e-12


def test_all_arithmetic_needs_more_bits_than_storage():
    # Section IV-C: approximating only the stored matrices allows coarser
    # types than approximating every operation; more bits lower the floor
    a = w.kernel_matrix(96, seed=0, box=10.0)
    floor = {}
    for bits in (10, 16, 23):
        _, e_ar, _ = arith.coupled_arith(a, 2, 20, "float", bits)
        _, e_st, _ = storage.coupled_stored(a, 2, 20, "float", bits)
        floor[bits] = min(e_ar)
        assert min(e_ar) > min(e_st)
    assert floor[10] > 8 * floor[16] > 64 * floor[23]
    for bits in (16, 24):
        _, e_ar, _ = arith.coupled_arith(a, 2, 20, "fixed", bits)
        _, e_st, _ = storage.coupled_stored(a, 2, 20, "fixed", bits)
        assert min(e_ar) > min(e_st)
