"""Pins of the approximate-storage oracle (oracle/storage.py): the rounding
rules against the rounding emulator and closed forms, the dense iteration
against its scalar recursion on diagonal matrices, the floors against the
number of stored bits, and the behaviour Section IV-C reports."""
import numpy as np
import pytest

import workloads as w
from oracle import rounding, storage


def test_float_store_is_the_emulators_rounding_and_survives_tiny_values():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(2000) * 10.0 ** rng.uniform(-200, 200, 2000)
    for bits in (1, 2, 7, 10, 23, 52):
        assert np.array_equal(storage.store(x, "float", bits), rounding.round_custom(x, bits))
    tiny = np.array([5e-324, -1e-310, 3e-300, 0.0, -0.0])
    out = storage.store(tiny, "float", 10)
    assert np.isfinite(out).all()
    assert np.array_equal(storage.store(tiny, "float", 52), tiny)
    assert storage.store(np.array([1.0 + 2.0 ** -11]), "float", 10)[0] == 1.0   # tie to even
    assert storage.store(np.array([1.0 + 3 * 2.0 ** -11]), "float", 10)[0] == 1.0 + 2.0 ** -9


def test_fixed_store_rounds_to_the_fractional_grid():
    x = np.array([0.3, -0.3, 1.0 / 32.0, 3.0 / 32.0, 1e6 + 0.1])
    y = storage.store(x, "fixed", 4)
    assert np.array_equal(y, [0.3125, -0.3125, 0.0, 0.125, 1e6 + 0.125])
    assert np.array_equal(storage.store(x, "fixed", 4) * 16, np.rint(x * 16))


def scalar_stored(lam, p, iters, fmt, bits):
    """The same storage rule applied to one eigenvalue of a diagonal A."""
    st = lambda v: storage.store(np.array([v]), fmt, bits)[0]
    lam = np.asarray(lam, dtype=np.float64)
    s2 = np.abs(lam).max() ** 2
    sigma = np.sqrt(s2)
    c0, cp = sigma ** (-1.0 / p), 1.0 / sigma
    out = []
    for l in lam:
        lt = st(l)
        m0 = cp * lt
        c, m, nn = st(c0), st(m0), st(1.0 + (1.0 - m0) * (1.0 / p))
        for _ in range(iters):
            c_new = st(c * nn)
            x = m
            for _ in range(p):
                x = st(nn * x)
            c, m, nn = c_new, x, st((p + 1.0) / p + (-1.0 / p) * x)
        out.append(c)
    return np.array(out)


@pytest.mark.parametrize("fmt,bits", [("float", 10), ("float", 3), ("fixed", 12)])
@pytest.mark.parametrize("p", [1, 2])
def test_diagonal_matrix_follows_the_scalar_recursion_bit_for_bit(fmt, bits, p):
    lam = np.geomspace(0.02, 1.0, 24)
    c, _, _ = storage.coupled_stored(np.diag(lam), p, 12, fmt, bits)
    assert np.array_equal(np.diag(c), scalar_stored(lam, p, 12, fmt, bits))
    assert np.count_nonzero(c - np.diag(np.diag(c))) == 0


def test_52_stored_bits_change_nothing():
    a, _, _ = w.spd_log_spectrum(40, 1e2, seed=1)
    c52, e52, _ = storage.coupled_stored(a, 2, 15, "float", 52)
    c64, e64, _ = storage.coupled_stored(a, 2, 15, None)
    assert np.array_equal(c52, c64) and e52 == e64


@pytest.mark.parametrize("fmt,bits_list", [("float", (10, 16, 23, 30)), ("fixed", (12, 18, 24, 30))])
def test_floor_falls_with_every_stored_bit(fmt, bits_list):
    a, _, _ = w.spd_log_spectrum(64, 10.0, seed=2)
    floors = [min(storage.coupled_stored(a, 2, 20, fmt, b)[1]) for b in bits_list]
    for f0, f1 in zip(floors, floors[1:]):
        assert f1 < f0 * 2.0 ** -4   # 6 or 7 more bits: at least 2^4 lower
    root_norm = np.linalg.norm(np.linalg.inv(np.linalg.cholesky(a)))  # ~ ||A^{-1/2}||_F
    assert floors[-1] < 2.0 ** -(bits_list[-1] - 12) * root_norm


def test_section_iv_observations_under_this_reading():
    """Sec. IV-C reports, for its well-conditioned overlap matrices at p = 2:
    storage-only float with 10 stored bits converges to a low floor; even 2
    stored bits still converge (to a coarse floor); 4 fractional fixed-point
    bits suffice to converge. The oracle at kappa = 10 shows the same."""
    a, _, _ = w.spd_log_spectrum(96, 10.0, seed=3)
    _, e10, _ = storage.coupled_stored(a, 2, 25, "float", 10)
    _, e2, _ = storage.coupled_stored(a, 2, 25, "float", 2)
    _, x4, _ = storage.coupled_stored(a, 2, 25, "fixed", 4)
    assert min(e10) < 2e-3 * e10[0] and e10[-1] < 2e-3 * e10[0]
    assert e2[-1] < 0.3 * e2[0]
    assert x4[-1] < 0.6 * x4[0]
