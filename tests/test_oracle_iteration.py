"""Pins of the FP64 oracle against mathematics and library routines that are
independent of it (Section II, eqs. (1)-(3))."""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as w
from oracle import iteration as it

U = np.finfo(np.float64).eps / 2


def _spd(n, kappa, seed):
    a, lam, q = w.spd_log_spectrum(n, kappa, seed=seed)
    return a, lam, q


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_eig_root_matches_scipy_fractional_power(p):
    a, _, _ = _spd(48, 1e3, 3)
    ref = np.real(scipy.linalg.fractional_matrix_power(a, -1.0 / p))
    assert it.rel_fro(it.eig_root(a, p), ref) < 1e-10


def test_eig_root_hand_worked_2x2():
    # A = [[2,1],[1,2]]: eigenvalues 1 and 3 with eigenvectors (1,-1)/sqrt2 and
    # (1,1)/sqrt2, so A^{-1/2} = 1/2 [[1 + 3^-1/2, 3^-1/2 - 1], [3^-1/2 - 1, 1 + 3^-1/2]]
    a = np.array([[2.0, 1.0], [1.0, 2.0]])
    r3 = 3.0 ** -0.5
    ref = 0.5 * np.array([[1 + r3, r3 - 1], [r3 - 1, 1 + r3]])
    assert np.max(np.abs(it.eig_root(a, 2) - ref)) < 4 * U
    res = it.solve(a, 2, 1e-14)
    assert res.status == it.OK
    assert np.max(np.abs(res.c - ref)) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("kappa", [1e2, 1e4])
def test_solve_reaches_definition(p, kappa):
    a, lam, q = _spd(96, kappa, 11)
    res = it.solve(a, p, 1e-10)
    assert res.status == it.OK
    ref = (q * lam ** (-1.0 / p)) @ q.T         # the definition with the known spectrum
    assert it.rel_fro(res.c, ref) < 1e-11
    assert res.residual_true < 1e-10


def test_p1_is_the_inverse():
    a, _, _ = _spd(80, 1e3, 5)
    inv = np.linalg.inv(a)
    for ev in ("coupled", "newton_schulz"):
        res = it.solve(a, 1, 1e-11, evaluation=ev)
        assert res.status == it.OK, ev
        assert it.rel_fro(res.c, inv) < 1e3 * 1e3 * U


@pytest.mark.parametrize("p", [1, 2, 3])
def test_diagonal_dense_equals_scalar_recursion_bitwise(p):
    lam = np.array([0.9, 0.013, 0.27, 1.0, 0.5, 0.0031])
    a = np.diag(lam)
    res = it.solve(a, p, 1e-13)
    assert res.status == it.OK
    # the coupled step on each diagonal entry, written out for scalars
    s = float(np.max(lam)) ** 2
    c = np.full_like(lam, s ** (-1.0 / (2 * p)))
    m = c.copy()
    for _ in range(p - 1):
        m = m * c
    m = m * lam
    for _ in range(res.iters):
        r = 1.0 - m
        nn = 1.0 + r / p
        c = c * nn
        for _ in range(p):
            m = nn * m
    assert np.array_equal(np.diag(res.c), c)
    assert np.count_nonzero(res.c - np.diag(np.diag(res.c))) == 0
    assert np.max(np.abs(c - lam ** (-1.0 / p)) / lam ** (-1.0 / p)) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 4])
def test_scaled_identity(p):
    a = 0.37 * np.eye(7)
    res = it.solve(a, p, 1e-14)
    assert res.status == it.OK
    assert np.max(np.abs(res.c - 0.37 ** (-1.0 / p) * np.eye(7))) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_dense_count_equals_spectral_count(p):
    for kappa, seed in ((1e2, 1), (1e3, 2)):
        a, lam, _ = _spd(128, kappa, seed)
        sigma = math.sqrt(it.norm_1(a) * it.norm_inf(a))
        res = it.solve(a, p, 1e-10)
        k, _ = it.spectral_count(lam, p, it.spectral_start(lam, p, "identity", sigma), 1e-10)
        assert res.status == it.OK and res.iters == k


def test_paper_start_spectrum_and_count():
    a, lam, _ = _spd(64, 1e2, 4)
    sigma = math.sqrt(it.norm_1(a) * it.norm_inf(a))
    c0 = it.start_paper(a, 1)
    # spectral_start("paper") must be the spectrum of eq. (3)'s C_0
    assert np.allclose(np.sort(np.linalg.eigvalsh(c0)),
                       np.sort(it.spectral_start(lam, 1, "paper", sigma)), rtol=0, atol=1e-15)
    res = it.solve(a, 1, 1e-10, init="paper", max_iter=200)
    k, _ = it.spectral_count(lam, 1, it.spectral_start(lam, 1, "paper", sigma), 1e-10)
    assert res.status == it.OK and res.iters == k


@pytest.mark.parametrize("p", [1, 2, 3])
def test_residual_strictly_decreases_then_quadratic(p):
    a, _, _ = _spd(128, 1e3, 9)
    res = it.solve(a, p, 1e-11)
    rho = np.array(res.rho)
    floor = 1e-12
    live = rho[rho > floor]
    assert np.all(np.diff(live) < 0)
    # g(r) = (p+1)/(2p) r^2 + O(r^3) per eigenvalue, so rho' <= ~(p+1)/(2p) rho^2
    for r0, r1 in zip(rho[:-1], rho[1:]):
        if 1e-5 < r0 < 0.05:
            assert r1 <= 1.2 * (p + 1) / (2 * p) * r0 * r0


def test_residual_map_closed_forms():
    r = np.linspace(-0.9, 0.9, 37)
    assert np.allclose(it.residual_map(r, 1), r * r, atol=1e-15)
    assert np.allclose(it.residual_map(r, 2), r * r * (3 + r) / 4, atol=1e-15)
    # 0 <= g(r) < |r| on (-1, 1) \ {0}
    for p in (1, 2, 3, 4):
        g = it.residual_map(r[r != 0], p)
        assert np.all(g >= 0) and np.all(g < np.abs(r[r != 0]))


def test_step_contraction_below_one_half():
    # p = 1: 1 - m(2 - m) = e^2, so the ratio is |e| and peaks at 1/2.
    # p = 2: 1 - m((3 - m)/2)^2 = e^2 (3 + e)/4 with m = 1 - e, peaking at
    # e = 1/2 with 7/16. Every p keeps |e| <= 1/2 to at most half of it, which
    # is what lets the floor rule count only below FLOOR_ZONE.
    assert it.step_contraction(1) == pytest.approx(0.5, abs=1e-12)
    assert it.step_contraction(2) == pytest.approx(7.0 / 16.0, abs=1e-12)
    for p in range(1, 9):
        assert it.step_contraction(p) <= 0.5 + 1e-12
    assert it.FLOOR_ZONE == 0.5
    # Above 1/2 a step can keep most of the error: e = 0.99 with p = 1 keeps 99%.
    assert it.step_contraction(1, emax=0.99) > 0.98


@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_tiny_orders_converge_through_the_slow_phase(n, p):
    # With kappa = 1e3 and n <= 3 the smallest eigenvalue alone sets the
    # residual through its slow phase, which stays above 1/2 for several steps
    # without halving; the run must still reach the tolerance.
    for seed in range(4):
        a, _, _ = _spd(n, 1e3, seed)
        res = it.solve(a, p, 1e-10)
        assert res.status == it.OK
        # residual r < 1e-10 gives C = A^{-1/p}(I - r)^{1/p}: error below r/p
        assert it.rel_fro(res.c, it.eig_root(a, p)) < 1e-10


def test_floor_rule_over_the_whole_range_misfires():
    # Counting stagnation anywhere below 1 ends this run in its slow phase.
    a, _, _ = _spd(2, 1e3, 0)
    saved = it.FLOOR_ZONE
    try:
        it.FLOOR_ZONE = 1.0
        res = it.solve(a, 2, 1e-10)
    finally:
        it.FLOOR_ZONE = saved
    assert res.status == it.EFLOOR and res.residual_true > 0.1


@pytest.mark.parametrize("p", [2, 3])
def test_invariants_symmetric_and_commuting(p):
    a, _, _ = _spd(128, 1e3, 12)
    res = it.solve(a, p, 1e-10)
    assert np.array_equal(res.c, res.c.T)
    assert it.commutator(res.c, a) < 1e-13


def test_literal_order_is_unstable():
    # Right-multiplied order of eq. (1) at kappa = 100 never reaches a small residual.
    a, _, _ = _spd(256, 1e2, 0)
    res = it.solve(a, 2, 1e-10, init="paper", evaluation="literal", max_iter=200)
    assert res.status != it.OK
    assert min(res.rho) > 1e-8


def test_paper_start_coupled_floor_near_u_kappa_p_plus_1():
    kappa, p = 1e2, 2
    a, _, _ = _spd(256, kappa, 0)
    res = it.solve(a, p, 1e-14, init="paper", max_iter=200)
    assert res.status == it.EFLOOR
    pred = U * kappa ** (p + 1)
    assert pred / 5 < res.residual_true < 5 * pred


def test_paper_start_violates_eq2_for_small_spectrum():
    # eq. (3) with A = 0.1 I and p = 2 gives C_0^p A = 10 I: ||I - C_0^p A||_2 = 9.
    a = 0.1 * np.eye(5)
    c0 = it.start_paper(a, 2)
    assert np.allclose(c0 @ c0 @ a, 10.0 * np.eye(5))
    res = it.solve(a, 2, 1e-10, init="paper")
    assert res.status == it.EDIVERGED


def test_newton_schulz_self_corrects_perturbation():
    # p = 1 Newton-Schulz order: a non-commuting perturbation of the start is removed.
    a, _, _ = _spd(64, 1e2, 6)
    inv = np.linalg.inv(a)
    rng = np.random.default_rng(0)
    e = rng.standard_normal(a.shape) * 1e-3 * np.linalg.norm(inv) / 64
    start = inv + 0.5 * (e + e.T)
    res = it.solve(a, 1, 1e-11, init=start, evaluation="newton_schulz")
    assert res.status == it.OK and it.rel_fro(res.c, inv) < 1e-11


def test_householder_root_is_the_definition():
    # the O(n^2 k) construction equals eigh's root and inverts A^p
    a, lam = w.householder_spd(300, 1e3, seed=4, nrefl=16)
    assert np.allclose(np.sort(np.linalg.eigvalsh(a)), np.sort(lam), atol=1e-14)
    lam2, v, t = w.householder_factors(300, 1e3, 4, nrefl=16)
    for p in (1, 2, 3):
        x = w.householder_congruence(v, t, lam2 ** (-1.0 / p))
        assert it.rel_fro(x, it.eig_root(a, p)) < 1e-12
        assert np.linalg.norm(np.eye(300) - np.linalg.matrix_power(x, p) @ a) < 1e-10
    a64, _ = w.householder_spd(256, 1e2, seed=9)
    assert it.rel_fro(it.householder_root(256, 1e2, 9, 2), it.eig_root(a64, 2)) < 1e-12


def test_scaled_newton_schulz_step_identity():
    # A Newton-Schulz step on mu C (residual (1 - mu) I + mu R, R = I - A C)
    # equals mu (2 - mu) C + mu^2 C R: the coefficients the p = 1 bulk phase's
    # scaled steps put into the update's epilogue. On the spectrum it is
    # m -> g(mu m), g(m) = m (2 - m), the coupled map for p = 1.
    a, lam, q = _spd(40, 1e3, 21)
    c = it.eig_root(a, 1) @ (np.eye(40) + 0.1 * a / lam.max())   # a polynomial in A
    r = np.eye(40) - a @ c
    for mu in (1.0, 1.3, 1.7):
        cs = mu * c
        direct = cs + cs @ (np.eye(40) - a @ cs)
        formula = mu * (2.0 - mu) * c + mu * mu * (c @ r)
        assert np.max(np.abs(direct - formula)) <= 1e-12 * np.max(np.abs(direct))
        m = np.sort(np.linalg.eigvals(a @ c).real)
        m1 = np.sort(np.linalg.eigvals(a @ formula).real)
        assert np.allclose(m1, np.sort(it.residual_map(1.0 - mu * m, 1) * -1.0 + 1.0),
                           rtol=0, atol=1e-10)
