"""GPU parity of the FP64 path (through the C ABI) against the oracle."""
import json
import math
import os

import numpy as np
import pytest

import workloads as w
from oracle import iteration as it
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
# Iterations the library's scaled steps may take beyond the oracle's (which
# chooses every scale factor from the exact spectrum).
SCALED_SLACK = 2
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
U = np.finfo(np.float64).eps / 2


@pytest.fixture(scope="module")
def ipr():
    import paper_1703_02283_amd as m
    m.load()
    return m


def _gemm_bound(L, R):
    # |L^T R - fl(L^T R)| <= n u |L|^T |R| (entrywise), with slack for FMA order
    n = L.shape[0]
    return 2 * n * U * (np.abs(L).T @ np.abs(R)) + 1e-300


@pytest.mark.parametrize("n", [1, 16, 64, 128, 200, 257, 384])
def test_gemm_full_matches_numpy(ipr, n):
    say("gemm full n", n)
    rng = np.random.default_rng(n)
    L = rng.standard_normal((n, n))
    R = rng.standard_normal((n, n))
    X = rng.standard_normal((n, n))
    D = host(ipr.ipr_gemm(dev(L), dev(R), dev(X), alpha=0.5, beta=-2.0, gamma=3.0))
    ref = 0.5 * (L.T @ R) - 2.0 * X + 3.0 * np.eye(n)
    assert np.all(np.abs(D - ref) <= 0.5 * _gemm_bound(L, R) + 4 * U * (np.abs(ref) + 1))


@pytest.mark.parametrize("n", [64, 130, 256, 385])
def test_gemm_triangle_mirrors_upper(ipr, n):
    say("gemm triangle n", n)
    rng = np.random.default_rng(n + 1)
    S = rng.standard_normal((n, n))
    S = S + S.T
    T = rng.standard_normal((n, n))
    T = T @ T.T / n
    D = host(ipr.ipr_gemm(dev(S), dev(T), None, triangle=True))
    ref = S @ T                        # not symmetric: only its upper triangle is compared
    up = np.triu_indices(n)
    assert np.array_equal(D, D.T)
    assert np.all(np.abs(D[up] - ref[up]) <= _gemm_bound(S, T)[up])


def test_norms(ipr):
    a = w.kernel_matrix(300, seed=2)
    a[3, 7] = a[7, 3] = -5.0
    n1, ni = ipr.ipr_norms(dev(a))
    assert abs(n1 - it.norm_1(a)) <= 1e-14 * n1
    assert abs(ni - it.norm_inf(a)) <= 1e-14 * ni


def _solve(ipr, a, p, tol, **sched):
    s = ipr.ipr_schedule_default(**sched)
    C, res = ipr.ipr_solve(dev(a), p, tol, schedule=s)
    return host(C), res


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("n,tri", [(96, 1), (257, 1), (300, 0), (130, 0)])
def test_solve_matches_oracle(ipr, p, n, tri):
    say("solve p", p, "n", n, "tri", tri)
    a, lam, q = w.spd_log_spectrum(n, 1e3, seed=100 + n + p)
    c, res = _solve(ipr, a, p, 1e-10, triangle=tri)
    ref = it.solve(a, p, 1e-10)
    assert res.status == ipr.IPR_OK, res.as_dict()
    assert it.rel_fro(c, ref.c) <= 1e-10
    assert it.rel_fro(c, it.eig_root(a, p)) <= 1e-10
    assert abs(res.iters_fp64 - ref.iters) <= 1
    assert res.residual_true < 1e-10
    assert np.array_equal(c, c.T)        # exactly symmetric in both modes
    assert abs(res.norm1 - it.norm_1(a)) <= 1e-13 * res.norm1


def test_cfg1_spd256_p2_golden_count(ipr):
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "iteration_counts.json")))
    g = gold["counts"]["spd_n256_logU[1e-2,1]_seed0"]
    a, lam, q = w.spd_log_spectrum(256, lam_range=(1e-2, 1.0), seed=0)
    c, res = _solve(ipr, a, 2, 1e-12)
    ref = it.solve(a, 2, 1e-12)
    assert res.status == ipr.IPR_OK
    assert abs(res.iters_fp64 - g["p2"]["identity"]) <= 1
    assert it.rel_fro(c, ref.c) <= 1e-10


@pytest.mark.parametrize("p", [1, 2, 3])
def test_literal_order_matches_oracle(ipr, p):
    # eq. (1) as printed, C_{k+1} = ((p+1) C_k - C_k (C_k^p A)) / p without
    # symmetrisation: at kappa = 10 it converges with the oracle's count; at
    # kappa = 1e3 rounding errors that do not commute with A grow and neither
    # the oracle nor the GPU reaches the root (the reason for the coupled order)
    say("literal p", p)
    a, _, _ = w.spd_log_spectrum(96, 10.0, seed=50 + p)
    ref = it.solve(a, p, 1e-10, evaluation="literal")
    c, r = _solve(ipr, a, p, 1e-10, evaluation=ipr.IPR_EVAL_LITERAL)
    assert ref.status == it.OK and r.status == ipr.IPR_OK, r.as_dict()
    assert abs(r.iters_fp64 - ref.iters) <= 1
    assert r.residual_true < 1e-10
    assert r.gemms == (p + 1) * r.iters_fp64 + p
    assert it.rel_fro(c, ref.c) <= 1e-10 and it.rel_fro(c, it.eig_root(a, p)) <= 1e-10
    a, _, _ = w.spd_log_spectrum(96, 1e3, seed=50 + p)
    ref = it.solve(a, p, 1e-10, evaluation="literal")
    _, r = _solve(ipr, a, p, 1e-10, evaluation=ipr.IPR_EVAL_LITERAL)
    assert ref.status != it.OK and r.status in (ipr.IPR_EDIVERGED, ipr.IPR_EFLOOR)


def test_newton_schulz_order(ipr):
    a, _, _ = w.spd_log_spectrum(200, 1e3, seed=61)
    ref = it.solve(a, 1, 1e-10, evaluation="newton_schulz")
    c, r = _solve(ipr, a, 1, 1e-10, evaluation=ipr.IPR_EVAL_NEWTON_SCHULZ)
    assert r.status == ipr.IPR_OK and ref.status == it.OK
    assert abs(r.iters_fp64 - ref.iters) <= 1
    assert r.residual_true < 1e-10
    assert it.rel_fro(c, np.linalg.inv(a)) <= 1e-10
    assert np.array_equal(c, c.T)
    with pytest.raises(ipr.IprError) as ei:
        _solve(ipr, a, 2, 1e-10, evaluation=ipr.IPR_EVAL_NEWTON_SCHULZ)
    assert ei.value.code == ipr.IPR_EARG
    with pytest.raises(ipr.IprError) as ei:
        _solve(ipr, a, 1, 1e-10, evaluation=ipr.IPR_EVAL_LITERAL, bulk_dtype=ipr.IPR_BF16)
    assert ei.value.code == ipr.IPR_EARG


def _solve_from(ipr, a, c0, p, tol, **sched):
    s = ipr.ipr_schedule_default(init=ipr.IPR_INIT_USER, **sched)
    C, res = ipr.ipr_solve(dev(a), p, tol, schedule=s, out=dev(c0))
    return host(C), res


@pytest.mark.parametrize("p", [1, 2, 3])
def test_user_start(ipr, p):
    n = 160
    a, lam, q = w.spd_log_spectrum(n, 1e3, seed=80 + p)
    # the scaled identity given as C_0: the default start's iterates
    c0 = it.start_identity(a, p)
    c, r = _solve_from(ipr, a, c0, p, 1e-10)
    _, r0 = _solve(ipr, a, p, 1e-10)
    assert r.status == ipr.IPR_OK and r.fallback_used == 0
    assert abs(r.iters_fp64 - r0.iters_fp64) <= 1
    assert it.rel_fro(c, it.eig_root(a, p)) <= 1e-10
    # a polynomial in A given as C_0: the POLY start's iterates. (A C_0 that
    # is not a function of A to rounding, e.g. an earlier iterate, stalls in
    # the coupled order: M_0 = C_0^p A then carries the non-commuting error.)
    poly = (0.7, 0.3, 0.0)   # q(x)^p x <= 1 on (0, 1]
    c0 = it.start_poly(a, p, poly)
    c, r = _solve_from(ipr, a, c0, p, 1e-10)
    cp, rp = _solve(ipr, a, p, 1e-10, init=ipr.IPR_INIT_POLY, poly=poly)
    assert r.status == ipr.IPR_OK and rp.status == ipr.IPR_OK and r.fallback_used == 0
    assert abs(r.iters_fp64 - rp.iters_fp64) <= 1
    # the Lanczos estimate of the top of the spectrum of C_0^p A (below 1 here)
    assert 0.0 < r.init_bound <= 1.0 + 1e-9 and r.init_scale == 0.0
    assert it.rel_fro(c, it.eig_root(a, p)) <= 1e-10
    # a start outside eq. (2): the scaled identity instead, or an error
    c0 = 10.0 * np.eye(n)
    c, r = _solve_from(ipr, a, c0, p, 1e-10)
    assert r.status == ipr.IPR_OK and r.fallback_used == 1
    assert r.iters_fp64 == r0.iters_fp64
    with pytest.raises(ipr.IprError) as ei:
        _solve_from(ipr, a, c0, p, 1e-10, guard_fallback=0)
    assert ei.value.code == ipr.IPR_EGUARD


def test_user_start_newton_schulz_self_corrects(ipr):
    # p = 1 in Newton-Schulz order from an inverse with a perturbation that
    # does not commute with A: the error squares every step
    n = 200
    a, _, _ = w.spd_log_spectrum(n, 1e3, seed=91)
    rng = np.random.default_rng(5)
    e = rng.standard_normal((n, n))
    e = (e + e.T) / 2
    ainv = np.linalg.inv(a)
    c0 = ainv + 1e-4 * ainv @ e @ ainv / np.linalg.norm(e, 2)   # ||I - A C_0||_F ~ 0.2
    c0 = 0.5 * (c0 + c0.T)
    ref = it.solve(a, 1, 1e-10, init=c0, evaluation="newton_schulz")
    c, r = _solve_from(ipr, a, c0, 1, 1e-10, evaluation=ipr.IPR_EVAL_NEWTON_SCHULZ)
    assert r.status == ipr.IPR_OK and r.fallback_used == 0 and ref.status == it.OK
    assert 0.1 < r.init_bound - 1.0 < 0.5
    assert abs(r.iters_fp64 - ref.iters) <= 1 and r.iters_fp64 <= 4
    assert it.rel_fro(c, ainv) <= 1e-10


@pytest.mark.parametrize("p,kappa,tol", [(1, 10.0, 1e-8), (2, 100.0, 1e-10),
                                         (3, 10.0, 1e-10), (2, 1e4, 1e-10), (4, 1e3, 1e-10)])
def test_last_step_without_m_update(ipr, p, kappa, tol):
    # Once (p + 1)/(2p) rho_k^2 bounds the next residual below tol, the last
    # step forms C only and the check of the true residual replaces the M
    # update: (p + 1) products per iteration in all instead of p more (for
    # p = 4, N^4 and C^4 by squaring: 4 per iteration). The oracle's residual
    # history shows the bound holds, with a wide margin.
    say("last step p", p, "kappa", kappa, "tol", tol)
    a, lam, _ = w.spd_log_spectrum(256, kappa, seed=90 + p)
    ref = it.solve(a, p, tol)
    assert (p + 1) / (2 * p) * ref.rho[-2] ** 2 < 0.2 * tol
    c, r = _solve(ipr, a, p, tol)
    assert r.status == ipr.IPR_OK and r.residual_true < tol
    assert r.iters_fp64 == ref.iters
    assert r.gemms == (4 if p == 4 else p + 1) * r.iters_fp64
    assert it.rel_fro(c, ref.c) <= 1e-10
    assert np.array_equal(c, c.T)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_power_scale_start(ipr, p):
    # scaled identity with the repeated-squaring bound: the same scale as the
    # oracle's power_scale, a certified bound on lambda_max, the oracle's
    # iteration count from that start, and never more iterations than sigma
    say("power scale p", p)
    n = 300
    a, lam, _ = w.spd_log_spectrum(n, 1e4, seed=40 + p)
    s_ref, k_ref = it.power_scale(a, p, 6)
    c0, r0 = _solve(ipr, a, p, 1e-10)
    c, r = _solve(ipr, a, p, 1e-10, scale_squarings=6)
    assert r.status == ipr.IPR_OK and r0.status == ipr.IPR_OK
    assert abs(r.init_scale - s_ref) <= 1e-9 * s_ref and k_ref >= 1
    assert lam.max() <= r.init_scale < np.sqrt(r.norm1 * r.norminf)
    ref = it.solve(a, p, 1e-10, init=r.init_scale ** (-1.0 / p) * np.eye(n))
    assert ref.status == it.OK and abs(r.iters_fp64 - ref.iters) <= 1
    assert r.iters_fp64 <= r0.iters_fp64
    assert it.rel_fro(c, it.eig_root(a, p)) <= 1e-10


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("squarings", [0, 6])
def test_dynamic_scaling(ipr, p, squarings):
    # scaled steps from a Lanczos estimate of lambda_min: a Ritz value in the
    # spectrum, fewer iterations than the plain iteration from the same
    # start, the same root, and the count of the oracle's scaled iteration,
    # which takes its own scale (power_scale) and chooses every factor from
    # the exact spectrum. The library knows less (the lower end is an
    # estimate from above, the top is held at its certified bound), so it may
    # take more iterations: at most SCALED_SLACK more.
    say("dynamic scaling p", p, "squarings", squarings)
    n = 300
    a, lam, _ = w.spd_log_spectrum(n, 1e4, seed=70 + p)
    c0, r0 = _solve(ipr, a, p, 1e-10, scale_squarings=squarings)
    c, r = _solve(ipr, a, p, 1e-10, scale_squarings=squarings, dynamic_scaling=1)
    assert r.status == ipr.IPR_OK and r0.status == ipr.IPR_OK
    assert lam.min() - 1e-12 * lam.max() <= r.lmin_est <= lam.max() * (1 + 1e-12)
    assert r.iters_fp64 < r0.iters_fp64
    assert it.rel_fro(c, it.eig_root(a, p)) <= 1e-10
    if r.reest_iter > 0:   # the lower end estimated again on M_k
        assert 0.0 < r.lmin_reest <= 1.0 + 1e-12
    s_ref, _ = it.power_scale(a, p, squarings, scaled_steps=True)
    assert abs(r.init_scale - s_ref) <= 1e-9 * s_ref
    ref = it.solve(a, p, 1e-10, scaled=s_ref)
    say("  iterations", r.iters_fp64, "oracle", ref.iters)
    assert ref.status == it.OK and -1 <= r.iters_fp64 - ref.iters <= SCALED_SLACK
    # A = c I: Lanczos stops after one step at c, and nothing is scaled
    C, r = ipr.ipr_solve(dev(2.5 * np.eye(64)), p, 1e-10,
                         schedule=ipr.ipr_schedule_default(dynamic_scaling=1))
    assert r.status == ipr.IPR_OK and abs(r.lmin_est - 2.5) < 1e-12
    assert np.allclose(host(C), 2.5 ** (-1.0 / p) * np.eye(64), rtol=1e-13, atol=0)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("dyn", [0, 1])
def test_lanczos_scale(ipr, p, dyn):
    # the scale from the largest Ritz value of the Lanczos run, times 1.01: at
    # most 1.01 lambda_max (a Ritz value lies inside the spectrum) and close to
    # it; the same root; the oracle's count from the start s = 1.01 lambda_max
    # (its own eigenvalues, nothing taken from the library)
    say("lanczos scale p", p, "scaled steps", dyn)
    n = 300
    a, lam, _ = w.spd_log_spectrum(n, 1e4, seed=90 + p)
    c, r = _solve(ipr, a, p, 1e-10, scale_lanczos=1, dynamic_scaling=dyn)
    assert r.status == ipr.IPR_OK and r.fallback_used == 0
    s_ref = 1.01 * lam.max()
    assert 0.95 * s_ref <= r.init_scale <= s_ref * (1 + 1e-12)
    assert it.rel_fro(c, it.eig_root(a, p)) <= 1e-10
    if dyn:
        ref = it.solve(a, p, 1e-10, scaled=s_ref)
        assert ref.status == it.OK and -1 <= r.iters_fp64 - ref.iters <= SCALED_SLACK
    else:
        ref = it.solve(a, p, 1e-10, init=s_ref ** (-1.0 / p) * np.eye(n))
        assert ref.status == it.OK and abs(r.iters_fp64 - ref.iters) <= 1
    # below order 32 there is no Lanczos run: the norm bound of eq. (3)
    a, lam, _ = w.spd_log_spectrum(24, 1e3, seed=5)
    c, r = _solve(ipr, a, p, 1e-10, scale_lanczos=1, dynamic_scaling=dyn)
    assert r.status == ipr.IPR_OK
    assert r.init_scale == pytest.approx(np.sqrt(r.norm1 * r.norminf), rel=1e-15)


def test_paper_eq3_start(ipr):
    # p = 1 from eq. (3) converges (Newton-Schulz); counts agree with the oracle
    a, _, _ = w.spd_log_spectrum(128, 1e2, seed=7)
    c, res = _solve(ipr, a, 1, 1e-10, init=ipr.IPR_INIT_PAPER_EQ3, max_iter=200)
    ref = it.solve(a, 1, 1e-10, init="paper", max_iter=200)
    assert res.status == ipr.IPR_OK and ref.status == it.OK
    assert abs(res.iters_fp64 - ref.iters) <= 1
    assert it.rel_fro(c, np.linalg.inv(a)) < 1e-11
    # p = 2 from eq. (3) floors above 1e-12 at kappa ~ 1e2 (as the oracle does)
    a, _, _ = w.spd_log_spectrum(256, lam_range=(1e-2, 1.0), seed=0)
    c, res = _solve(ipr, a, 2, 1e-12, init=ipr.IPR_INIT_PAPER_EQ3, max_iter=200)
    ref = it.solve(a, 2, 1e-12, init="paper", max_iter=200)
    assert ref.status == it.EFLOOR and res.status in (ipr.IPR_EFLOOR, ipr.IPR_EMAXITER)
    assert it.rel_fro(c, it.eig_root(a, 2)) < 1e-8


def test_guard_falls_back_for_eq3_small_spectrum(ipr):
    a = 0.1 * np.eye(40)
    c, res = _solve(ipr, a, 2, 1e-12, init=ipr.IPR_INIT_PAPER_EQ3)
    assert res.fallback_used == 1 and res.status == ipr.IPR_OK
    assert np.max(np.abs(c - 0.1 ** -0.5 * np.eye(40))) < 1e-12
    with pytest.raises(ipr.IprError):
        _solve(ipr, a, 2, 1e-12, init=ipr.IPR_INIT_PAPER_EQ3, guard_fallback=0)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_poly_start(ipr, p):
    a, _, _ = w.spd_log_spectrum(200, 1e3, seed=21)
    b = (1.2, -0.3, 0.05)
    c, res = _solve(ipr, a, p, 1e-10, init=ipr.IPR_INIT_POLY, poly=b)
    ref = it.solve(a, p, 1e-10, init="poly", poly=b)
    assert res.status == ipr.IPR_OK and res.fallback_used == 0
    assert abs(res.iters_fp64 - ref.iters) <= 1
    assert it.rel_fro(c, ref.c) <= 1e-10


def test_degenerate_inputs(ipr):
    c, res = _solve(ipr, np.array([[4.0]]), 2, 1e-14)
    assert res.status == ipr.IPR_OK and abs(c[0, 0] - 0.5) < 1e-15
    lam = np.array([0.9, 0.013, 0.27, 1.0, 0.5, 0.0031])
    c, res = _solve(ipr, np.diag(lam), 3, 1e-13)
    assert res.status == ipr.IPR_OK
    assert np.max(np.abs(np.diag(c) - lam ** (-1 / 3)) / lam ** (-1 / 3)) < 1e-13
    assert np.count_nonzero(c - np.diag(np.diag(c))) == 0
    c, res = _solve(ipr, 0.37 * np.eye(33), 4, 1e-14)
    assert res.status == ipr.IPR_OK and np.max(np.abs(c - 0.37 ** -0.25 * np.eye(33))) < 1e-14


def test_argument_errors(ipr):
    import torch
    a = dev(np.eye(8))
    with pytest.raises(ipr.IprError):
        ipr.ipr_solve(a, 2, 0.0)
    with pytest.raises(ipr.IprError):
        ipr.ipr_solve(a, 0, 1e-10)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(ipr.IprError):
        ipr.ipr_solve(a, 2, 1e-10, workspace=small)
    with pytest.raises(ipr.IprError) as ei:   # the output may not overwrite the input
        ipr.ipr_solve(a, 2, 1e-10, out=a)
    assert ei.value.code == ipr.IPR_EARG
    for bad in (dict(evaluation=3), dict(init=5)):
        with pytest.raises(ipr.IprError) as ei:
            ipr.ipr_solve(a, 2, 1e-10, schedule=ipr.ipr_schedule_default(**bad))
        assert ei.value.code == ipr.IPR_EARG


def test_maxiter_and_divergence_status(ipr):
    a, _, _ = w.spd_log_spectrum(64, 1e4, seed=3)
    c, res = _solve(ipr, a, 2, 1e-10, max_iter=3)
    assert res.status == ipr.IPR_EMAXITER and res.iters_fp64 == 3
    ind = np.diag(np.linspace(-1.0, 1.0, 32))      # indefinite: diverges, twice
    c, res = _solve(ipr, ind, 2, 1e-10)
    say("indefinite: status", res.status, "iters", res.iters_fp64, "fallback", res.fallback_used)
    assert res.status == ipr.IPR_EDIVERGED and res.fallback_used == 1
    # (after the restart from the scaled identity, which diverges again)
    ref = it.solve(ind, 2, 1e-10)
    assert ref.status == it.EDIVERGED and abs(res.iters_fp64 - 2 * ref.iters) <= 2
    # the literal order reports its first divergence (a diagnostic)
    c, res = _solve(ipr, ind, 2, 1e-10, evaluation=ipr.IPR_EVAL_LITERAL)
    assert res.status == ipr.IPR_EDIVERGED and res.fallback_used == 0


def test_repeat_runs_are_bitwise_identical(ipr):
    a, _, _ = w.spd_log_spectrum(320, 1e3, seed=5)
    c1, r1 = _solve(ipr, a, 2, 1e-10)
    c2, r2 = _solve(ipr, a, 2, 1e-10)
    assert np.array_equal(c1, c2) and r1.residual_proxy == r2.residual_proxy
