"""Pins of the oracle's rounding emulator, MLP reference, features and guard."""
import math

import numpy as np
import pytest
import torch

from oracle import features as ft
from oracle import guard, mlp, rounding


@pytest.mark.parametrize("fmt,dtype", [("bf16", torch.bfloat16), ("fp16", torch.float16),
                                       ("fp8_e4m3", torch.float8_e4m3fn)])
def test_round_to_format_matches_torch_casts(fmt, dtype):
    rng = np.random.default_rng(0)
    vmax = rounding.FORMATS[fmt][2]
    x = rng.standard_normal(20000).astype(np.float32) * np.float32(4.0) ** rng.integers(-8, 5, 20000)
    x = x[np.abs(x) < 0.9 * vmax].astype(np.float32)
    ref = torch.from_numpy(x).to(dtype).to(torch.float64).numpy()
    got = rounding.round_to_format(x.astype(np.float64), fmt)
    assert np.array_equal(got, ref)


def test_custom_10_bits_is_half_precision_in_range():
    rng = np.random.default_rng(1)
    x = rng.uniform(-1000, 1000, 5000)
    x = x[np.abs(x) > 2.0 ** -14]
    assert np.array_equal(rounding.round_custom(x, 10), rounding.round_to_format(x, "fp16"))


def test_round_half_to_even():
    # 1 + 2^-8 is halfway between two bf16 neighbours: ties go to the even one (1.0)
    assert rounding.round_to_format(np.array([1 + 2.0 ** -8]), "bf16")[0] == 1.0
    assert rounding.round_to_format(np.array([1 + 3 * 2.0 ** -8]), "bf16")[0] == 1 + 2.0 ** -6


def test_tile_scaling_roundtrip_and_exponents():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((300, 260)) * 1e-5
    x[:128, :128] *= 1e6
    codes, ex = rounding.quantize(x, "fp8_e4m3", 128)
    assert ex.shape == (3, 3)
    # largest magnitude of each tile lands in [2^7, 2^8) before rounding
    for bi in range(3):
        for bj in range(3):
            blk = codes[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128]
            assert 2 ** 7 <= np.max(np.abs(blk)) <= 2 ** 8
    back = rounding.dequantize(codes, ex, 128)
    rel = np.abs(back - x) / np.maximum(np.abs(x), 1e-300)
    big = np.abs(x) > 2.0 ** -6 * np.ldexp(1.0, np.repeat(np.repeat(ex, 128, 0), 128, 1)[:300, :260] + 7)
    assert np.all(rel[big] <= 2.0 ** -4)


def test_gelu_known_values():
    # GELU(x) = x Phi(x); Phi(1) = 0.8413447460685429 (standard normal table)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array([-1.0]))[0] + (1 - 0.8413447460685429)) < 1e-15
    h = 1e-6
    x = np.linspace(-3, 3, 13)
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, atol=1e-8)


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    nparam = mlp.n_params()
    assert nparam == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3
    theta = rng.standard_normal(nparam) * 0.2
    x = rng.standard_normal((7, 16))
    t = rng.standard_normal((7, 3))
    g, _ = mlp.backward(theta, x, t)
    idx = rng.choice(nparam, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(nparam); e[i] = h
        lp = mlp.loss(mlp.forward(theta + e, x)[0], t)
        lm = mlp.loss(mlp.forward(theta - e, x)[0], t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), i


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # bias-corrected first step: -lr * g / (|g| + eps)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_on_hand_matrix():
    a = np.array([[4.0, -1.0, 0.0], [-1.0, 3.0, 1.0], [0.0, 1.0, 2.0]])
    f = ft.features(a, 2)
    sigma = 5.0                       # ||A||_1 = ||A||_inf = 5
    b = a / sigma
    assert f.shape == (16,)
    assert f[0] == 0.6 and f[1] == 0.5            # order clipped up to 2^6 (training sizes)
    assert ft.features(np.eye(128), 1)[0] == 0.7
    assert ft.features(np.eye(2048), 1)[0] == 1.0   # and down to 2^10
    assert abs(f[2] - 9.0 / 5 / 3) < 1e-15                       # trace/sigma/n
    assert abs(f[3] - (16 + 9 + 4 + 4 * 1) / 25 / 3) < 1e-15      # ||B||_F^2 / n
    assert abs(f[7] - 0.4) < 1e-15 and abs(f[8] - 0.8) < 1e-15
    assert abs(f[10] - min(0.8 - 0.2, 0.6 - 0.4, 0.4 - 0.2)) < 1e-15
    assert abs(f[11] - (5 + 5 + 3) / 5 / 3) < 1e-15
    assert abs(f[12] - (1 + 2 + 1) / 9) < 1e-15
    assert abs(f[13] - 0.2) < 1e-15
    assert abs(f[15] - math.log10(5)) < 1e-15
    assert abs(f[14] - np.std([0.8, 0.6, 0.4]) / 0.6) < 1e-15


def test_guard_identity_and_paper_starts():
    # scaled identity: phi(x) = x on (0,1] -> accepted, sup 1
    ok, sup, qmin = guard.check((1.0, 0.0, 0.0), 2)
    assert ok and abs(sup - 1.0) < 1e-12
    # eq. (3) start is C_0 = A/sigma^2 -> q(x) = sigma^{1/p - 1} x, phi = sigma^{1-p} x^{p+1}
    for sigma, p, expect in ((0.1, 2, False), (3.0, 2, True), (0.5, 3, False), (1.0, 1, True)):
        b = (0.0, sigma ** (1.0 / p - 1.0), 0.0)
        ok, sup, _ = guard.check(b, p)
        assert ok == expect and abs(sup - sigma ** (1 - p)) < 1e-9
    # a start whose phi overshoots 2 is rejected
    assert not guard.check((2.0, 0.0, 0.0), 1)[0]
    assert not guard.check((1.0, -2.0, 0.0), 2)[0]


def test_power_scale_bounds_lambda_max_and_tightens():
    # A = c I and diagonal A: the norm bound sigma is already lambda_max, the
    # first squaring's bound (with its 1% margin) is above it, so s = sigma
    # and squaring stops after one product
    import workloads as w
    from oracle import iteration as it
    s, k = it.power_scale(3.0 * np.eye(5), 2, 6)
    assert k == 1 and s == 3.0
    lam = np.array([1e-3, 0.2, 0.5, 2.0])
    s, k = it.power_scale(np.diag(lam), 3, 6)
    assert k == 1 and s == 2.0
    # a matrix whose norm bound is loose: A = Q diag(lam) Q^T with a Haar Q
    # has sigma well above lambda_max = 1; each squaring brings the bound
    # closer, and stays >= lambda_max
    # a general SPD matrix: s >= lambda_max, never above sigma, and no worse
    # with more squarings allowed
    a, lam, _ = w.spd_log_spectrum(64, 1e3, seed=3)
    sig = np.sqrt(it.norm_1(a) * it.norm_inf(a))
    prev = sig
    for m in range(0, 5):
        s, k = it.power_scale(a, 2, m)
        assert lam.max() <= s <= prev + 1e-15 and k <= m
        prev = s


def test_scale_factor_closed_forms():
    # Where the cap does not bind, the best mu balances the two ends of the
    # spectrum, g(mu a) = g(mu b). For p = 1, g(m) = m (2 - m) is symmetric about
    # 1, so mu (a + b) = 2. For p = 2, g(m) = m (3 - m)^2 / 4 and the balance
    # a (3 - mu a)^2 = b (3 - mu b)^2 divided by (a - b) is the quadratic
    # mu^2 (a^2 + ab + b^2) - 6 mu (a + b) + 9 = 0, whose smaller root is
    # mu = 3 (a + b - sqrt(ab)) / (a^2 + ab + b^2).
    from oracle import iteration as it
    for a, b in ((0.3, 1.0), (0.2, 0.9), (0.45, 0.8)):
        assert abs(it.scaled_step_factor(np.array([a, 0.5 * (a + b), b]), 1)
                   - 2.0 / (a + b)) < 1e-7
        mu2 = 3.0 * (a + b - np.sqrt(a * b)) / (a * a + a * b + b * b)
        assert mu2 * b < it.mu_cap(2)
        assert abs(it.scaled_step_factor(np.array([a, b]), 2) - mu2) < 1e-7
    # a spectrum reaching far down: the lower end still rises at the cap
    for p in (1, 2, 3, 4):
        assert abs(it.scaled_step_factor(np.array([1e-4, 0.5]), p)
                   - it.mu_cap(p) / 0.5) < 1e-12
        # quadratic phase, and a spectrum whose top is already at the cap
        assert it.scaled_step_factor(np.array([0.6, 1.0]), p) == 1.0
        assert it.scaled_step_factor(np.array([0.01, it.mu_cap(p)]), p) == 1.0


def test_scale_factor_beats_every_other_scale_on_whole_spectra():
    # brute force over every eigenvalue (not only the ends): no scale in the
    # allowed range gives a larger smallest eigenvalue after the step
    from oracle import iteration as it
    rng = np.random.default_rng(5)
    for p in (1, 2, 3, 4):
        for _ in range(4):
            m = np.exp(rng.uniform(np.log(1e-5), 0.0, 200)) * rng.uniform(0.3, 1.0)
            mu = it.scaled_step_factor(m, p)
            assert 1.0 <= mu and mu * m.max() <= it.mu_cap(p) * (1 + 1e-15)
            got = np.min(it.step_map(mu * m, p))
            for t in np.linspace(1.0, it.mu_cap(p) / m.max(), 3001):
                assert np.min(it.step_map(t * m, p)) <= got * (1 + 1e-9)


def test_scaled_iteration_reaches_the_root_in_fewer_steps():
    # the dense scaled iteration: the exact-arithmetic count of the same
    # schedule (per eigenvalue), the root by definition, fewer iterations than
    # the plain iteration from the same start
    import workloads as w
    from oracle import iteration as it
    for p in (1, 2, 3):
        a, lam, _ = w.spd_log_spectrum(120, 1e4, seed=60 + p)
        for s in (np.sqrt(it.norm_1(a) * it.norm_inf(a)), it.power_scale(a, p, 6, True)[0]):
            plain = it.solve(a, p, 1e-10, init=s ** (-1.0 / p) * np.eye(120))
            r = it.solve(a, p, 1e-10, scaled=s)
            k, rho, mus = it.scaled_spectral_count(lam, p, s, 1e-10)
            assert r.status == it.OK and r.iters < plain.iters and r.iters == k
            assert all(mu >= 1.0 for mu in mus) and mus[0] > 1.0
            assert it.rel_fro(r.c, it.eig_root(a, p)) < 1e-11
            # the residual trajectory follows the exact one until the rounding floor
            for x, y in zip(r.rho, rho):
                if y > 1e-6:
                    assert abs(x - y) <= 1e-8 * y


def test_scaled_iteration_from_a_polynomial_start():
    # C_0 = s^{-1/p} q(A/s) with q(x) = b0 + b1 x: the dense count equals the
    # per-eigenvalue count, and the iteration reaches the root
    import workloads as w
    from oracle import iteration as it
    a, lam, _ = w.spd_log_spectrum(100, 1e3, seed=81)
    for p, b in ((1, (1.2, -0.4, 0.0)), (2, (1.1, -0.3, 0.05)), (3, (1.0, -0.2, 0.0))):
        s = it.power_scale(a, p, 6, True)[0]
        r = it.solve(a, p, 1e-10, init="poly", poly=b, scaled=s)
        k, _, _ = it.scaled_spectral_count(lam, p, s, 1e-10, poly=b)
        assert r.status == it.OK and r.iters == k
        assert it.rel_fro(r.c, it.eig_root(a, p)) < 1e-11


def test_scaled_iteration_on_diagonal_matrices_is_the_scalar_recursion():
    # diagonal A: every product is exact up to one rounding per entry, and the
    # scaled iteration's diagonal follows c <- mu^{1/p} c (p + 1 - mu c^p lam)/p
    from oracle import iteration as it
    lam = np.array([1e-3, 0.02, 0.3, 0.7, 1.0])
    p, s = 2, 1.0
    r = it.solve(np.diag(lam), p, 1e-12, scaled=s)
    k, _, mus = it.scaled_spectral_count(lam, p, s, 1e-12)
    assert r.status == it.OK and r.iters == k
    c = np.full_like(lam, s ** (-1.0 / p))
    for mu in mus[:k]:
        c = mu ** (1.0 / p) * c * (p + 1 - mu * c ** p * lam) / p
    assert np.allclose(np.diag(r.c), c, rtol=1e-14, atol=0)
    assert np.allclose(np.diag(r.c), lam ** (-1.0 / p), rtol=1e-12, atol=0)


def test_scaled_iteration_keeps_the_p1_floor():
    # p = 1 at kappa = 6e4: with the scaled top capped at 1 + 1/sqrt(2) the
    # scaled iteration reaches 1e-10 like the plain one (a cap of 1.98 left
    # it at ~1.9e-10)
    import workloads as w
    from oracle import iteration as it
    a, lam, _ = w.spd_log_spectrum(200, 6e4, seed=10)
    s, _ = it.power_scale(a, 1, 6)
    plain = it.solve(a, 1, 1e-10, init=s ** (-1.0) * np.eye(200))
    r = it.solve(a, 1, 1e-10, scaled=s)
    assert plain.status == it.OK and r.status == it.OK and r.iters < plain.iters
    assert r.residual_true < 2.0 * plain.residual_true