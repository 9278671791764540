"""GPU parity of the learned start's kernels (features, MLP forward,
backward and Adam, spectral labels) against the oracle, and the learned start
inside ipr_solve (guard, fallback, gain)."""
import numpy as np
import pytest

import workloads as w
from oracle import features as ft
from oracle import iteration as it
from oracle import mlp
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipr():
    import paper_1703_02283_amd as m
    m.load()
    return m


def test_features_match_oracle(ipr):
    import torch
    mats = [w.spd_log_spectrum(n, 1e3, seed=n)[0] for n in (2, 5, 64, 200)]
    mats.append(w.kernel_matrix(150, seed=1))
    ns = [a.shape[0] for a in mats]
    ps = [1, 2, 3, 4, 2]
    offs = np.cumsum([0] + [n * n for n in ns[:-1]]).tolist()
    buf = np.concatenate([a.ravel() for a in mats])
    f = ipr.ipr_features(dev(buf), offs, ns, ps).cpu().numpy()
    for i, (a, p) in enumerate(zip(mats, ps)):
        ref = ft.features(a, p)
        assert np.allclose(f[i], ref, rtol=2e-6, atol=2e-6), (i, f[i], ref)


def test_mlp_forward_matches_oracle(ipr):
    import torch
    rng = np.random.default_rng(0)
    theta = (rng.standard_normal(mlp.n_params()) * 0.3).astype(np.float32)
    x = rng.standard_normal((333, 16)).astype(np.float32)
    y = ipr.ipr_mlp_forward(torch.tensor(theta).cuda(), torch.tensor(x).cuda()).cpu().numpy()
    ref, _ = mlp.forward(theta.astype(np.float64), x.astype(np.float64))
    assert np.allclose(y, ref, rtol=1e-4, atol=1e-5)


def test_mlp_train_step_matches_oracle(ipr):
    import torch
    rng = np.random.default_rng(1)
    theta = (rng.standard_normal(mlp.n_params()) * 0.3).astype(np.float32)
    x = rng.standard_normal((300, 16)).astype(np.float32)
    t = rng.standard_normal((300, 3)).astype(np.float32)
    th = torch.tensor(theta).cuda()
    g = torch.zeros_like(th)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    loss = torch.zeros(1, device="cuda")
    ipr.ipr_mlp_train_step(th, g, m, v, torch.tensor(x).cuda(), torch.tensor(t).cuda(), 1,
                           1e-3, loss)
    gref, lref = mlp.backward(theta.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    gg = g.cpu().numpy()
    scale = np.abs(gref).max()
    assert np.max(np.abs(gg - gref)) <= 1e-4 * scale
    assert abs(loss.item() - lref) <= 1e-5 * lref
    tref, mref, vref = mlp.adam(theta.astype(np.float64), gg.astype(np.float64),
                                np.zeros_like(gref), np.zeros_like(gref), 1, lr=1e-3)
    assert np.allclose(th.cpu().numpy(), tref, rtol=1e-5, atol=1e-6)


def test_spectral_counts_match_oracle(ipr):
    import torch
    rng = np.random.default_rng(2)
    lams, ns, ps, scales = [], [], [], []
    for i in range(12):
        n = int(rng.integers(2, 400))
        p = int(rng.integers(1, 5))
        lam = w.log_spectrum(n, 10 ** rng.uniform(1, 5), rng)
        lams.append(lam)
        ns.append(n)
        ps.append(p)
        scales.append(float(lam.max() * rng.uniform(1.0, 4.0)))
    cands = np.array([[1.0, 0, 0], [1.2, 0, 0], [0.9, -0.3, 0], [1.1, -0.4, 0.1]])
    offs = np.cumsum([0] + ns[:-1]).tolist()
    lam_d = torch.tensor(np.concatenate(lams), dtype=torch.float64).cuda()
    got = ipr.ipr_spectral_counts(lam_d, offs, ns, ps, scales, cands, 1e-10, 300)
    for i in range(12):
        for c, b in enumerate(cands):
            c0 = it.spectral_start(lams[i], ps[i], "poly", scales[i], poly=b)
            k, rho = it.spectral_count(lams[i], ps[i], c0, 1e-10, 300)
            # both run eq. (1) per eigenvalue in FP64 with different (equivalent)
            # formulas; a count can differ only when the residual lands on tol
            near = any(abs(r / 1e-10 - 1) < 1e-3 for r in rho)
            assert got[i, c] == k or (near and abs(got[i, c] - k) <= 1), (i, c, got[i, c], k)
    per = ipr.ipr_spectral_counts(lam_d, offs, ns, ps, scales, np.tile(cands[1], (12, 1)),
                                  1e-10, 300, per_item=True)
    assert np.array_equal(per, got[:, 1])


def _weights():
    from paper_1703_02283_amd import train_start
    return train_start.load_weights()


def test_learned_start_guard_and_fallback(ipr):
    import torch
    a, _, _ = w.spd_log_spectrum(200, 1e3, seed=3)
    # b0 = e^3: beyond eq. (2) (sup q^p x = b0^p); the start is scaled back
    # inside the guard set, b0^p = 1.98, and no fallback is needed
    theta = np.zeros(mlp.n_params(), np.float32)
    theta[-3] = 3.0
    s = ipr.ipr_schedule_default(init=ipr.IPR_INIT_LEARNED, mlp_params=torch.tensor(theta).cuda())
    C, res = ipr.ipr_solve(dev(a), 2, 1e-10, schedule=s)
    assert res.fallback_used == 0 and res.status == ipr.IPR_OK
    assert abs(res.poly_used[0] ** 2 - 1.98) < 1e-12 and res.init_bound < 2.0
    assert it.rel_fro(host(C), it.eig_root(a, 2)) <= 1e-10
    # q(x) = 1 - 3x is negative on part of (0, 1]: no scaling repairs that,
    # so the solver falls back to the scaled identity
    theta[-3], theta[-2] = 0.0, -3.0
    s = ipr.ipr_schedule_default(init=ipr.IPR_INIT_LEARNED, mlp_params=torch.tensor(theta).cuda())
    C, res = ipr.ipr_solve(dev(a), 2, 1e-10, schedule=s)
    assert res.fallback_used == 1 and res.status == ipr.IPR_OK
    assert list(res.poly_used) == [1.0, 0.0, 0.0]
    assert it.rel_fro(host(C), it.eig_root(a, 2)) <= 1e-10
    # the same start with the fallback switched off is an error
    s = ipr.ipr_schedule_default(init=ipr.IPR_INIT_LEARNED, guard_fallback=0,
                                 mlp_params=torch.tensor(theta).cuda())
    with pytest.raises(ipr.IprError) as ei:
        ipr.ipr_solve(dev(a), 2, 1e-10, schedule=s)
    assert ei.value.code == ipr.IPR_EGUARD
    theta[-2] = 0.0
    # b0 = 1 in units of the certified bound: accepted, and the bound is >= lambda_max
    theta[-3] = 0.0
    s = ipr.ipr_schedule_default(init=ipr.IPR_INIT_LEARNED, mlp_params=torch.tensor(theta).cuda())
    C, res = ipr.ipr_solve(dev(a), 2, 1e-10, schedule=s)
    lmax = np.linalg.eigvalsh(a).max()
    assert res.fallback_used == 0 and res.status == ipr.IPR_OK
    assert lmax <= res.init_scale <= np.sqrt(res.norm1 * res.norminf)
    assert it.rel_fro(host(C), it.eig_root(a, 2)) <= 1e-10


@pytest.mark.skipif(_weights() is None, reason="no trained weights in the package")
@pytest.mark.parametrize("n", [200, 512, 1000])
def test_learned_start_uses_the_batched_features(ipr, n):
    # The single solve computes its features with one workgroup below n = 256
    # and with n / 16 workgroups from there on; either way the polynomial it
    # uses is the network's output on the features of ipr_features (pinned to
    # the oracle above), up to float rounding and the guard's common scale.
    import torch
    theta = torch.tensor(_weights()).cuda()
    a, _ = w.batch_matrix(n, 3e3, 11 + n)
    f = ipr.ipr_features(dev(a.ravel()), [0], [n], [2])
    assert np.allclose(f.cpu().numpy()[0], ft.features(a, 2), rtol=2e-6, atol=2e-6)
    y = ipr.ipr_mlp_forward(theta, f).cpu().numpy()[0].astype(np.float64)
    b = np.array([np.exp(y[0]), y[1], y[2]])
    if abs(b[1]) < 0.05 * b[0] and abs(b[2]) < 0.05 * b[0]:
        b[1] = b[2] = 0.0
    s = ipr.ipr_schedule_default(init=ipr.IPR_INIT_LEARNED, mlp_params=theta)
    C, r = ipr.ipr_solve(dev(a), 2, 1e-10, schedule=s)
    assert r.status == ipr.IPR_OK and r.fallback_used == 0
    used = np.array(list(r.poly_used))
    t = used[0] / b[0]
    assert 0.0 < t <= 1.0 + 1e-5
    assert np.allclose(used, t * b, rtol=1e-4, atol=1e-5 * b[0])
    assert it.rel_fro(host(C), it.eig_root(a, 2)) <= 1e-10


@pytest.mark.skipif(_weights() is None, reason="no trained weights in the package")
def test_learned_start_gains_on_heldout_sample(ipr):
    # every item counts, solved or not: where the learned start fails and the
    # identity succeeds, the solve would be repeated from the identity, so
    # the identity's products are added to the learned start's (items where
    # both fail, at condition numbers whose 1e-10 lies below the FP64 floor,
    # count their own products); device time of both starts is reported
    import torch
    from paper_1703_02283_amd import train_start as ts
    theta = torch.tensor(_weights()).cuda()
    items = ts.recipe(60, 3 * 10**6, n_range=(64, 400))
    tot_i = tot_l = 0
    ms_i = ms_l = 0.0
    fallbacks = fail_i = fail_l = 0
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for (n, p, kappa, seed, _) in items:
        a, lam = w.batch_matrix(n, kappa, seed)
        A = dev(a)
        s = ipr.ipr_schedule_default(init=ipr.IPR_INIT_LEARNED, mlp_params=theta)
        ev[0].record()
        _, ri = ipr.ipr_solve(A, p, 1e-10)
        ev[1].record()
        C, rl = ipr.ipr_solve(A, p, 1e-10, schedule=s)
        ev[2].record()
        torch.cuda.synchronize()
        ms_i += ev[0].elapsed_time(ev[1])
        ms_l += ev[1].elapsed_time(ev[2])
        tot_i += ri.gemms
        loss = rl.status != ipr.IPR_OK and ri.status == ipr.IPR_OK
        tot_l += rl.gemms + (ri.gemms if loss else 0)
        fail_i += ri.status != ipr.IPR_OK
        fail_l += rl.status != ipr.IPR_OK
        if rl.status == ipr.IPR_OK:
            assert it.rel_fro(host(C), it.eig_root(a, p)) <= 1e-10
        fallbacks += rl.fallback_used
    say("products identity", tot_i, "learned", tot_l, "fallbacks", fallbacks,
        "failed identity", fail_i, "learned", fail_l, "ms identity", ms_i, "learned", ms_l)
    assert tot_l < 0.97 * tot_i
    assert fail_l <= fail_i
    assert fallbacks <= len(items) // 10


@pytest.mark.skipif(_weights() is None, reason="no trained weights in the package")
@pytest.mark.parametrize("n,kappa,seed,p", [(300, 1e4, 5, 2), (500, 1e3, 6, 3), (400, 3e4, 7, 1)])
def test_learned_start_with_scaled_steps(ipr, n, kappa, seed, p):
    # The learned start combined with scaled steps. The oracle builds the
    # start on its own (its features and network on the stored weights, the
    # 5% rule, eq. (2)'s rescale, the certified bound from A^2 by numpy) and
    # runs the scaled iteration from the exact spectrum: the same root, the
    # library's polynomial proportional to the oracle's (the library folds
    # the first factor mu_0^{1/p} into it), and its count within -1..+2.
    import torch
    from oracle import guard, mlp
    th = _weights()
    a, lam = w.batch_matrix(n, kappa, seed)
    s = ipr.ipr_schedule_default(init=ipr.IPR_INIT_LEARNED, dynamic_scaling=1,
                                 mlp_params=torch.tensor(th).cuda())
    C, r = ipr.ipr_solve(dev(a), p, 1e-10, schedule=s)
    assert r.status == ipr.IPR_OK and r.fallback_used == 0, r.as_dict()
    assert it.rel_fro(host(C), it.eig_root(a, p)) <= 1e-10
    y = mlp.forward(th.astype(np.float64), ft.features(a, p)[None, :])[0][0]
    b = np.array([np.exp(y[0]), y[1], y[2]])
    if abs(b[1]) < 0.05 * b[0] and abs(b[2]) < 0.05 * b[0]:
        b[1] = b[2] = 0.0
    ok, sup, _ = guard.check(b, p)
    if sup >= 2.0:
        b = b * (1.98 / sup) ** (1.0 / p)
    a2 = a @ a
    sigma = np.sqrt(it.norm_1(a) * it.norm_inf(a))
    sc = min(sigma, np.sqrt(np.sqrt(it.norm_1(a2) * it.norm_inf(a2))) * (1 + 8 * n * 2.0 ** -52))
    assert abs(r.init_scale - sc) <= 1e-12 * sc
    used = np.array(list(r.poly_used))
    t = used[0] / b[0]
    assert np.allclose(used, t * b, rtol=1e-4, atol=1e-5 * used[0])
    ref = it.solve(a, p, 1e-10, init="poly", poly=tuple(b), scaled=sc)
    r0 = ipr.ipr_solve(dev(a), p, 1e-10, schedule=ipr.ipr_schedule_default(
        init=ipr.IPR_INIT_LEARNED, mlp_params=torch.tensor(th).cuda()))[1]
    say("learned + scaled: iterations", r.iters_fp64, "oracle", ref.iters,
        "learned unscaled", r0.iters_fp64, "poly", used)
    assert ref.status == it.OK and -1 <= r.iters_fp64 - ref.iters <= 2
    assert r.iters_fp64 < r0.iters_fp64
