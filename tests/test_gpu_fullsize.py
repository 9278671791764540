"""Parity at the full sizes the bench runs: n = 16384 (p = 2, Householder
spectrum matrices) and the n = 4096 kernel matrix (p = 1, 2, 3), in the
bench's launch configuration (FP64, triangle products: the headline's
Lanczos-scale start with scaled steps, the squaring scale, and the default
scaled identity)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as w
from oracle import iteration as it
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "iteration_counts.json")))["counts"]


@pytest.fixture(scope="module")
def ipr():
    import paper_1703_02283_amd as m
    m.load()
    return m


@pytest.mark.parametrize("schedule", ["default", "power", "lanczos"])
@pytest.mark.parametrize("kappa", [1e4, 1e2])
def test_householder_16384_p2(ipr, kappa, schedule):
    # lanczos = the schedule the bench times (Lanczos-scale start, scaled
    # steps); power = the same steps from the certified squaring scale;
    # default = the plain iteration, whose count the oracle fixes
    import torch
    n, p = 16384, 2
    say("full size householder n", n, "kappa", kappa, "schedule", schedule)
    a, lam = w.householder_spd(n, kappa, seed=0)
    A = dev(a)
    del a
    kw = {"default": {}, "power": dict(scale_squarings=6, dynamic_scaling=1),
          "lanczos": dict(scale_lanczos=1, dynamic_scaling=1)}[schedule]
    headline = schedule != "default"
    C, res = ipr.ipr_solve(A, p, 1e-10, schedule=ipr.ipr_schedule_default(**kw))
    say("  status", res.status, "iters", res.iters_fp64, "residual", res.residual_true)
    c = host(C)
    del A, C
    torch.cuda.empty_cache()
    ref = it.householder_root(n, kappa, 0, p)
    err = it.rel_fro(c, ref)
    say("  rel err vs definition", err)
    g = GOLD[f"householder_n16384_kappa{kappa:g}_seed0"]["p2"]["identity"]
    assert res.status == ipr.IPR_OK, res.as_dict()
    assert res.residual_true < 1e-10
    assert err <= 1e-10
    if headline:
        # the oracle's power scale and its exact-arithmetic count of the
        # scaled iteration on the known spectrum (golden file)
        gs = GOLD[f"householder_n16384_kappa{kappa:g}_seed0"]["p2"]
        say("  scale", res.init_scale, "golden", gs["power_scale"]["scale"],
            "iterations golden", gs["scaled"])
        assert res.iters_fp64 < g       # fewer iterations than the plain iteration
        assert abs(res.iters_fp64 - gs["scaled"]) <= 1
        if schedule == "power":
            assert abs(res.init_scale - gs["power_scale"]["scale"]) <= 1e-9 * res.init_scale
            assert lam.max() <= res.init_scale < math.sqrt(res.norm1 * res.norminf)
        else:
            # 1.01 times a Ritz value: at most 1.01 lambda_max, and close to
            # it; the oracle's count from that start on the known spectrum
            s_ref = 1.01 * lam.max()
            assert 0.95 * s_ref <= res.init_scale <= s_ref * (1 + 1e-12)
            k_ref = it.scaled_spectral_count(lam, p, s_ref, 1e-10)[0]
            say("  oracle count from s = 1.01 lambda_max", k_ref)
            assert -1 <= res.iters_fp64 - k_ref <= 1
        assert lam.min() * (1 - 1e-12) <= res.lmin_est <= lam.max()
    else:
        assert abs(res.iters_fp64 - g) <= 1
    assert np.array_equal(c[:64, :], c[:, :64].T)


@pytest.fixture(scope="module")
def kernel4096():
    a = w.kernel_matrix(4096, seed=0)
    lam, v = np.linalg.eigh(a)
    return a, lam, v


@pytest.mark.parametrize("p", [1, 2, 3])
def test_kernel_matrix_4096(ipr, kernel4096, p):
    a, lam, v = kernel4096
    say("kernel matrix n 4096 p", p)
    C, res = ipr.ipr_solve(dev(a), p, 1e-10)
    c = host(C)
    ref = (v * lam ** (-1.0 / p)) @ v.T
    err = it.rel_fro(c, ref)
    say("  status", res.status, "iters", res.iters_fp64, "residual", res.residual_true, "err", err)
    g = GOLD["kernel_n4096_seed0"][f"p{p}"]["identity"]
    assert res.status == ipr.IPR_OK, res.as_dict()
    assert err <= 1e-10
    assert abs(res.iters_fp64 - g) <= 1
    # power-scale start and scaled steps: the oracle's scale and its
    # exact-arithmetic count of the scaled iteration (golden file)
    gs = GOLD["kernel_n4096_seed0"][f"p{p}"]
    C, res = ipr.ipr_solve(dev(a), p, 1e-10, schedule=ipr.ipr_schedule_default(
        scale_squarings=6, dynamic_scaling=1))
    err = it.rel_fro(host(C), ref)
    say("  scaled: status", res.status, "iters", res.iters_fp64, "golden", gs["scaled"], "err", err)
    assert res.status == ipr.IPR_OK, res.as_dict()
    assert err <= 1e-10
    assert abs(res.init_scale - gs["power_scale"]["scale"]) <= 1e-9 * res.init_scale
    assert -1 <= res.iters_fp64 - gs["scaled"] <= 2


def test_householder_16384_p2_int8_slice_products(ipr):
    """The headline schedule with every iteration product from int8 digit
    slices (10 digits, the default): the same root as the definition."""
    import torch
    n, p, kappa = 16384, 2, 1e4
    say("full size householder int8-slice products")
    a, lam = w.householder_spd(n, kappa, seed=0)
    A = dev(a)
    del a
    s = ipr.ipr_schedule_default(bulk_dtype=ipr.IPR_FP64_INT8_EMUL, scale_squarings=6,
                                 dynamic_scaling=1, timing=1)
    C, res = ipr.ipr_solve(A, p, 1e-10, schedule=s)
    say("  status", res.status, "iters", res.iters_fp64, "residual", res.residual_true)
    c = host(C)
    del A, C
    torch.cuda.empty_cache()
    err = it.rel_fro(c, it.householder_root(n, kappa, 0, p))
    say("  rel err vs definition", err)
    assert res.status == ipr.IPR_OK, res.as_dict()
    assert res.residual_true < 1e-10
    assert err <= 1e-10
    assert res.lp_gemm_launches >= res.iters_fp64 and res.gemm_launches <= 10
