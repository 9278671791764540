"""GPU parity of the FP64-accurate int8-slice product (ipr_gemm_emul)
against the oracle's error-free splitting: bit for bit, since both sides add
exact integer level sums in the same order."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle import slices
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipr():
    import paper_1703_02283_amd as m
    m.load()
    return m


def wide(rng, shape, lo=-3, hi=2):
    mag = 10.0 ** rng.uniform(lo, hi, size=shape)
    return np.where(rng.random(shape) < 0.5, -mag, mag)


@pytest.mark.parametrize("s", [1, 3, 9])
@pytest.mark.parametrize("n", [1, 100, 256, 300, 517])
def test_emul_product_is_bitwise_the_oracle(ipr, n, s):
    say("gemm_emul", n, s)
    rng = np.random.default_rng(10 * n + s)
    L = wide(rng, (n, n))            # not symmetric: D = L^T R is checked as such
    R = rng.standard_normal((n, n))
    R[:, : min(n, 40)] *= 1e-9       # columns of very different scale
    D = host(ipr.ipr_gemm_emul(dev(L), dev(R), s))
    ref = slices.product(L, R, s)
    assert np.array_equal(D, ref), np.abs(D - ref).max()


def test_emul_on_the_iteration_operands_matches_float64(ipr):
    """A and its inverse square root (the operands of the n = 1024 case):
    within the oracle's bound of the exact product and near a float64 product."""
    say("gemm_emul iterates")
    n = 1024
    a, _ = w.householder_spd(n, 1e4, seed=0)
    lam, v = np.linalg.eigh(a)
    c = (v * lam ** -0.5) @ v.T
    c = (c + c.T) / 2
    D = host(ipr.ipr_gemm_emul(dev(c), dev(a), 9))
    assert np.array_equal(D, slices.product(c, a, 9))
    f64 = host(ipr.ipr_gemm(dev(c), dev(a)))
    ext = c.astype(np.longdouble).T @ a.astype(np.longdouble)
    err_emul = float(np.abs(D - ext).max())
    err_f64 = float(np.abs(f64 - ext).max())
    assert np.all(np.abs(D - ext) <= slices.error_bound(c, a, 9))
    assert err_emul <= 4 * err_f64 + 1e-15, (err_emul, err_f64)


def test_emul_chunked_level_is_still_exact(ipr):
    """Order 11264 with 12 slices: the 12 pairs of level 13 exceed one int32
    accumulation (11 pairs fit), so that level runs in two chunks whose exact
    sums meet in float64. Sampled entries against the oracle, bit for bit."""
    say("gemm_emul chunked n=11264 s=12")
    n, s = 11264, 12
    g = torch.Generator(device="cpu").manual_seed(5)
    L = torch.randn(n, n, generator=g, dtype=torch.float64)
    R = torch.randn(n, n, generator=g, dtype=torch.float64)
    D = ipr.ipr_gemm_emul(L.cuda(), R.cuda(), s)
    rows = np.array([0, 1, 255, 256, 5000, n - 1])
    cols = np.array([0, 7, 511, 8191, n - 2, n - 1])
    Ln, Rn = L.numpy(), R.numpy()
    ref = slices.product(Ln[:, rows], Rn[:, cols], s)
    got = host(D)[np.ix_(rows, cols)]
    assert np.array_equal(got, ref)


def test_emul_full_size_sampled(ipr):
    """The n = 16384 product in the launch configuration the benchmark times
    (9 slices; level 10 runs in two chunks): sampled entries bit for bit."""
    say("gemm_emul n=16384 s=9")
    n, s = 16384, 9
    g = torch.Generator(device="cpu").manual_seed(6)
    L = torch.randn(n, n, generator=g, dtype=torch.float64)
    R = torch.randn(n, n, generator=g, dtype=torch.float64)
    L[:, :100] *= 1e-6
    D = ipr.ipr_gemm_emul(L.cuda(), R.cuda(), s)
    rows = np.array([0, 99, 100, 8000, n - 1])
    cols = np.array([1, 4095, 4096, 12345, n - 1])
    ref = slices.product(L.numpy()[:, rows], R.numpy()[:, cols], s)
    assert np.array_equal(host(D)[np.ix_(rows, cols)], ref)


def test_emul_non_finite_column_gives_nan(ipr):
    say("gemm_emul nan")
    rng = np.random.default_rng(3)
    n = 300
    L = rng.standard_normal((n, n))
    R = rng.standard_normal((n, n))
    L[5, 17] = np.inf
    D = host(ipr.ipr_gemm_emul(dev(L), dev(R), 9))
    assert np.isnan(D[17]).all()
    mask = np.ones(n, bool)
    mask[17] = False
    assert np.isfinite(D[mask]).all()
    assert np.array_equal(D[mask], slices.product(L[:, mask], R, 9))


def test_emul_argument_errors(ipr):
    say("gemm_emul errors")
    a = dev(np.eye(64))
    b = dev(np.eye(64))
    for s in (0, 13):
        with pytest.raises(ipr.IprError):
            ipr.ipr_gemm_emul(a, b, s)
    with pytest.raises(ipr.IprError):
        ipr.ipr_gemm_emul(a, b, 9, out=a)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ipr.IprError):
        ipr.ipr_gemm_emul(a, b, 9, workspace=small)
    assert ipr.ipr_gemm_emul_workspace(64, 0) == 0


# ---- the iteration with every product from int8 slices ---------------------

def emul_schedule(ipr, **kw):
    return ipr.ipr_schedule_default(bulk_dtype=ipr.IPR_FP64_INT8_EMUL, timing=1, **kw)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("n", [300, 517])
def test_emul_solve_reaches_the_root(ipr, n, p):
    from oracle import iteration as it
    say("emul solve", n, p)
    a, _, _ = w.spd_log_spectrum(n, 1e4, seed=70 + p)
    ref = it.eig_root(a, p)
    C, res = ipr.ipr_solve(dev(a), p, 1e-10, schedule=emul_schedule(ipr))
    _, r64 = ipr.ipr_solve(dev(a), p, 1e-10)
    assert res.status == ipr.IPR_OK, res.as_dict()
    assert res.residual_true < 1e-10
    assert it.rel_fro(host(C), ref) <= 1e-10
    assert res.iters_bulk == 0 and abs(res.iters_fp64 - r64.iters_fp64) <= 1
    # the iteration's products ran on the int8 matrix cores; the FP64 cores
    # did only the final check (p products)
    assert res.lp_gemm_launches >= res.iters_fp64
    assert res.gemm_launches <= p


def test_emul_headline_schedule_n1024(ipr):
    from oracle import iteration as it
    say("emul headline n=1024")
    a, _ = w.householder_spd(1024, 1e4, seed=0)
    s = emul_schedule(ipr, scale_squarings=6, dynamic_scaling=1)
    C, res = ipr.ipr_solve(dev(a), 2, 1e-10, schedule=s)
    assert res.status == ipr.IPR_OK, res.as_dict()
    assert res.residual_true < 1e-10
    assert it.rel_fro(host(C), it.eig_root(a, 2)) <= 1e-10


def test_emul_few_slices_floor_and_report_it(ipr):
    """Four digits (28 bits) cannot carry the iteration to 1e-10: the solve
    stops above it (on its floor) rather than claiming convergence."""
    say("emul 4 slices")
    a, _, _ = w.spd_log_spectrum(300, 1e2, seed=3)
    C, res = ipr.ipr_solve(dev(a), 2, 1e-10, schedule=emul_schedule(ipr, emul_slices=4),
                           raise_on=(ipr.IPR_EARG, ipr.IPR_EHIP))
    assert res.status != ipr.IPR_OK, res.as_dict()


def test_emul_argument_errors_of_the_solve(ipr):
    say("emul solve errors")
    a = dev(np.eye(64) * 2.0)
    for kw in ({"emul_slices": 13}, {"emul_slices": -1},
               {"evaluation": ipr.IPR_EVAL_LITERAL}):
        with pytest.raises(ipr.IprError):
            ipr.ipr_solve(a, 2, 1e-10, schedule=emul_schedule(ipr, **kw))
    A = torch.eye(64, dtype=torch.float64, device="cuda").reshape(-1) * 2.0
    with pytest.raises(ipr.IprError):
        ipr.ipr_solve_batched(A, [0], [64], [2], 1e-10, schedule=emul_schedule(ipr))
