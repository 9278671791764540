"""GPU parity of the all-arithmetic regime (store_regime = 1: every scalar
operation rounded to a custom float or fixed-point type) against the
oracle's oracle/arith.py, bit for bit: both sum each dot product over k in
increasing order with one rounded multiply and one rounded add per term, so
the same float64 operations meet the same roundings. Inputs are put on a
2^-30 grid first, so that the norms of eq. (3) (and hence the start's scale)
are exact on both sides whatever their summation order."""
import numpy as np
import pytest

import workloads as w
from oracle import arith
from oracle import iteration as it
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
FMT = {"float": 1, "fixed": 2}


@pytest.fixture(scope="module")
def ipr():
    import paper_1703_02283_amd as m
    m.load()
    return m


def on_grid(a):
    g = np.ldexp(np.rint(np.ldexp(a, 30)), -30)
    return 0.5 * (g + g.T)


def arith_solve(ipr, a, p, fmt, bits, iters, ref=None):
    import torch
    err = (np.zeros(iters + 2) if ref is not None else None)
    rho = np.full(iters + 2, np.nan)
    s = ipr.ipr_schedule_default(store_format=FMT[fmt], store_bits=bits, store_regime=1,
                                 max_iter=iters)
    R = dev(ref) if ref is not None else None
    if R is not None:
        s.hist_ref = R.data_ptr()
        s.hist_err = err.ctypes.data
    s.hist_rho = rho.ctypes.data
    s.hist_len = iters + 2
    C, res = ipr.ipr_solve(dev(a), p, 1e-30, schedule=s, raise_on=(ipr.IPR_EARG, ipr.IPR_EHIP))
    torch.cuda.synchronize()
    return host(C), res, err, rho


@pytest.mark.parametrize("fmt,bits", [("float", 10), ("float", 16), ("fixed", 18)])
@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("n", [40, 130])
def test_dense_matrix_bitwise(ipr, n, p, fmt, bits):
    say("all arithmetic dense n", n, "p", p, fmt, bits)
    a = on_grid(w.kernel_matrix(n, seed=n, box=20.0 * (n / 768) ** (1 / 3)))
    iters = 12
    root = it.eig_root(a, p)
    c, res, err, rho = arith_solve(ipr, a, p, fmt, bits, iters, ref=root)
    k = res.iters_fp64            # (fewer than `iters` if the floor rule stopped it)
    say("  iterations", k, "status", res.status, "error", err[k])
    assert k >= 3, res.as_dict()
    ref_c, ref_err, ref_rho = arith.coupled_arith(a, p, k, fmt, bits)
    assert np.array_equal(c, ref_c), np.abs(c - ref_c).max()
    assert np.allclose(err[:k + 1], ref_err, rtol=1e-12, atol=1e-300)
    assert np.allclose(rho[:k + 1], ref_rho, rtol=1e-12, atol=1e-300)
    assert np.isfinite(res.residual_true)


def test_diagonal_matrix_bitwise(ipr):
    lam = np.geomspace(0.02, 1.0, 70)
    a = np.diag(lam)
    c, res, _, _ = arith_solve(ipr, a, 2, "float", 10, 9)
    ref_c, _, _ = arith.coupled_arith(a, 2, res.iters_fp64, "float", 10)
    assert np.array_equal(c, ref_c)


def test_all_arithmetic_floor_above_storage_at_768(ipr):
    """The paper's N = 768, p = 2 case on the overlap-like stand-in: with
    every operation rounded the error settles higher than with storage-only
    rounding of as many bits, and falls as bits are added."""
    import torch
    a = w.kernel_matrix(768, seed=0)
    root = it.eig_root(a, 2)
    R = dev(root)
    floors = {}
    for regime in (0, 1):
        for bits in (10, 16, 23):
            err = np.zeros(42)
            s = ipr.ipr_schedule_default(store_format=1, store_bits=bits, store_regime=regime,
                                         max_iter=40)
            s.hist_ref, s.hist_err, s.hist_len = R.data_ptr(), err.ctypes.data, 42
            _, res = ipr.ipr_solve(dev(a), 2, 1e-10, schedule=s,
                                   raise_on=(ipr.IPR_EARG, ipr.IPR_EHIP))
            torch.cuda.synchronize()
            floors[(regime, bits)] = err[:res.iters_fp64 + 1].min()
            say("  regime", regime, "bits", bits, "iterations", res.iters_fp64,
                "status", res.status, "lowest error", floors[(regime, bits)])
    for bits in (10, 16, 23):
        assert floors[(1, bits)] > floors[(0, bits)]
    assert floors[(1, 10)] > floors[(1, 16)] > floors[(1, 23)]
