"""GPU parity of the low-precision products against the oracle's rounding
emulator, and of the mixed-precision schedules against the FP64 oracle."""
import numpy as np
import pytest

import workloads as w
from oracle import iteration as it
from oracle import rounding
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
FMTS = [(1, "bf16"), (2, "fp16"), (3, "fp8_e4m3")]


@pytest.fixture(scope="module")
def ipr():
    import paper_1703_02283_amd as m
    m.load()
    return m


@pytest.mark.parametrize("dtype,fmt", FMTS)
@pytest.mark.parametrize("n", [1, 100, 128, 300, 520])
def test_gemm_lowp_matches_emulator(ipr, dtype, fmt, n):
    say("gemm_lowp", fmt, n)
    rng = np.random.default_rng(n + dtype)
    L = rng.standard_normal((n, n))
    R = rng.standard_normal((n, n))
    L[: min(n, 64), :] *= 1e-3          # tiles of very different magnitude
    R[:, 128:200] *= 37.0
    D = host(ipr.ipr_gemm_lowp(dev(L), dev(R), dtype))
    qa = rounding.dequantize(*rounding.quantize(L, fmt, 128), 128)
    qb = rounding.dequantize(*rounding.quantize(R, fmt, 128), 128)
    ref = qa.T @ qb
    mag = np.abs(qa).T @ np.abs(qb)
    bound = 2 * n * 2.0 ** -24 * mag + 1e-300
    if fmt == "fp8_e4m3":
        # the fp8 matrix-core instruction does not sum its products exactly in
        # fp32: measured on gfx950, its error reaches ~2^-15.6 of sum |products|
        bound = bound + 2.0 ** -14 * mag
    assert np.all(np.abs(D - ref) <= bound)


@pytest.mark.parametrize("dtype", [1, 2, 3])
@pytest.mark.parametrize("n", [256, 300])
def test_p1_lowp_bulk_then_fp64_newton_schulz_reaches_oracle(ipr, dtype, n):
    say("mixed p=1 dtype", dtype, "n", n)
    a, _, _ = w.spd_log_spectrum(n, 1e2, seed=40 + dtype)
    s = ipr.ipr_schedule_default(bulk_dtype=dtype)
    C, res = ipr.ipr_solve(dev(a), 1, 1e-11, schedule=s)
    c = host(C)
    ref = it.solve(a, 1, 1e-11, evaluation="newton_schulz")
    assert res.status == ipr.IPR_OK, res.as_dict()
    assert res.iters_bulk > 0
    # fp8 (3 stored bits) stalls after a few iterations and saves little
    assert res.iters_fp64 < ref.iters if dtype != 3 else res.iters_fp64 <= ref.iters
    assert it.rel_fro(c, ref.c) <= 1e-10


@pytest.mark.parametrize("dtype", [1, 2])
def test_p1_lowp_bulk_with_scaled_steps(ipr, dtype):
    # scaled Newton-Schulz steps in the bulk phase (factor in the update's
    # epilogue, chosen from the Lanczos bounds): fewer bulk iterations than
    # the plain bulk phase, no restart, the same root as the oracle's
    say("mixed p=1 scaled bulk dtype", dtype)
    a, _, _ = w.spd_log_spectrum(300, 1e2, seed=60 + dtype)
    C0, r0 = ipr.ipr_solve(dev(a), 1, 1e-11, schedule=ipr.ipr_schedule_default(bulk_dtype=dtype))
    s = ipr.ipr_schedule_default(bulk_dtype=dtype, dynamic_scaling=1, scale_lanczos=1)
    C, res = ipr.ipr_solve(dev(a), 1, 1e-11, schedule=s)
    say("  bulk iterations", res.iters_bulk, "plain bulk", r0.iters_bulk, "fp64", res.iters_fp64)
    assert res.status == ipr.IPR_OK and res.fallback_used == 0, res.as_dict()
    assert 0 < res.iters_bulk < r0.iters_bulk
    ref = it.solve(a, 1, 1e-11, evaluation="newton_schulz")
    assert it.rel_fro(host(C), ref.c) <= 1e-10
    assert it.rel_fro(host(C), it.eig_root(a, 1)) <= 1e-10


def test_p1_bf16_bulk_on_kernel_matrix(ipr):
    a = w.kernel_matrix(512, seed=3)
    s = ipr.ipr_schedule_default(bulk_dtype=1)
    C, res = ipr.ipr_solve(dev(a), 1, 1e-10, schedule=s)
    assert res.status == ipr.IPR_OK, res.as_dict()
    assert it.rel_fro(host(C), np.linalg.inv(a)) <= 1e-9


@pytest.mark.parametrize("dtype", [1, 2])
def test_p2_lowp_bulk_restarts_in_fp64(ipr, dtype):
    # For p >= 2 the low-precision phase leaves an error that does not commute
    # with A; FP64 steps of the coupled form amplify it (the residual grows or
    # stalls). The solver notices and starts again in FP64 from the scaled
    # identity, so the answer is right but the bulk phase was wasted.
    # So by default the phase is skipped for p >= 2 (bulk_skipped) and the
    # solve is the FP64 one; bulk_force runs it anyway.
    a, _, _ = w.spd_log_spectrum(256, 1e2, seed=8)
    ref = it.eig_root(a, 2)
    C64, r64 = ipr.ipr_solve(dev(a), 2, 1e-10)
    C, res = ipr.ipr_solve(dev(a), 2, 1e-10, schedule=ipr.ipr_schedule_default(bulk_dtype=dtype))
    assert res.status == ipr.IPR_OK and res.bulk_skipped == 1 and res.iters_bulk == 0
    assert res.fallback_used == 0 and res.gemms == r64.gemms
    assert np.array_equal(host(C), host(C64))
    s = ipr.ipr_schedule_default(bulk_dtype=dtype, bulk_force=1)
    C, res = ipr.ipr_solve(dev(a), 2, 1e-10, schedule=s)
    assert res.status == ipr.IPR_OK and res.fallback_used == 1, res.as_dict()
    assert res.residual_true < 1e-10 and res.iters_bulk > 0 and res.bulk_skipped == 0
    assert it.rel_fro(host(C), ref) <= 1e-10
    assert res.gemms > r64.gemms
    # as an approximation (the paper's first use case: a few-percent error,
    # Frobenius residual of order one at n = 256) it needs no FP64 step
    C, res = ipr.ipr_solve(dev(a), 2, 10.0, schedule=s)
    assert res.status == ipr.IPR_OK and res.iters_fp64 == 0 and res.iters_bulk > 0


@pytest.fixture(scope="module")
def big_operands():
    """One operand X per full size (float32 normals widened to float64, tiles
    of very different magnitude); the product X^T X is symmetric, so the
    triangle mode's mirrored tiles have a reference too."""
    out = {}
    for n in (4096, 16384):
        rng = np.random.default_rng(n)
        x = rng.standard_normal((n, n), dtype=np.float32).astype(np.float64)
        x[:64, :] *= 1e-3
        x[:, 128:200] *= 37.0
        x[:, 3000:3100] *= 1e-2
        out[n] = x
    return out


@pytest.mark.parametrize("dtype,fmt", FMTS)
@pytest.mark.parametrize("n,tri", [(4096, 0), (4096, 1), (16384, 1), (16384, 0)])
def test_gemm_lowp_full_size_sampled(ipr, big_operands, dtype, fmt, n, tri):
    # the sizes of the bulk phases: at n = 16384 every workgroup of the
    # persistent kernel walks several output tiles; sampled rows and columns
    # (tile edges included) against the emulator on the same rounded operands
    import torch
    say("gemm_lowp full size", fmt, "n", n, "triangle", tri)
    x = big_operands[n]
    X = dev(x)
    D = ipr.ipr_gemm_lowp(X, X, dtype, triangle=bool(tri))
    rng = np.random.default_rng(7 * n + dtype)
    edges = {0, 127, 128, 255, 256, 4095, n - 256, n - 1}
    rows = np.array(sorted(edges | set(rng.choice(n, 40, replace=False).tolist())))
    cols = np.array(sorted(edges | set(rng.choice(n, 40, replace=False).tolist())))
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    got = host(D.index_select(0, ri).index_select(1, ci))
    got_t = host(D.index_select(0, ci).index_select(1, ri))
    del D, X
    torch.cuda.empty_cache()
    qx = rounding.dequantize(*rounding.quantize(x, fmt, 128), 128)
    ref = qx[:, rows].T @ qx[:, cols]
    mag = np.abs(qx[:, rows]).T @ np.abs(qx[:, cols])
    bound = 2 * n * 2.0 ** -24 * mag + 1e-300
    if fmt == "fp8_e4m3":
        bound = bound + 2.0 ** -14 * mag
    err = np.max(np.abs(got - ref) / (mag + 1e-300))
    say("  largest error / sum |products|", err)
    assert np.all(np.abs(got - ref) <= bound)
    if tri:
        assert np.array_equal(got, got_t.T)          # mirrored exactly
