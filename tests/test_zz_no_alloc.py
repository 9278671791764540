"""The allocation-free entry point ipr_solve_noalloc (the solve on the
library's fixed device scratch) against ipr_solve on the same inputs: the same
kernels on the same data, so the same iterate bit for bit, on two calls in a
row (the second smaller, on the scratch the first left behind)."""
import numpy as np
import pytest

import workloads as w
from oracle import iteration as it
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipr():
    import paper_1703_02283_amd as m
    m.load()
    return m


@pytest.mark.parametrize("sched", [{}, {"scale_squarings": 6, "dynamic_scaling": 1}])
def test_noalloc_matches_ipr_solve(ipr, sched):
    import torch
    for n, p, seed in ((1000, 2, 11), (300, 3, 12)):
        say("no-alloc solve n", n, "p", p, "schedule", sched)
        a, lam, _ = w.spd_log_spectrum(n, 1e3, seed=seed)
        A = dev(a)
        s = ipr.ipr_schedule_default(**sched)
        C_ref, r_ref = ipr.ipr_solve(A, p, 1e-10, schedule=s)
        C = torch.empty_like(A)
        torch.cuda.synchronize()
        C, r = ipr.ipr_solve_noalloc(A, p, 1e-10, schedule=s, out=C)
        torch.cuda.synchronize()
        say("  status", r.status, "iters", r.iters_fp64, "ref iters", r_ref.iters_fp64)
        assert r.status == ipr.IPR_OK and r_ref.status == ipr.IPR_OK
        assert r.iters_fp64 == r_ref.iters_fp64 and r.gemms == r_ref.gemms
        assert r.residual_true == r_ref.residual_true
        assert torch.equal(C, C_ref)
        assert r.ms_refine == 0.0                      # no events in this entry point
        c = host(C)
        assert it.rel_fro(c, it.eig_root(a, p)) <= 1e-10


def test_noalloc_rejects_what_it_cannot_hold(ipr):
    import torch
    n = 1100                                           # workspace beyond the 64 MiB scratch
    assert ipr.ipr_workspace_size(n, 2) > ipr.IPR_NOALLOC_SCRATCH_BYTES
    A = torch.eye(n, dtype=torch.float64, device="cuda")
    with pytest.raises(ipr.IprError) as ei:
        ipr.ipr_solve_noalloc(A, 2, 1e-10)
    assert ei.value.code == ipr.IPR_EARG and "scratch" in str(ei.value)
    A = torch.eye(64, dtype=torch.float64, device="cuda")
    with pytest.raises(ipr.IprError) as ei:            # timing needs events
        ipr.ipr_solve_noalloc(A, 2, 1e-10, schedule=ipr.ipr_schedule_default(timing=1))
    assert ei.value.code == ipr.IPR_EARG
    # a valid call afterwards still works (A = I: C = I)
    C, r = ipr.ipr_solve_noalloc(A, 2, 1e-10)
    torch.cuda.synchronize()
    assert r.status == ipr.IPR_OK and torch.equal(C, A)
