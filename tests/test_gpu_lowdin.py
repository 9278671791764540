"""GPU parity of the Loewdin transform (ipr_lowdin) against the oracle and
scipy's generalised eigenvalues."""
import numpy as np
import pytest
import scipy.linalg as sl
import torch

import workloads as w
from oracle import iteration as it
from oracle import lowdin
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipr():
    import paper_1703_02283_amd as m
    m.load()
    return m


@pytest.mark.parametrize("n,box", [(300, 12.0), (1024, 20.0)])
def test_lowdin_matches_oracle_and_generalised_eigenvalues(ipr, n, box):
    say("lowdin", n)
    s, h = w.overlap_and_hamiltonian(n, seed=5, box=box)
    X, Ht, res = ipr.ipr_lowdin(dev(s), dev(h), 1e-10)
    assert res.status == ipr.IPR_OK, res.as_dict()
    x_ref, ht_ref = lowdin.lowdin(s, h)
    x, ht = host(X), host(Ht)
    assert it.rel_fro(x, x_ref) <= 1e-10
    assert it.rel_fro(ht, ht_ref) <= 1e-9
    assert np.array_equal(ht, ht.T)
    ev = np.linalg.eigvalsh(ht)
    ref = sl.eigh(h, s, eigvals_only=True)
    assert np.allclose(ev, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_lowdin_reports_the_solve_status_and_leaves_hout(ipr):
    say("lowdin status")
    s, h = w.overlap_and_hamiltonian(200, seed=6, box=12.0)
    sch = ipr.ipr_schedule_default(max_iter=2)
    Ht = torch.full((200, 200), 7.0, dtype=torch.float64, device="cuda")
    _, _, res = ipr.ipr_lowdin(dev(s), dev(h), 1e-10, schedule=sch, out_h=Ht,
                               raise_on=(ipr.IPR_EARG, ipr.IPR_EHIP))
    assert res.status == ipr.IPR_EMAXITER
    assert bool((Ht == 7.0).all())


def test_lowdin_argument_errors(ipr):
    say("lowdin errors")
    s, h = w.overlap_and_hamiltonian(64, seed=7, box=8.0)
    S, H = dev(s), dev(h)
    with pytest.raises(ipr.IprError):
        ipr.ipr_lowdin(S, H, 1e-10, out_h=H)
    with pytest.raises(ipr.IprError):
        ipr.ipr_lowdin(S, H, 1e-10, out_x=H)
    with pytest.raises(ipr.IprError):
        ipr.ipr_lowdin(S, H, 1e-10, workspace=torch.empty(64, dtype=torch.uint8, device="cuda"))
