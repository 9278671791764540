"""GPU parity of the symmetric eigenvalue solver (ipr_eigvalsh: Householder
tridiagonalisation and Sturm multisection) against the oracle (oracle/eig.py),
closed forms, and the generalised eigenvalues of the Loewdin problem."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import workloads as w
from oracle import eig
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipr():
    import paper_1703_02283_amd as m
    m.load()
    return m


def bound(n, lam):
    # backward error of the reduction: a modest multiple of n u ||A||_2
    return 8.0 * n * 2.0 ** -53 * max(np.abs(lam).max(), 1e-300)


@pytest.mark.parametrize("n", [1, 2, 3, 64, 130, 257, 700])
def test_random_symmetric(ipr, n):
    say("eigvalsh random n", n)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n))
    a = x + x.T
    got = host(ipr.ipr_eigvalsh(dev(a)))
    ref = eig.eigenvalues(a)
    assert np.all(np.diff(got) >= 0)
    assert np.max(np.abs(got - ref)) <= bound(n, ref), np.max(np.abs(got - ref))


def test_bench_order_4096(ipr):
    # the order the bench's Loewdin section solves, against LAPACK's values
    n = 4096
    rng = np.random.default_rng(4096)
    x = rng.standard_normal((n, n))
    a = x + x.T
    got = host(ipr.ipr_eigvalsh(dev(a)))
    ref = eig.eigenvalues(a)
    say("eigvalsh n 4096: max error", np.max(np.abs(got - ref)), "bound", bound(n, ref))
    assert np.all(np.diff(got) >= 0)
    assert np.max(np.abs(got - ref)) <= bound(n, ref)


def test_all_row_tiers_of_the_column_step(ipr):
    # trailing blocks above order 4096 take four rows per wave, above 2048 two,
    # then one: n = 4500 runs through all three
    n = 4500
    rng = np.random.default_rng(4500)
    x = rng.standard_normal((n, n))
    a = x + x.T
    got = host(ipr.ipr_eigvalsh(dev(a)))
    ref = eig.eigenvalues(a)
    say("eigvalsh n 4500: max error", np.max(np.abs(got - ref)), "bound", bound(n, ref))
    assert np.all(np.diff(got) >= 0)
    assert np.max(np.abs(got - ref)) <= bound(n, ref)


def test_closed_forms_and_degenerate_spectra(ipr):
    n = 1000
    t = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    ref = np.sort(2.0 - 2.0 * np.cos(np.arange(1, n + 1) * math.pi / (n + 1)))
    got = host(ipr.ipr_eigvalsh(dev(t)))
    assert np.max(np.abs(got - ref)) <= bound(n, ref)
    # multiple eigenvalues: to the spacing of doubles
    got = host(ipr.ipr_eigvalsh(dev(3.5 * np.eye(200))))
    assert np.max(np.abs(got - 3.5)) <= 4 * 2.0 ** -52 * 3.5
    assert np.max(np.abs(host(ipr.ipr_eigvalsh(dev(np.zeros((50, 50))))))) <= 1e-300
    d = np.random.default_rng(1).standard_normal(300)
    got = host(ipr.ipr_eigvalsh(dev(np.diag(d))))
    assert np.max(np.abs(got - np.sort(d))) <= bound(300, d)
    # a matrix whose columns are already reduced below the first off-diagonal
    a = np.diag(np.arange(1.0, 9.0)) + np.diag(np.full(7, 0.5), 1) + np.diag(np.full(7, 0.5), -1)
    assert np.max(np.abs(host(ipr.ipr_eigvalsh(dev(a))) - eig.eigenvalues(a))) <= bound(8, a)


def test_loewdin_then_eigenvalues_are_the_generalised_ones(ipr):
    # the step after the root: X = S^{-1/2}, then the eigenvalues of X H X
    # are those of H c = e S c
    n = 1024
    s, h = w.overlap_and_hamiltonian(n, seed=5, box=20.0)
    X, Ht, res = ipr.ipr_lowdin(dev(s), dev(h), 1e-10)
    assert res.status == ipr.IPR_OK, res.as_dict()
    got = host(ipr.ipr_eigvalsh(Ht))
    ref = sl.eigh(h, s, eigvals_only=True)
    say("loewdin eigenvalues: largest difference", np.max(np.abs(got - ref)),
        "largest |e|", np.abs(ref).max())
    assert np.allclose(got, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_argument_errors(ipr):
    import torch
    a = dev(np.eye(8))
    with pytest.raises(ipr.IprError) as ei:
        ipr.ipr_eigvalsh(a, workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == ipr.IPR_EARG
