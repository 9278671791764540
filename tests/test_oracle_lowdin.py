"""Pins of the Löwdin oracle against scipy's generalised eigensolver and
closed forms."""
import numpy as np
import scipy.linalg as sl

import workloads as w
from oracle import lowdin


def test_eigenvalues_are_the_generalised_eigenvalues():
    s, h = w.overlap_and_hamiltonian(200, seed=1)
    _, ht = lowdin.lowdin(s, h)
    ev = np.linalg.eigvalsh(0.5 * (ht + ht.T))
    ref = sl.eigh(h, s, eigvals_only=True)
    assert np.allclose(ev, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_identity_overlap_leaves_h():
    rng = np.random.default_rng(2)
    h = rng.standard_normal((30, 30))
    h = h + h.T
    x, ht = lowdin.lowdin(np.eye(30), h)
    assert np.allclose(x, np.eye(30), atol=1e-15) and np.allclose(ht, h, atol=1e-14)


def test_diagonal_overlap_closed_form():
    rng = np.random.default_rng(3)
    d = rng.uniform(0.1, 4.0, 20)
    h = rng.standard_normal((20, 20))
    h = h + h.T
    _, ht = lowdin.lowdin(np.diag(d), h)
    assert np.allclose(ht, h / np.sqrt(np.outer(d, d)), rtol=1e-13, atol=1e-14)


def test_back_transformed_vectors_solve_the_generalised_problem():
    s, h = w.overlap_and_hamiltonian(150, seed=4, box=12.0)
    x, ht = lowdin.lowdin(s, h)
    e, y = np.linalg.eigh(0.5 * (ht + ht.T))
    c = x @ y
    assert np.allclose(h @ c, s @ c * e, atol=1e-8 * np.abs(e).max())
    assert np.allclose(c.T @ s @ c, np.eye(150), atol=1e-9)


def test_overlap_generator_is_the_kernel_matrix_and_h_is_symmetric():
    s, h = w.overlap_and_hamiltonian(300, seed=9, box=15.0)
    assert np.array_equal(s, w.kernel_matrix(300, seed=9, box=15.0))
    assert np.array_equal(h, h.T)
    # kinetic form: H_ij / S_ij = (3 - d^2 / 2) / 4 off the diagonal, with d^2 = -2 log S_ij
    i, j = np.triu_indices(300, 1)
    keep = s[i, j] > 1e-6
    d2 = -2.0 * np.log(s[i, j][keep])
    assert np.allclose(h[i, j][keep] / s[i, j][keep], (3.0 - d2 / 2.0) / 4.0, rtol=1e-9, atol=1e-9)
