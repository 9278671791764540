"""Pins of the eigenvalue oracle (oracle/eig.py) against closed forms and
invariants that a mistake in the call (a transposed or unsorted result, a
wrong triangle) would break."""
import math

import numpy as np

from oracle import eig


def test_tridiagonal_toeplitz_closed_form():
    # a on the diagonal, b beside it: a + 2 b cos(k pi / (n + 1)), k = 1..n
    for n, a, b in ((1, 2.0, 0.0), (5, 2.0, -1.0), (64, 0.3, 0.7)):
        t = np.diag(np.full(n, a)) + np.diag(np.full(n - 1, b), 1) + np.diag(np.full(n - 1, b), -1)
        ref = np.sort(a + 2 * b * np.cos(np.arange(1, n + 1) * math.pi / (n + 1)))
        assert np.allclose(eig.eigenvalues(t), ref, rtol=0, atol=1e-14 * (abs(a) + 2 * abs(b)))


def test_two_by_two_and_diagonal():
    # [[p, q], [q, r]]: (p + r)/2 -+ sqrt(((p - r)/2)^2 + q^2)
    p, q, r = 3.0, -1.5, 0.5
    m, h = (p + r) / 2, math.sqrt(((p - r) / 2) ** 2 + q * q)
    assert np.allclose(eig.eigenvalues(np.array([[p, q], [q, r]])), [m - h, m + h], atol=1e-15)
    d = np.array([4.0, -2.0, 0.5, 9.0])
    assert np.array_equal(eig.eigenvalues(np.diag(d)), np.sort(d))


def test_trace_and_frobenius_invariants():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((50, 50))
    a = x + x.T
    lam = eig.eigenvalues(a)
    assert np.all(np.diff(lam) >= 0)
    assert abs(lam.sum() - np.trace(a)) < 1e-12 * np.abs(a).sum()
    assert abs((lam ** 2).sum() - (a * a).sum()) < 1e-12 * (a * a).sum()
    # a similarity by an orthogonal matrix leaves the spectrum unchanged
    q, _ = np.linalg.qr(rng.standard_normal((50, 50)))
    b = q @ a @ q.T
    b = 0.5 * (b + b.T)
    assert np.allclose(eig.eigenvalues(b), lam, atol=1e-12 * np.abs(lam).max())
