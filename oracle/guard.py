"""Convergence guard for polynomial starts (Section II, eq. (2)).

Test infrastructure only (see the package docstring).

For C_0 = sigma^{-1/p} q(A/sigma), q(x) = b0 + b1 x + b2 x^2 and
sigma = sqrt(||A||_1 ||A||_inf), the eigenvalues of C_0^p A are
phi(x) = q(x)^p x at the eigenvalues x of A/sigma, which lie in (0, 1]
(||A||_2 <= sigma). Eq. (2), ||I - C_0^p A||_2 < 1, holds when
0 < phi(x) < 2 on the spectrum, and q(x) > 0 keeps the iterates on the
principal (positive) branch. This reference checks phi and q on a dense grid of
(0, 1], which is what a reader can verify by eye.
"""
from __future__ import annotations

import numpy as np


def phi(x, b, p):
    q = b[0] + b[1] * x + b[2] * x * x
    return q ** p * x, q


def check(b, p, grid: int = 200001):
    """Returns (accept, sup_phi, min_q) over x in (0, 1] sampled on ``grid`` points."""
    x = np.linspace(0.0, 1.0, grid)[1:]
    f, q = phi(x, b, p)
    sup = float(np.max(f))
    qmin = float(np.min(q))
    return (qmin > 0.0 and sup < 2.0), sup, qmin
