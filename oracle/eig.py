"""Eigenvalues of a dense symmetric matrix (the step after the Loewdin
transform of Section IV-A: the eigenvalues of S^{-1/2} H S^{-1/2} are those of
the generalized problem H c = e S c).

Test infrastructure only (see the package docstring).

The definition is the spectrum itself; numpy's eigvalsh (LAPACK's symmetric
eigensolver) serves as the step that computes it, ascending.
"""
from __future__ import annotations

import numpy as np


def eigenvalues(a: np.ndarray) -> np.ndarray:
    """The eigenvalues of the symmetric matrix a, ascending."""
    a = np.asarray(a, dtype=np.float64)
    if not np.array_equal(a, a.T):
        raise ValueError("the matrix must be exactly symmetric")
    return np.linalg.eigvalsh(a)
