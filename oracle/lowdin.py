"""Löwdin orthogonalisation, the step that follows the inverse square root in
the paper's application (Section IV-A): the generalised eigenproblem
H c = e S c of a non-orthogonal basis becomes the standard problem
(S^{-1/2} H S^{-1/2}) y = e y with c = S^{-1/2} y.

Test infrastructure only (see the package docstring).

Pins (tests/test_oracle_lowdin.py): the eigenvalues of the transformed
matrix equal the generalised eigenvalues of (H, S) from scipy.linalg.eigh;
S = I leaves H unchanged; diagonal S gives h_ij / sqrt(s_i s_j); the
back-transformed vectors satisfy H c = e S c and are S-orthonormal.
"""
from __future__ import annotations

import numpy as np

from oracle.iteration import eig_root


def lowdin(s: np.ndarray, h: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(X, X H X) with X = S^{-1/2} from the definition (eigendecomposition)."""
    x = eig_root(s, 2)
    return x, x @ h @ x
