"""Plain NumPy reference of the 16 cheap matrix features read by the learned
initial guess.

Test infrastructure only (see the package docstring).

All features are O(n^2) functions of A (n x n, symmetric) and p. With
sigma = sqrt(||A||_1 ||A||_inf) (the scale of the start in eq. (3)) and
B = A / sigma, d = diag(B), s_i = sum_j |B_ij|, o_i = s_i - |d_i|:

  0 clamp(log2 n, 6, 10)/10 (the order, clipped to the training sizes)
  1 p/4                2 t1 = trace(B)/n
  3 t2 = ||B||_F^2/n   4 log10 t1          5 log10 t2
  6 t1^2/t2            7 min d             8 max d
  9 log10 max(min d, 1e-30)               10 min_i (d_i - o_i)  (Gershgorin low)
 11 mean_i s_i         12 sum o / sum |d|  13 max_{i!=j} |B_ij|
 14 std(d)/mean(d)     15 log10 sigma
"""
from __future__ import annotations

import numpy as np

N_FEATURES = 16


def features(a: np.ndarray, p: int) -> np.ndarray:
    n = a.shape[0]
    s1 = float(np.max(np.sum(np.abs(a), axis=0)))
    si = float(np.max(np.sum(np.abs(a), axis=1)))
    sigma = np.sqrt(s1 * si)
    b = a / sigma
    d = np.diag(b).copy()
    s = np.sum(np.abs(b), axis=1)
    o = s - np.abs(d)
    t1 = float(np.sum(d)) / n
    t2 = float(np.sum(b * b)) / n
    off = np.abs(b - np.diag(d))
    return np.array([
        min(max(np.log2(n), 6.0), 10.0) / 10.0,
        p / 4.0,
        t1,
        t2,
        np.log10(t1),
        np.log10(t2),
        t1 * t1 / t2,
        d.min(),
        d.max(),
        np.log10(max(d.min(), 1e-30)),
        float(np.min(d - o)),
        float(np.mean(s)),
        float(np.sum(o) / np.sum(np.abs(d))),
        float(off.max()) if n > 1 else 0.0,
        float(np.std(d) / np.mean(d)),
        np.log10(sigma),
    ])
