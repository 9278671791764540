"""Approximate arithmetic: every scalar operation of the iteration rounded
(Section IV: custom-precision types "for all involved calculations"; Section
IV-B methodology; Section IV-C, Figs. 2a and 3a).

Test infrastructure only (see the package docstring).

The paper simulates custom floating-point and fixed-point types by giving
NumPy arrays a scalar type whose addition, subtraction and multiplication
return values of that type: every operation of the iteration is computed and
then rounded. Here that regime is applied to the coupled form of eq. (1) from
the scaled identity, the same iteration the approximate-storage oracle runs
(``oracle.storage``), with rnd() = ``storage.store`` (custom float with
``bits`` stored mantissa bits and unbounded exponent, or fixed point with
``bits`` fractional bits; round to nearest, ties to even). Each operation is
one float64 operation followed by rnd():

* the input and the start's scalars are in the type: A~ = rnd(A),
  c = rnd(sigma^(-1/p)), c_p = rnd(c^p) with sigma = sqrt(||A||_1 ||A||_inf)
  (the scale itself is a start parameter, computed in float64);
* C_0 = c I, M_0 = rnd(c_p A~) entry by entry;
* R = rnd(I - M), N = rnd(I + rnd(R / p)) entry by entry (the p-th part of
  the residual added to the identity);
* a product D = X^T Y of the iteration's symmetric matrices: for i <= j the
  dot product over k = 0, 1, ..., n - 1 in that order, acc <- rnd(acc +
  rnd(x_ki y_kj)) from acc = 0; D_ji = D_ij (one triangle computed and
  mirrored, as everywhere in this build);
* C_{k+1} = C_k N_k, M_{k+1} = N_k (N_k (... (N_k M_k))) (p products), then
  N_{k+1} from M_{k+1}.

The error ||C_k - A^{-1/p}||_F (Section IV-C's metric, against the float64
root) and the residual ||I - M_k||_F are measured in float64.
"""
from __future__ import annotations

import math

import numpy as np

from oracle.iteration import norm_1, norm_inf, eig_root
from oracle.storage import store


def rnd(x, fmt: str, bits: int):
    """One value (or array) of the custom type: storage.store's rounding."""
    return store(np.asarray(x, dtype=np.float64), fmt, bits)


def product(x: np.ndarray, y: np.ndarray, fmt: str, bits: int) -> np.ndarray:
    """D = X^T Y with every multiplication and every partial sum rounded, the
    sum over k in increasing order; the upper triangle is computed and
    mirrored (the iteration's products are symmetric)."""
    n = x.shape[0]
    iu, ju = np.triu_indices(n)
    acc = np.zeros(iu.size)
    for k in range(n):
        acc = rnd(acc + rnd(x[k, iu] * y[k, ju], fmt, bits), fmt, bits)
    d = np.zeros((n, n))
    d[iu, ju] = acc
    d[ju, iu] = acc
    return d


def next_n(m: np.ndarray, p: int, fmt: str, bits: int) -> np.ndarray:
    """N = rnd(I + rnd(rnd(I - M) / p)) entry by entry."""
    eye = np.eye(m.shape[0])
    r = rnd(eye - m, fmt, bits)
    return rnd(eye + rnd(r / p, fmt, bits), fmt, bits)


def coupled_arith(a: np.ndarray, p: int, iters: int, fmt: str, bits: int):
    """Run `iters` coupled updates with every operation rounded.

    Returns (C_iters, errors, residuals): errors[k] = ||C_k - A^{-1/p}||_F
    against the float64 root of A, residuals[k] = ||I - M_k||_F."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    eye = np.eye(n)
    sigma = math.sqrt(norm_1(a) * norm_inf(a))
    c0 = float(rnd(sigma ** (-1.0 / p), fmt, bits))
    cp = float(rnd(c0 ** p, fmt, bits))
    at = rnd(a, fmt, bits)
    c = c0 * eye
    m = rnd(cp * at, fmt, bits)
    nmat = next_n(m, p, fmt, bits)
    root = eig_root(a, p)
    errors = [float(np.linalg.norm(c - root))]
    residuals = [float(np.linalg.norm(eye - m))]
    for _ in range(iters):
        c_new = product(c, nmat, fmt, bits)
        x = m
        for _ in range(p):
            x = product(nmat, x, fmt, bits)
        c, m = c_new, x
        nmat = next_n(m, p, fmt, bits)
        errors.append(float(np.linalg.norm(c - root)))
        residuals.append(float(np.linalg.norm(eye - m)))
    return c, errors, residuals
