"""Approximate storage of the iteration's matrices (Sections III-C and IV).

Test infrastructure only (see the package docstring).

The paper's storage-only experiments keep the input and the intermediate
results of the iteration in a narrow type while the arithmetic stays
precise, and follow the error of C_k against the root. Here that regime is
applied to the coupled form of eq. (1) from the scaled identity:

* the input is stored: A~ = store(A);
* the start is stored: C_0 = store(c I), M_0 = store(A~ / sigma),
  N_0 = store(I + (I - A~ / sigma) / p), with sigma = sqrt(||A||_1 ||A||_inf)
  and c = sigma^(-1/p) (the scaled identity of the design notes);
* every matrix the iteration keeps between products is stored when it is
  written: C_{k+1} = store(sym(C_k N_k)); for N^p M the intermediates
  X_j = store(sym(N X_{j-1})) (X_0 = M_k) and M_{k+1} = store(sym(N X_{p-1}));
  N_{k+1} = store((p + 1)/p I - M_{k+1}/p) from the stored M_{k+1};
* products are float64 and symmetrised, sym(X) = (X + X^T)/2, before the
  rounding.

store() is the custom float of the paper's experiments (``bits`` stored
mantissa bits, unbounded exponent) or fixed point (``bits`` fractional bits,
enough integer bits), both rounded to nearest with ties to even. Where the
paper does not say which matrices count as stored intermediates, the
reading is every matrix that lives in memory between two products (design
notes, reading R16).
"""
from __future__ import annotations

import math

import numpy as np

from oracle.iteration import norm_1, norm_inf, eig_root


def store(x: np.ndarray, fmt: str | None, bits: int) -> np.ndarray:
    """x as the approximate storage keeps it."""
    if fmt is None:
        return np.asarray(x, dtype=np.float64)
    if fmt == "float":
        # round_custom's rule, with the scaling done by ldexp so that values
        # whose last stored bit lies below the float64 range stay finite
        x = np.asarray(x, dtype=np.float64)
        _, e = np.frexp(x)               # x = f 2^e, 0.5 <= |f| < 1
        sh = e - 1 - bits                # weight of the last stored bit
        return np.where(x == 0.0, x, np.ldexp(np.rint(np.ldexp(x, -sh)), sh))
    if fmt == "fixed":
        return np.ldexp(np.rint(np.ldexp(np.asarray(x, dtype=np.float64), bits)), -bits)
    raise ValueError(fmt)


def _sym(x: np.ndarray) -> np.ndarray:
    return (x + x.T) / 2.0


def coupled_stored(a: np.ndarray, p: int, iters: int, fmt: str | None, bits: int = 0):
    """Run `iters` coupled updates with approximate storage.

    Returns (C_iters, errors, residuals): errors[k] = ||C_k - A^{-1/p}||_F
    (the paper's error measure against the float64 root of the stored-free
    A), residuals[k] = ||I - M_k||_F of the stored M_k.
    """
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    eye = np.eye(n)
    s2 = norm_1(a) * norm_inf(a)
    sigma = math.sqrt(s2)
    c0 = sigma ** (-1.0 / p)
    cp = 1.0 / sigma
    at = store(a, fmt, bits)
    m0 = cp * at
    c = store(c0 * eye, fmt, bits)
    m = store(m0, fmt, bits)
    nmat = store(eye + (eye - m0) * (1.0 / p), fmt, bits)
    root = eig_root(a, p)
    errors = [float(np.linalg.norm(c - root))]
    residuals = [float(np.linalg.norm(eye - m))]
    sa, sc = (p + 1.0) / p, -1.0 / p
    for _ in range(iters):
        c_new = store(_sym(c @ nmat), fmt, bits)
        x = m
        for j in range(p):
            y = _sym(nmat @ x)
            x = store(y, fmt, bits)
        m_new = x
        n_new = store(sa * eye + sc * m_new, fmt, bits)
        c, m, nmat = c_new, m_new, n_new
        errors.append(float(np.linalg.norm(c - root)))
        residuals.append(float(np.linalg.norm(eye - m)))
    return c, errors, residuals
