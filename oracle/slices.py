"""FP64-accurate products from 8-bit integer slices.

Test infrastructure only (see the package docstring).

The paper asks for low-precision arithmetic units that still deliver the
accuracy the iteration needs (Section III-B). Its storage regime rounds the
operands and loses their low bits; an error-free splitting keeps them. This
module follows the splitting of Ozaki, Ogita, Oishi and Rump (Numer.
Algorithms 59, 2012), specialised to integer slices of beta = 7 bits, as the
int8 matrix-core path computes it:

1. Row scale. For row i of an operand X (k entries), e_i is the smallest
   integer with max_j |x_ij| < 2^e_i (0 for a zero row), so y = x 2^-e_i lies
   in (-1, 1).
2. Digits. d_1 = round(2^beta y), r_1 = 2^beta y - d_1, d_2 = round(2^beta r_1),
   and so on to d_s, each rounded to nearest (ties to even) and clamped to
   [-127, 127] (2^beta y can reach 128 only by rounding up; the clamp leaves
   a remainder of magnitude at most 1). Rounding to nearest rather than
   truncating keeps the digit remainders unbiased, so over k they add like
   a random walk instead of in step with the operand's sign. Every step is
   exact in float64 (a power-of-two scaling and the removal of an integer),
   and y = sum_t d_t 2^(-beta t) + 2^(-beta s) r with |r| <= 1.
3. Product. For D = L^T R the rows of L^T (columns of L) and of R^T (columns
   of R) are split: a_t and b_u. The integer products P_tu = a_t b_u^T are
   exact. Level g collects the pairs with t + u = g, 2 <= g <= s + 1 (the
   pairs beyond s + 1 are dropped, as in the cited scheme): I_g = sum P_tu,
   still an exact integer. Then D_ij = sum over g of 2^(e_i + f_j - beta g)
   I_g[i, j], added in float64 from the smallest level (g = s + 1) to the
   largest (g = 2).

Pins (tests/test_oracle_slices.py): the digits reproduce dyadic inputs
exactly and other inputs within 2^(e - beta s); level sums equal brute-force
integer sums; products of small integers come out exact; inputs of two
digits lose nothing but the final float64 roundings; products of random
inputs against exact rational arithmetic (fractions) stay within the error
bound of the dropped pairs and the digit remainders.
"""
from __future__ import annotations

import numpy as np

BETA = 7


def row_exponents(X: np.ndarray) -> np.ndarray:
    """e_i = smallest integer with max_j |x_ij| < 2^e_i (0 for a zero row)."""
    m = np.max(np.abs(np.asarray(X, dtype=np.float64)), axis=1)
    _, e = np.frexp(m)  # m = f 2^e with 0.5 <= f < 1, so m < 2^e and m >= 2^(e-1)
    return np.where(m > 0, e, 0).astype(np.int64)


def split_rows(X: np.ndarray, s: int, beta: int = BETA):
    """Digits (s, m, k) as int64 in [-(2^beta - 1), 2^beta - 1] and row exponents (m,)."""
    X = np.asarray(X, dtype=np.float64)
    e = row_exponents(X)
    y = np.ldexp(X, -e[:, None])
    digits = np.zeros((s,) + X.shape, dtype=np.int64)
    r = y
    for t in range(s):
        r = np.ldexp(r, beta)
        d = np.clip(np.rint(r), -(2 ** beta - 1), 2 ** beta - 1)
        digits[t] = d.astype(np.int64)
        r = r - d
    return digits, e


def join_rows(digits: np.ndarray, e: np.ndarray, beta: int = BETA) -> np.ndarray:
    """sum_t d_t 2^(e - beta t), summed from the last digit to the first."""
    s = digits.shape[0]
    out = np.zeros(digits.shape[1:], dtype=np.float64)
    for t in range(s, 0, -1):
        out = out + np.ldexp(digits[t - 1].astype(np.float64), e[:, None] - beta * t)
    return out


def level_sums(L: np.ndarray, R: np.ndarray, s: int, beta: int = BETA):
    """Exact integer level sums I_g (g = 2 .. s + 1) of D = L^T R, with the
    row exponents of L^T and R^T.

    The digit products go through a float64 matmul: every product of two
    digits is an integer below 2^(2 beta) and every partial sum over k stays
    an integer below k 2^(2 beta) < 2^53, so any summation order is exact.
    """
    a, el = split_rows(np.asarray(L, dtype=np.float64).T, s, beta)
    b, er = split_rows(np.asarray(R, dtype=np.float64).T, s, beta)
    k = a.shape[2]
    assert s * k * (2 ** beta - 1) ** 2 < 2 ** 53, "level sums would not stay exact"
    levels = {}
    for g in range(2, s + 2):
        acc = np.zeros((a.shape[1], b.shape[1]), dtype=np.float64)
        for t in range(1, g):
            u = g - t
            if u > s:
                continue
            acc = acc + a[t - 1].astype(np.float64) @ b[u - 1].astype(np.float64).T
        levels[g] = acc.astype(np.int64)
    return levels, el, er


def product(L: np.ndarray, R: np.ndarray, s: int = 8, beta: int = BETA) -> np.ndarray:
    """D = L^T R from s-digit slices (step 3 of the module docstring)."""
    levels, el, er = level_sums(L, R, s, beta)
    scale = el[:, None] + er[None, :]
    out = np.zeros(scale.shape, dtype=np.float64)
    for g in range(s + 1, 1, -1):
        out = out + np.ldexp(levels[g].astype(np.float64), scale - beta * g)
    return out


def error_bound(L: np.ndarray, R: np.ndarray, s: int = 8, beta: int = BETA) -> np.ndarray:
    """Bound on |product(L, R) - L^T R| elementwise.

    Per k, with x = 2^e (X' + 2^(-beta s) r) and y = 2^f (Y' + 2^(-beta s) q),
    |r|, |q| <= 1 and |X'|, |Y'| < 1 + 2^(-beta s), the kept pairs miss the
    pairs with t + u >= s + 2 (at most s - 1 of weight 2^(-beta s) each and
    fewer of smaller weight, every digit product below 2^(2 beta)) and the
    remainder terms (below 2.01 2^(-beta s)): together below
    (s + 2) 2^(e + f - beta s). Over k that is k (s + 2) 2^(e_i + f_j - beta s).
    The s float64 additions of the levels add at most s u times the sum of
    the levels' magnitudes (u = 2^-53), below s u (sum_k |l_ki| |r_kj| + the
    truncation term); the bound takes twice that.
    """
    L = np.asarray(L, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    k = L.shape[0]
    el = row_exponents(L.T)
    er = row_exponents(R.T)
    trunc = k * (s + 2) * np.ldexp(1.0, (el[:, None] + er[None, :]) - beta * s)
    rounding = 2.0 * s * 2.0 ** -53 * (np.abs(L).T @ np.abs(R) + trunc)
    return trunc + rounding
