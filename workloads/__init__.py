"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module builds input matrices only. It contains none of the inverse p-th
root method's arithmetic: no norms of the method, no initial guesses, no
iteration. Every generator draws from ``numpy.random.default_rng(seed)`` in the
order written in its docstring, so a (recipe, seed) pair names one matrix.

The paper evaluates on overlap matrices of water systems (Section IV-A), which
are not available here. The recipes below stand in for them:

* ``spd_log_spectrum``: A = Q diag(lam) Q^T with a Haar orthogonal Q and a
  log-uniform spectrum (dense, no structure; the general case).
* ``kernel_matrix``: a Gaussian-kernel Gram matrix of random points in a 3-D box,
  A_ij = exp(-|x_i - x_j|^2 / (2 l^2)) + shift * delta_ij. Its entries decay
  with distance like an overlap matrix S_ij = <phi_i|phi_j> of localized basis
  functions (the "nearsightedness" the paper describes in Section IV-A).
* ``householder_spd``: A = H diag(lam) H^T with H a product of k Householder
  reflectors, for sizes where a Haar Q is too costly to draw (n = 16384).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar_orthogonal", "log_spectrum", "spd_from_spectrum", "spd_log_spectrum",
    "kernel_matrix", "householder_spd", "batch_recipe", "training_recipe",
    "diagonal_spd",
]


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal n x n matrix: QR of a Gaussian matrix with the
    columns' signs fixed by sign(diag(R)). Draws n*n normals."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def log_spectrum(n: int, kappa: float, rng: np.random.Generator,
                 pin_ends: bool = True) -> np.ndarray:
    """n eigenvalues log-uniform on [1/kappa, 1]. With ``pin_ends`` the first is
    exactly 1/kappa and the second exactly 1, so the condition number is kappa
    exactly. Draws n uniforms."""
    lam = np.exp(rng.uniform(np.log(1.0 / kappa), 0.0, n))
    if pin_ends and n >= 2:
        lam[0] = 1.0 / kappa
        lam[1] = 1.0
    elif pin_ends and n == 1:
        lam[0] = 1.0
    return lam


def spd_from_spectrum(q: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """A = Q diag(lam) Q^T, made exactly symmetric by averaging with its transpose."""
    a = (q * lam) @ q.T
    return 0.5 * (a + a.T)


def spd_log_spectrum(n: int, kappa: float | None = None, seed: int = 0,
                     lam_range: tuple[float, float] | None = None):
    """Dense SPD matrix A = Q diag(lam) Q^T with Haar Q.

    Draw order: Q (n*n normals), then lam (n uniforms). Either ``kappa`` (endpoints
    pinned to 1/kappa and 1) or ``lam_range=(lo, hi)`` (log-uniform, endpoints not
    pinned) is given. Returns (A, lam, Q).
    """
    rng = np.random.default_rng(seed)
    q = haar_orthogonal(n, rng)
    if lam_range is not None:
        lo, hi = lam_range
        lam = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    else:
        lam = log_spectrum(n, float(kappa), rng, pin_ends=True)
    return spd_from_spectrum(q, lam), lam, q


def diagonal_spd(n: int, kappa: float, seed: int = 0) -> np.ndarray:
    """Diagonal SPD matrix with a log-uniform spectrum (endpoints pinned)."""
    rng = np.random.default_rng(seed)
    return np.diag(log_spectrum(n, kappa, rng))


def kernel_matrix(n: int = 4096, seed: int = 0, box: float = 20.0,
                  length: float = 1.0, shift: float = 1e-3) -> np.ndarray:
    """Gaussian-kernel Gram matrix of n points uniform in [0, box]^3, plus
    ``shift`` on the diagonal. Draw order: the n*3 point coordinates."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, box, (n, 3))
    sq = np.sum(x * x, axis=1)
    d2 = sq[:, None] + sq[None, :] - 2.0 * (x @ x.T)
    np.maximum(d2, 0.0, out=d2)
    np.fill_diagonal(d2, 0.0)
    a = np.exp(-d2 / (2.0 * length * length))
    a += shift * np.eye(n)
    return 0.5 * (a + a.T)


def overlap_and_hamiltonian(n: int = 1024, seed: int = 0, box: float = 20.0,
                            shift: float = 1e-3):
    """(S, H) for n s-type Gaussians (exponent 1/2, unit length) at points
    uniform in [0, box]^3: S = kernel_matrix(n, seed, box, 1, shift), and a
    Hamiltonian-like H with the same decay: the kinetic-energy form of
    Gaussians, S_ij (3 - d_ij^2 / 2) / 4, plus a potential -exp(-|x_i - c|^2 / 50)
    on the diagonal (c the box centre). Same draw order as kernel_matrix (the
    points); H is exactly symmetric."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, box, (n, 3))
    sq = np.sum(x * x, axis=1)
    d2 = sq[:, None] + sq[None, :] - 2.0 * (x @ x.T)
    np.maximum(d2, 0.0, out=d2)
    np.fill_diagonal(d2, 0.0)
    d2 = 0.5 * (d2 + d2.T)
    g = np.exp(-d2 / 2.0)
    s = g + shift * np.eye(n)
    h = g * (3.0 - d2 / 2.0) / 4.0
    c = np.full(3, box / 2.0)
    h -= np.diag(np.exp(-np.sum((x - c) ** 2, axis=1) / 50.0))
    return 0.5 * (s + s.T), 0.5 * (h + h.T)


def householder_factors(n: int, kappa: float, seed: int = 0, nrefl: int = 64):
    """Spectrum and compact-WY form of H = H_1 H_2 ... H_k, H_i = I - 2 v_i v_i^T / |v_i|^2.

    Draw order: lam (n uniforms, endpoints pinned to 1/kappa and 1), then the k
    Gaussian vectors v_i (k*n normals). Returns (lam, V, T) with H = I - V T V^T,
    V n x k with unit columns and T k x k upper triangular."""
    rng = np.random.default_rng(seed)
    lam = log_spectrum(n, kappa, rng, pin_ends=True)
    v = rng.standard_normal((nrefl, n))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    vmat = v.T
    t = np.zeros((nrefl, nrefl))
    for j in range(nrefl):
        t[j, j] = 2.0
        if j:
            t[:j, j] = -2.0 * t[:j, :j] @ (vmat[:, :j].T @ vmat[:, j])
    return lam, vmat, t


def householder_congruence(vmat: np.ndarray, t: np.ndarray, d: np.ndarray) -> np.ndarray:
    """H diag(d) H^T for H = I - V T V^T in O(n^2 k): with W = V T V^T,
    (I - W) D (I - W)^T = D - W D - D W^T + W D W^T. Exactly symmetric."""
    n = vmat.shape[0]
    vd = vmat.T * d                                 # k x n  = V^T D
    wd = vmat @ (t @ vd)                            # n x n  = W D
    k_small = vd @ vmat                             # k x k  = V^T D V
    a = vmat @ (t @ k_small @ t.T) @ vmat.T         # n x n  = W D W^T
    a -= wd
    a -= wd.T
    a[np.diag_indices(n)] += d
    return 0.5 * (a + a.T)


def householder_spd(n: int, kappa: float, seed: int = 0, nrefl: int = 64):
    """A = H diag(lam) H^T with H a product of ``nrefl`` Householder reflectors
    (see ``householder_factors`` for the draw order). Building A costs O(n^2 k)
    instead of O(n^3). Returns (A, lam)."""
    lam, vmat, t = householder_factors(n, kappa, seed, nrefl)
    return householder_congruence(vmat, t, lam), lam


def batch_recipe(count: int = 2000, base_seed: int = 1000,
                 n_range=(32, 512), p_choices=(1, 2, 4),
                 kappa_range=(10.0, 1e5)):
    """Descriptors of a batch of independent SPD problems, one per seed
    base_seed + i. Draw order per item: n, p, kappa, then Q and lam as in
    ``spd_log_spectrum``. Returns a list of (n, p, kappa, seed)."""
    items = []
    for i in range(count):
        s = base_seed + i
        rng = np.random.default_rng(s)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(p_choices[int(rng.integers(0, len(p_choices)))])
        kappa = float(np.exp(rng.uniform(np.log(kappa_range[0]), np.log(kappa_range[1]))))
        items.append((n, p, kappa, s))
    return items


def batch_matrix(n: int, kappa: float, seed: int):
    """The matrix of one ``batch_recipe`` item: the generator of that seed is
    advanced past the three descriptor draws, then Q and lam are drawn."""
    rng = np.random.default_rng(seed)
    rng.integers(0, 2)          # n
    rng.integers(0, 2)          # p index
    rng.uniform(0.0, 1.0)       # kappa
    q = haar_orthogonal(n, rng)
    lam = log_spectrum(n, kappa, rng, pin_ends=True)
    return spd_from_spectrum(q, lam), lam


def training_recipe(count: int, base_seed: int, n_range=(64, 1024),
                    p_range=(1, 4), kappa_range=(10.0, 1e6)):
    """Descriptors for the learned-initial-guess data set: one seed per item,
    (n, p, kappa, seed) drawn as in ``batch_recipe``."""
    return batch_recipe(count, base_seed, n_range,
                        tuple(range(p_range[0], p_range[1] + 1)), kappa_range)
