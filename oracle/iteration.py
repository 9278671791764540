"""FP64 oracle of the Bini-type iteration for A^{-1/p} (Section II, eqs. (1)-(3)).

Test infrastructure only (see the package docstring).

Notation follows Section II of the paper: A is symmetric positive definite,
C_k the k-th iterate, p >= 1 the root. The update is eq. (1),
    C_{k+1} = ((p + 1) C_k - C_k^{p+1} A) / p,
convergent when the start satisfies eq. (2), ||I - C_0^p A||_2 < 1; the paper's
start is eq. (3), C_0 = A^T / (||A||_1 ||A||_inf). For p = 1 the update is the
Newton-Schulz iteration for the inverse (Section II).

Readings of what the paper leaves open (each is listed in the design notes):
  * evaluation order of C_k^{p+1} A: the default is the coupled form that
    carries M_k = C_k^p A beside C_k, N_k = I + (I - M_k)/p,
    C_{k+1} = C_k N_k, M_{k+1} = N_k^p M_k. In exact arithmetic it gives the same
    iterates as eq. (1) (every factor is a polynomial in A, so they commute);
    the literal right-multiplied order is kept as a diagnostic.
  * start: eq. (3) ("paper"), or the scaled identity
    C_0 = (||A||_1 ||A||_inf)^{-1/(2p)} I ("identity"), whose C_0^p A has its
    spectrum in (0, 1] for every SPD A, so eq. (2) always holds.
  * stopping: the Frobenius norm of I - M_k below tol, confirmed by the
    directly computed ||I - C_k^p A||_F below tol.
  * every iterate is symmetrised, X <- (X + X^T)/2.
  * precision floor: reported once the residual, below 1/2, has not halved
    its best value for floor_window iterations (below 1/2 every exact step
    at least halves it: ``step_contraction``).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

OK, EMAXITER, EFLOOR, EDIVERGED = 0, 2, 3, 4

# Residual below which a step that fails to halve it can only be rounding
# (see ``solve``)
FLOOR_ZONE = 0.5


def step_contraction(p: int, emax: float = 0.5, samples: int = 200001) -> float:
    """max |1 - g(1 - e)| / |e| over 0 < |e| <= emax, g the coupled form's
    eigenvalue map m -> m ((p + 1 - m) / p)^p (a dense sample of e)."""
    e = np.linspace(-emax, emax, samples)
    e = e[e != 0.0]
    m = 1.0 - e
    return float(np.max(np.abs(1.0 - m * ((p + 1 - m) / p) ** p) / np.abs(e)))


def norm_1(a: np.ndarray) -> float:
    """||A||_1: the largest column sum of absolute values (eq. (3))."""
    return float(np.max(np.sum(np.abs(a), axis=0)))


def norm_inf(a: np.ndarray) -> float:
    """||A||_inf: the largest row sum of absolute values (eq. (3))."""
    return float(np.max(np.sum(np.abs(a), axis=1)))


def sym(x: np.ndarray) -> np.ndarray:
    return 0.5 * (x + x.T)


def start_paper(a: np.ndarray, p: int) -> np.ndarray:
    """Eq. (3): C_0 = A^T / (||A||_1 ||A||_inf)."""
    return a.T / (norm_1(a) * norm_inf(a))


def start_identity(a: np.ndarray, p: int) -> np.ndarray:
    """Scaled identity C_0 = c I with c^p = (||A||_1 ||A||_inf)^{-1/2}.

    ||A||_2 <= sqrt(||A||_1 ||A||_inf), so the eigenvalues of C_0^p A lie in
    (0, 1] and eq. (2) holds for every SPD A."""
    s = norm_1(a) * norm_inf(a)
    return s ** (-1.0 / (2 * p)) * np.eye(a.shape[0])


def power_scale(a: np.ndarray, p: int, max_squarings: int, scaled_steps: bool = False):
    """Scale s >= lambda_max(A) of the scaled-identity start from repeated
    squaring (a reading that extends eq. (3)'s norm bound, not the paper's):
    with sigma = sqrt(||A||_1 ||A||_inf) and S_k = (A / sigma)^(2^k),
    b_k = 1.01 sigma (||S_k||_1 ||S_k||_inf)^(1 / 2^(k+1)) bounds lambda_max
    (1% margin for rounding). Squaring stops after max_squarings, or once the
    next squaring is predicted (square root of the last improvement b_{k-1}/b_k)
    to improve the bound by less than what one product buys in the slow phase:
    w = ((1 + 1/p)^p c)^(1/(p+1)), c = mu_cap(p) with scaled steps, else 1.
    Returns (s, squarings done) with s = min(sigma, b_1, ...)."""
    sigma = np.sqrt(norm_1(a) * norm_inf(a))
    grow = (1.0 + 1.0 / p) ** p * (mu_cap(p) if scaled_steps else 1.0)
    worth = grow ** (1.0 / (p + 1.0))
    best = prev = sigma
    s_k = a / sigma
    k = 0
    for k in range(1, max_squarings + 1):
        s_k = s_k @ s_k
        b = 1.01 * sigma * (norm_1(s_k) * norm_inf(s_k)) ** (1.0 / 2 ** (k + 1))
        if not (b > 0.0) or not np.isfinite(b):
            k -= 1
            break
        best = min(best, b)
        if np.sqrt(prev / b) < worth:
            break
        prev = b
    return best, k


def step_map(m, p: int):
    """One coupled step on an eigenvalue m of M: g(m) = m ((p + 1 - m) / p)^p
    (the eigenvalue c^p lam of eq. (1)'s scalar recursion, c <- c (p + 1 - m) / p)."""
    return m * ((p + 1.0 - m) / p) ** p


def mu_cap(p: int) -> float:
    """Largest scaled top of the spectrum: 1.98 (< 2, eq. (2)); for p = 1 the
    m with g(m) = m (2 - m) = 1/2, 1 + 1/sqrt(2), so that the step does not
    push top eigenvalues near 0 (for p >= 2, g(2) >= 1/2)."""
    return 1.0 + np.sqrt(0.5) if p == 1 else 1.98


def scaled_step_factor(m: np.ndarray, p: int) -> float:
    """Scale factor mu of one dynamically scaled step (a reading beyond the
    paper), from the eigenvalues m of M_k: the step maps each eigenvalue m_i to
    g(mu m_i), and mu is the value in [1, mu_cap(p) / max m] for which the
    smallest of them after the step is largest; mu = 1 (plain step) once
    min m >= 1/2, where the iteration is already quadratic.

    Found by brute force: min_i g(mu m_i) on a grid of 100001 values of mu,
    then on a grid of 2001 values between the best point's neighbours. Since g
    rises up to its peak at 1 and falls after it, min_i g(mu m_i) is the
    smaller of the values at the two ends of the spectrum."""
    m = np.asarray(m, dtype=np.float64)
    lo, top = float(m.min()), float(m.max())
    if not (lo > 0.0) or lo >= 0.5:
        return 1.0
    hi = mu_cap(p) / top
    if hi <= 1.0:
        return 1.0

    def lower_end(mu):
        return np.minimum(step_map(mu * lo, p), step_map(mu * top, p))

    grid = np.linspace(1.0, hi, 100001)
    j = int(np.argmax(lower_end(grid)))
    fine = np.linspace(grid[max(j - 1, 0)], grid[min(j + 1, grid.size - 1)], 2001)
    return float(fine[int(np.argmax(lower_end(fine)))])


def start_poly(a: np.ndarray, p: int, b) -> np.ndarray:
    """Polynomial start C_0 = sigma^{-1/p} (b0 I + b1 A/sigma + b2 (A/sigma)^2),
    sigma = sqrt(||A||_1 ||A||_inf). b = (1, 0, 0) is the scaled identity."""
    sigma = np.sqrt(norm_1(a) * norm_inf(a))
    ah = a / sigma
    n = a.shape[0]
    q = b[0] * np.eye(n) + b[1] * ah + b[2] * (ah @ ah)
    return sigma ** (-1.0 / p) * sym(q)


def matpow(x: np.ndarray, p: int) -> np.ndarray:
    out = x
    for _ in range(p - 1):
        out = out @ x
    return out


def true_residual(c: np.ndarray, a: np.ndarray, p: int) -> float:
    """||I - C^p A||_F, computed from C and A directly."""
    n = a.shape[0]
    return float(np.linalg.norm(np.eye(n) - matpow(c, p) @ a))


def eig_root(a: np.ndarray, p: int) -> np.ndarray:
    """A^{-1/p} by definition: A = V diag(lam) V^T -> V diag(lam^{-1/p}) V^T."""
    lam, v = np.linalg.eigh(a)
    if np.any(lam <= 0):
        raise ValueError("matrix is not positive definite")
    return sym((v * lam ** (-1.0 / p)) @ v.T)


def householder_root(n: int, kappa: float, seed: int, p: int) -> np.ndarray:
    """A^{-1/p} by definition for the ``workloads.householder_spd`` matrix of the
    same arguments: its eigenvectors are H's columns and its eigenvalues are
    known, so A^{-1/p} = H diag(lam^{-1/p}) H^T (built in O(n^2 k))."""
    import workloads
    lam, vmat, t = workloads.householder_factors(n, kappa, seed)
    return workloads.householder_congruence(vmat, t, lam ** (-1.0 / p))


def rel_fro(x: np.ndarray, ref: np.ndarray) -> float:
    """Relative Frobenius error ||X - ref||_F / ||ref||_F (the paper's metric of
    Section IV-C made relative)."""
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


@dataclass
class Result:
    c: np.ndarray
    status: int
    iters: int
    rho: list = field(default_factory=list)     # ||I - M_k||_F per iteration
    residual_true: float = float("nan")


def _make_start(a, p, init, poly):
    if isinstance(init, np.ndarray):
        return init.copy()
    if init == "paper":
        return start_paper(a, p)
    if init == "identity":
        return start_identity(a, p)
    if init == "poly":
        return start_poly(a, p, poly)
    raise ValueError(f"unknown start {init!r}")


def solve(a: np.ndarray, p: int, tol: float, init="identity", max_iter: int = 100,
          evaluation: str = "coupled", poly=(1.0, 0.0, 0.0),
          floor_window: int = 3, scaled=None) -> Result:
    """Run the iteration of eq. (1) until ||I - C^p A||_F < tol.

    evaluation:
      "coupled"        M_0 = C_0^p A; R = I - M; N = I + R/p; C <- C N;
                       M <- N (N (... (N M))) (p products); both symmetrised.
      "literal"        X = C^p A; C <- ((p + 1) C - C X) / p (eq. (1) as printed).
      "newton_schulz"  p = 1 only: C <- C (2I - A C), symmetrised (Section II).

    scaled=s: the dynamically scaled coupled iteration (a reading beyond the
    paper) from C_0 = s^{-1/p} q(A/s), s >= lambda_max(A), with
    q(x) = b0 + b1 x + b2 x^2 given by ``poly`` when init="poly" and q = 1
    (the scaled identity) otherwise. Step k uses N = ((p + 1) I - mu_k M)/p,
    C <- mu_k^{1/p} C N, M <- N^p mu_k M, with mu_k = scaled_step_factor of
    the eigenvalues of M_k. Those eigenvalues are followed exactly: M_0 has
    q(x)^p x at x = lambda / s (lambda from numpy's eigvalsh of A), and each
    step maps them by g(mu_k m) (M_k is a polynomial in A).

    The returned iteration count is the number of updates applied. Status:
    OK; EMAXITER after max_iter updates; EDIVERGED on a NaN or a residual above
    1e6; EFLOOR when, once below 1/2, the residual has not fallen below half
    its best value for ``floor_window`` consecutive iterations. Below 1/2 every
    eigenvalue error e of M_k has |e| <= 1/2, and one exact step maps it to at
    most |e|/2 (``step_contraction``), so only rounding can keep the residual
    from halving; between 1/2 and 1 a single small eigenvalue still in its slow
    phase can hold the residual nearly flat for many steps.
    """
    if not np.array_equal(a, a.T):
        raise ValueError("A must be exactly symmetric")
    if p < 1:
        raise ValueError("p must be >= 1")
    if evaluation == "newton_schulz" and p != 1:
        raise ValueError("Newton-Schulz order is the p = 1 case")
    n = a.shape[0]
    eye = np.eye(n)
    if scaled is not None:
        if evaluation != "coupled":
            raise ValueError("the scaled iteration is a coupled form")
        s = float(scaled)
        b = poly if init == "poly" else (1.0, 0.0, 0.0)
        ah = a / s
        c = s ** (-1.0 / p) * sym(b[0] * np.eye(n) + b[1] * ah + b[2] * (ah @ ah))
        x = np.linalg.eigvalsh(a) / s
        m_eig = (b[0] + b[1] * x + b[2] * x * x) ** p * x
    else:
        c = _make_start(a, p, init, poly)
    m = matpow(c, p) @ a if evaluation == "coupled" else None
    rhos = []
    best = np.inf
    stale = 0
    for k in range(max_iter + 1):
        if evaluation == "coupled":
            r = eye - m
        elif evaluation == "literal":
            x = matpow(c, p) @ a
            r = eye - x
        else:
            x = a @ c
            r = eye - x
        rho = float(np.linalg.norm(r))
        rhos.append(rho)
        if not np.isfinite(rho) or rho > 1e6:
            return Result(c, EDIVERGED, k, rhos)
        if rho < tol:
            tau = true_residual(c, a, p)
            if tau < tol:
                return Result(c, OK, k, rhos, tau)
        if rho < FLOOR_ZONE:
            if rho < 0.5 * best:
                best = rho
                stale = 0
            else:
                stale += 1
                if stale >= floor_window:
                    return Result(c, EFLOOR, k, rhos, true_residual(c, a, p))
        if k == max_iter:
            break
        if evaluation == "coupled" and scaled is not None:
            mu = scaled_step_factor(m_eig, p)
            nmat = ((p + 1) * eye - mu * m) / p
            c = sym(mu ** (1.0 / p) * (c @ nmat))
            m = mu * m
            for _ in range(p):
                m = nmat @ m
            m = sym(m)
            m_eig = step_map(mu * m_eig, p)
        elif evaluation == "coupled":
            nmat = eye + r / p
            c = sym(c @ nmat)
            for _ in range(p):
                m = nmat @ m
            m = sym(m)
        elif evaluation == "literal":
            c = ((p + 1) * c - c @ x) / p
        else:
            c = sym(c @ (2.0 * eye - x))
    return Result(c, EMAXITER, max_iter, rhos, true_residual(c, a, p))


def scalar_step(c, lam, p):
    """Eq. (1) on one eigenvalue: c <- c (p + 1 - c^p lam) / p."""
    return c * (p + 1 - c ** p * lam) / p


def spectral_count(lam: np.ndarray, p: int, c0: np.ndarray, tol: float,
                   max_iter: int = 200):
    """Iteration count and residual trajectory of eq. (1) in exact arithmetic,
    computed per eigenvalue: for A = V diag(lam) V^T and C_0 = V diag(c0) V^T the
    iterates stay V diag(c_k) V^T, so ||I - C_k^p A||_F = sqrt(sum (1 - c^p lam)^2).

    Returns (count, rho_list); count = max_iter + 1 when tol is not reached."""
    c = np.asarray(c0, dtype=np.float64).copy()
    rhos = []
    for k in range(max_iter + 1):
        rho = float(np.sqrt(np.sum((1.0 - c ** p * lam) ** 2)))
        rhos.append(rho)
        if rho < tol:
            return k, rhos
        if not np.isfinite(rho) or rho > 1e6:
            return max_iter + 1, rhos
        c = scalar_step(c, lam, p)
    return max_iter + 1, rhos


def scaled_spectral_count(lam: np.ndarray, p: int, s: float, tol: float,
                          max_iter: int = 200, poly=(1.0, 0.0, 0.0)):
    """Iteration count and residual trajectory of the dynamically scaled
    iteration (``solve(scaled=s)``) in exact arithmetic, per eigenvalue: from
    C_0 = s^{-1/p} q(A/s) the eigenvalues of M_0 are q(x)^p x at x = lam / s
    (q = 1: lam / s), and step k maps them by m <- g(mu_k m) with
    mu_k = scaled_step_factor(m). The residual is ||I - M_k||_F =
    sqrt(sum (1 - m)^2). Returns (count, rho_list, mu_list); count =
    max_iter + 1 when tol is not reached."""
    x = np.asarray(lam, dtype=np.float64) / float(s)
    m = (poly[0] + poly[1] * x + poly[2] * x * x) ** p * x
    rhos, mus = [], []
    for k in range(max_iter + 1):
        rho = float(np.sqrt(np.sum((1.0 - m) ** 2)))
        rhos.append(rho)
        if rho < tol:
            return k, rhos, mus
        if not np.isfinite(rho) or rho > 1e6:
            break
        mu = scaled_step_factor(m, p)
        mus.append(mu)
        m = step_map(mu * m, p)
    return max_iter + 1, rhos, mus


def spectral_start(lam: np.ndarray, p: int, init: str, sigma: float,
                   poly=(1.0, 0.0, 0.0)) -> np.ndarray:
    """Eigenvalues of C_0 for the starts above, given sigma = sqrt(||A||_1 ||A||_inf)
    (for symmetric A, ||A||_1 = ||A||_inf, so sigma^2 = ||A||_1 ||A||_inf)."""
    if init == "paper":
        return lam / sigma ** 2
    if init == "identity":
        return np.full_like(lam, sigma ** (-1.0 / p))
    if init == "poly":
        x = lam / sigma
        return sigma ** (-1.0 / p) * (poly[0] + poly[1] * x + poly[2] * x * x)
    raise ValueError(init)


def commutator(c: np.ndarray, a: np.ndarray) -> float:
    """||CA - AC||_F / (||C||_F ||A||_F); zero for any function of A."""
    return float(np.linalg.norm(c @ a - a @ c) / (np.linalg.norm(c) * np.linalg.norm(a)))


def residual_map(r: np.ndarray, p: int) -> np.ndarray:
    """Per-eigenvalue residual law of the coupled step: r = 1 - c^p lam maps to
    1 - (1 - r)(1 + r/p)^p (the scalar form of M_{k+1} = N^p M)."""
    return 1.0 - (1.0 - r) * (1.0 + r / p) ** p
