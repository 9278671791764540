"""Writes iteration_counts.json: exact-arithmetic iteration counts of eq. (1)
for the seeded workloads, from the oracle's per-eigenvalue recursion.

Run from the repository root: python tests/golden/make_counts.py
Calls only the oracle and the seeded input generators.
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as w                       # noqa: E402
from oracle import iteration as it          # noqa: E402


def counts(lam, p, sigma, tol, a=None):
    """Counts from the scaled identity and from eq. (3); with the matrix given,
    also the power-scale start's scale (the oracle's repeated squaring, at
    most 6 squarings) and the count of the dynamically scaled iteration from
    it, both in exact arithmetic on the known spectrum."""
    out = {}
    for init in ("identity", "paper"):
        k, rho = it.spectral_count(lam, p, it.spectral_start(lam, p, init, sigma), tol, 400)
        out[init] = k
    if a is not None:
        s, sq = it.power_scale(a, p, 6, scaled_steps=True)
        k, _, mus = it.scaled_spectral_count(lam, p, s, tol)
        out["power_scale"] = {"scale": s, "squarings": sq}
        out["scaled"] = k
    return out


def main():
    rec = {}
    a, lam, _ = w.spd_log_spectrum(256, lam_range=(1e-2, 1.0), seed=0)
    sig = math.sqrt(it.norm_1(a) * it.norm_inf(a))
    rec["spd_n256_logU[1e-2,1]_seed0"] = {"sigma": sig, "tol": 1e-12,
                                          "p2": counts(lam, 2, sig, 1e-12)}
    a = w.kernel_matrix(4096, seed=0)
    lam = np.linalg.eigvalsh(a)
    sig = math.sqrt(it.norm_1(a) * it.norm_inf(a))
    rec["kernel_n4096_seed0"] = {"sigma": sig, "tol": 1e-10, "lam_min": float(lam[0]),
                                 "lam_max": float(lam[-1]),
                                 **{f"p{p}": counts(lam, p, sig, 1e-10, a) for p in (1, 2, 3)}}
    for kappa in (1e2, 1e4):
        a, lam = w.householder_spd(16384, kappa, seed=0)
        sig = math.sqrt(it.norm_1(a) * it.norm_inf(a))
        rec[f"householder_n16384_kappa{kappa:g}_seed0"] = {
            "sigma": sig, "tol": 1e-10, "p2": counts(lam, 2, sig, 1e-10, a)}
        del a
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "iteration_counts.json")
    with open(path, "w") as f:
        json.dump({"source": "oracle.iteration.spectral_count on workloads generators "
                             "(eq. (1) per eigenvalue; starts: scaled identity and eq. (3)); "
                             "scaled: oracle.iteration.scaled_spectral_count from the "
                             "oracle's power_scale",
                   "counts": rec}, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
