"""Training and evaluation of the learned start (weights: start_mlp.npz).

    python -m paper_1703_02283_amd.train_start --train 200000 --heldout 10000 \
        --hh-train 40000 --hh-heldout 2000

or in parts: --build SET:START:STOP:FILE writes the features and labels of
part of one set, and --shards FILE... trains and evaluates from such parts.

The start C_0 = s^{-1/p} q(A/s), q(x) = b0 + b1 x + b2 x^2, is expressed in
units of the certified bound s = (||A^2||_1 ||A^2||_inf)^{1/4} >= lambda_max,
so the spectrum of A/s lies in (0, 1] and eq. (2) is checked on that interval.
The network (16 -> 64 -> 64 -> 3, GELU) maps ipr_features(A) to
(log b0, b1, b2).

Data: SPD matrices A = Q diag(lam) Q^T with Haar Q, n ~ U{64..1024},
p ~ U{1..4}, kappa log-uniform in [10, 1e6] (seeds 1e6 + i for training,
2e6 + i held out), plus matrices of the same draws whose eigenvectors are a
product of 4, 16 or 64 Householder reflectors (seeds 3e6 + i and 4e6 + i):
near-diagonal matrices, whose features the Haar set never shows and which
large problems (the n = 16384 workload) resemble. The matrices are drawn on
the GPU with torch (QR of Gaussian matrices or reflector updates, grouped by
order); features, labels, training and inference all run in libipr's
kernels:
  * labels: for every matrix, ipr_spectral_counts gives the exact-arithmetic
    iteration count of the method itself for each candidate start; the label
    is the candidate with the fewest matrix products in total (the scale
    bound's product, p more when q is not constant, p + 1 per iteration);
  * training: ipr_mlp_train_step (forward, backward, Adam on the GPU).
Feature standardisation is folded into the first layer after training, so the
stored network reads raw features.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import binding as ipr

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "start_mlp.npz")
NPARAM = ipr.IPR_MLP_NPARAM
TOL = 1e-10
MAXIT = 200


def log(*a):
    print("[train_start]", *a, file=sys.stderr, flush=True)


def recipe(count, base_seed, n_range=(64, 1024), p_range=(1, 4), kappa_range=(10.0, 1e6),
           reflectors=0):
    """(n, p, kappa, seed, reflectors) per item; the first four are the same
    draws as workloads.training_recipe. reflectors = 0: Haar eigenvectors;
    otherwise the eigenvectors are a product of that many Householder
    reflectors (4, 16 or 64, drawn per item when `reflectors` is "mix")."""
    out = []
    for i in range(count):
        s = base_seed + i
        rng = np.random.default_rng(s)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(p_range[0] + int(rng.integers(0, p_range[1] - p_range[0] + 1)))
        kappa = float(np.exp(rng.uniform(np.log(kappa_range[0]), np.log(kappa_range[1]))))
        k = int((4, 16, 64)[int(rng.integers(0, 3))]) if reflectors == "mix" else int(reflectors)
        out.append((n, p, kappa, s, k))
    return out


def spectrum(n, kappa, seed):
    """lam log-uniform on [1/kappa, 1], both ends pinned (host, seeded)."""
    rng = np.random.default_rng(seed + 7_919)
    lam = np.exp(rng.uniform(np.log(1.0 / kappa), 0.0, n))
    if n >= 2:
        lam[0], lam[1] = 1.0 / kappa, 1.0
    return lam


def make_group(items, device):
    """Matrices of one order n (and one eigenvector family): Haar Q by QR of
    seeded Gaussians (batched on the GPU), A = Q diag(lam) Q^T symmetrised; or,
    for items with k > 0 reflectors, A = H diag(lam) H^T with H a product of k
    Householder reflectors of seeded Gaussian directions (diagonal plus a
    rank-2k part: the shape of large matrices such as the n = 16384 workload).
    Returns (A [b, n, n], lam list)."""
    n = items[0][0]
    if items[0][4] > 0:
        return make_group_householder(items, device)
    gen = torch.Generator(device=device)
    gen.manual_seed(items[0][3])
    g = torch.randn((len(items), n, n), dtype=torch.float64, device=device, generator=gen)
    # Q of G = Q R with diag(R) > 0 (the Haar draw): Q = G R^{-1} with R^T R =
    # G^T G (Cholesky), done twice so that Q is orthogonal to rounding
    # (Cholesky QR; the same Q as a Householder QR with the signs fixed, which
    # batched on the GPU is an order of magnitude slower)
    q = g
    for _ in range(2):
        low = torch.linalg.cholesky(q.transpose(-1, -2) @ q)
        # (the batched triangular solve runs out of library workspace on
        # large batches: eight matrices per call)
        qt = q.transpose(-1, -2).contiguous()
        for s0 in range(0, len(items), 8):
            qt[s0:s0 + 8] = torch.linalg.solve_triangular(low[s0:s0 + 8], qt[s0:s0 + 8],
                                                          upper=False)
        q = qt.transpose(-1, -2)
    lams = [spectrum(n, kappa, seed) for (_, _, kappa, seed, _) in items]
    lam_t = torch.tensor(np.stack(lams), dtype=torch.float64, device=device)
    a = (q * lam_t.unsqueeze(-2)) @ q.transpose(-1, -2).contiguous()
    a = 0.5 * (a + a.transpose(-1, -2))
    return a.contiguous(), lams


def make_group_householder(items, device):
    n, k = items[0][0], items[0][4]
    gen = torch.Generator(device=device)
    gen.manual_seed(items[0][3])
    lams = [spectrum(n, kappa, seed) for (_, _, kappa, seed, _) in items]
    lam_t = torch.tensor(np.stack(lams), dtype=torch.float64, device=device)
    a = torch.diag_embed(lam_t)
    v = torch.randn((len(items), n, k), dtype=torch.float64, device=device, generator=gen)
    v = v / torch.linalg.vector_norm(v, dim=1, keepdim=True)
    for j in range(k):   # A <- (I - 2 v v^T) A (I - 2 v v^T)
        x = v[:, :, j]
        ax = torch.bmm(a, x.unsqueeze(-1)).squeeze(-1)
        xax = (x * ax).sum(-1, keepdim=True)
        a = (a - 2.0 * x.unsqueeze(-1) * ax.unsqueeze(-2) - 2.0 * ax.unsqueeze(-1) * x.unsqueeze(-2)
             + 4.0 * xax.unsqueeze(-1) * x.unsqueeze(-1) * x.unsqueeze(-2))
    a = 0.5 * (a + a.transpose(-1, -2))
    return a.contiguous(), lams


def guard_ok(b, p):
    """0 < q(x) and q(x)^p x < 2 on (0, 1] (eq. (2) for the spectrum in (0, 1])."""
    x = np.linspace(0.0, 1.0, 4001)[1:]
    q = b[0] + b[1] * x + b[2] * x * x
    return bool(np.all(q > 0) and np.all(q ** p * x < 2.0 * (1 - 1e-6)))


def candidates(p):
    """Candidate starts of the label search, all satisfying eq. (2) on (0, 1]:
    constant, linear and quadratic q (a quadratic term costs the solver no
    more than a linear one: A^2 is formed for the scale anyway, and either
    needs the p products of M_0)."""
    out = []
    for b0 in np.geomspace(0.5, 2.0 ** (1.0 / p) * 0.999, 28):
        out.append((b0, 0.0, 0.0))
        for t in (0.25, 0.5, 0.75):
            out.append((b0, -t * b0, 0.0))
        for t in (0.5, 0.75, 1.0):
            for u in (0.15, 0.3):
                out.append((b0, -t * b0, u * b0))
    return np.array([c for c in out if guard_ok(c, p)])


def build_dataset(items, device, chunk=256):
    """Features (float32), scales, labels (log b0, b1, b2) and the identity
    start's iteration count for every item."""
    order = {}
    for k, it in enumerate(items):
        order.setdefault((it[0], it[4]), []).append(k)
    m = len(items)
    feats = np.zeros((m, 16), np.float32)
    labels = np.zeros((m, 3), np.float32)
    scales = np.zeros(m)
    sigmas = np.zeros(m)
    best_products = np.zeros(m)
    ident_products = np.zeros(m)
    cands = {p: candidates(p) for p in (1, 2, 3, 4)}
    t0 = time.time()
    done = 0
    phase = {"matrices": 0.0, "features": 0.0, "scales": 0.0, "labels": 0.0}
    ws_norms = torch.empty(8 * (1024 * (1024 // 256 + 4) + 64), dtype=torch.uint8, device=device)
    g_buf = None

    def tick(name, t):
        torch.cuda.synchronize()
        now = time.time()
        phase[name] += now - t
        return now
    for (n, _), idx in sorted(order.items()):
        # (batched triangular solves of large orders run out of library
        # workspace beyond a few hundred MB per call)
        step = max(16, min(chunk, (1 << 25) // (n * n)))
        for c0 in range(0, len(idx), step):
            sel = idx[c0:c0 + step]
            its = [items[k] for k in sel]
            t = time.time()
            a, lams = make_group(its, device)
            t = tick("matrices", t)
            b = len(its)
            flat = a.reshape(-1)
            offs = [j * n * n for j in range(b)]
            ns = [n] * b
            ps = [it[1] for it in its]
            f = ipr.ipr_features(flat, offs, ns, ps)
            feats[sel] = f.cpu().numpy()
            t = tick("features", t)
            # certified scale and the norm scale, by the library's kernels (the
            # solver's own norms and FP64 product)
            sig = np.zeros(b)
            bound = np.zeros(b)
            if g_buf is None or g_buf.shape[0] != n:
                g_buf = torch.empty((n, n), dtype=torch.float64, device=device)
            for j in range(b):
                n1, ni = ipr.ipr_norms(a[j], workspace=ws_norms)
                ipr.ipr_gemm(a[j], a[j], triangle=True, out=g_buf)
                g1, gi = ipr.ipr_norms(g_buf, workspace=ws_norms)
                sig[j] = math.sqrt(n1 * ni)
                bound[j] = math.sqrt(math.sqrt(g1 * gi)) * (1 + 8 * n * 2.0 ** -52)
            sc = np.minimum(sig, bound)
            scales[sel] = sc
            sigmas[sel] = sig
            t = tick("scales", t)
            lam_flat = torch.tensor(np.concatenate(lams), dtype=torch.float64, device=device)
            loffs = [j * n for j in range(b)]
            for pv in sorted(set(ps)):
                sub = [j for j in range(b) if ps[j] == pv]
                cc = cands[pv]
                cnt = ipr.ipr_spectral_counts(
                    lam_flat, [loffs[j] for j in sub], [n] * len(sub), [pv] * len(sub),
                    [sc[j] for j in sub], cc, TOL, MAXIT)
                extra = np.where((cc[:, 1] != 0) | (cc[:, 2] != 0), pv, 0)
                cost = 1 + extra[None, :] + (pv + 1) * cnt
                k = np.argmin(cost, axis=1)
                ident = ipr.ipr_spectral_counts(
                    lam_flat, [loffs[j] for j in sub], [n] * len(sub), [pv] * len(sub),
                    [sig[j] for j in sub], np.array([[1.0, 0.0, 0.0]]), TOL, MAXIT)[:, 0]
                for r, j in enumerate(sub):
                    gj = sel[j]
                    bb = cc[k[r]]
                    labels[gj] = (math.log(bb[0]), bb[1], bb[2])
                    best_products[gj] = cost[r, k[r]]
                    ident_products[gj] = (pv + 1) * ident[r]
            tick("labels", t)
            done += b
            del a
        log(f"n={n}: {done}/{m} items, {time.time() - t0:.0f} s, phases "
            + ", ".join(f"{k} {v:.0f} s" for k, v in phase.items()))
    return dict(feats=feats, labels=labels, scales=scales, sigmas=sigmas,
                best_products=best_products, ident_products=ident_products)


def init_params(rng):
    sizes = (16, 64, 64, 3)
    parts = []
    for i in range(3):
        fi, fo = sizes[i], sizes[i + 1]
        parts.append(rng.standard_normal(fo * fi) * math.sqrt(2.0 / fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def fold_standardisation(theta, mu, sd):
    """First layer reading standardised x' = (x - mu) / sd -> reading raw x."""
    th = theta.copy()
    w1 = th[:64 * 16].reshape(64, 16)
    b1 = th[64 * 16:64 * 16 + 64]
    w1n = w1 / sd[None, :]
    b1n = b1 - w1n @ mu
    th[:64 * 16] = w1n.ravel()
    th[64 * 16:64 * 16 + 64] = b1n
    return th


def train(data, device, epochs=30, batch=1024, lr=2e-3, seed=0):
    x = data["feats"].astype(np.float64)
    mu = x.mean(0)
    sd = x.std(0) + 1e-6
    xs = ((x - mu) / sd).astype(np.float32)
    X = torch.tensor(xs, device=device)
    T = torch.tensor(data["labels"], device=device)
    rng = np.random.default_rng(seed)
    theta = torch.tensor(init_params(rng), device=device)
    grad = torch.zeros_like(theta)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    loss = torch.zeros(1, device=device)
    ws = torch.empty(ipr.ipr_mlp_workspace(batch), dtype=torch.uint8, device=device)
    nb = len(xs) // batch
    step = 0
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(len(xs)), device=device)
        tot = 0.0
        for bi in range(nb):
            sel = perm[bi * batch:(bi + 1) * batch]
            xb = X[sel].contiguous()
            tb = T[sel].contiguous()
            step += 1
            lr_t = lr * (0.5 * (1 + math.cos(math.pi * step / (epochs * nb))))
            ipr.ipr_mlp_train_step(theta, grad, m, v, xb, tb, step, max(lr_t, 1e-5), loss,
                                   workspace=ws)
            tot += float(loss.item()) if bi % 50 == 0 else 0.0
        log(f"epoch {ep}: loss {loss.item():.4e}")
    th = fold_standardisation(theta.cpu().numpy().astype(np.float64), mu, sd)
    return th.astype(np.float32), float(loss.item())


def predict(theta, feats, device):
    y = ipr.ipr_mlp_forward(torch.tensor(theta, device=device),
                            torch.tensor(feats, device=device).contiguous())
    return y.cpu().numpy()


def project(b, p):
    """The start the solver uses for a prediction: polynomial terms below 5%
    of b0 dropped, then scaled into eq. (2)'s set when it overshoots."""
    b = np.array(b, dtype=np.float64)
    if abs(b[1]) < 0.05 * b[0] and abs(b[2]) < 0.05 * b[0]:
        b[1] = b[2] = 0.0
    x = np.linspace(0.0, 1.0, 4001)[1:]
    q = b[0] + b[1] * x + b[2] * x * x
    if np.all(q > 0):
        sup = float(np.max(q ** p * x))
        if sup >= 2.0:
            b = b * (1.98 / sup) ** (1.0 / p)
    return b


def evaluate(theta, items, data, device):
    """Iterations and products of the learned start against the scaled
    identity, exact arithmetic (ipr_spectral_counts) on held-out items."""
    y = predict(theta, data["feats"], device)
    ps = np.array([it[1] for it in items])
    b = np.stack([project((np.exp(y[k, 0]), y[k, 1], y[k, 2]), ps[k])
                  for k in range(len(items))])
    ok = np.array([np.all(np.isfinite(b[k])) and guard_ok(b[k], ps[k])
                   for k in range(len(items))])
    res = {"fallback_rate": float(1 - ok.mean())}
    learned_products = np.where(ok, 0.0, np.nan)
    # group by n for the count kernel
    order = {}
    for k, it in enumerate(items):
        order.setdefault(it[0], []).append(k)
    iters_l = np.zeros(len(items))
    iters_i = data["ident_products"] / (ps + 1)
    for n, idx in sorted(order.items()):
        lams = [spectrum(n, items[k][2], items[k][3]) for k in idx]
        lam_flat = torch.tensor(np.concatenate(lams), dtype=torch.float64, device=device)
        bb = np.where(ok[idx, None], b[idx], np.array([1.0, 0.0, 0.0]))
        sc = np.where(ok[idx], data["scales"][idx], data["sigmas"][idx])
        cnt = ipr.ipr_spectral_counts(lam_flat, [j * n for j in range(len(idx))], [n] * len(idx),
                                      [int(ps[k]) for k in idx], list(sc), bb, TOL, MAXIT,
                                      per_item=True)
        iters_l[idx] = cnt
    extra = np.where(ok, 1 + np.where((b[:, 1] != 0) | (b[:, 2] != 0), ps, 0), 0)
    learned_products = extra + (ps + 1) * iters_l
    res.update({
        "items": len(items),
        "mean_iterations_identity": float(iters_i.mean()),
        "mean_iterations_learned": float(iters_l.mean()),
        "mean_products_identity": float(data["ident_products"].mean()),
        "mean_products_learned": float(learned_products.mean()),
        "mean_products_best_candidate": float(data["best_products"].mean()),
        "products_saved_fraction": float(1 - learned_products.mean() / data["ident_products"].mean()),
        "not_converged_learned": int((iters_l > MAXIT).sum()),
    })
    return res


def sets_of(args):
    return {"tr": recipe(args.train, 10**6), "ho": recipe(args.heldout, 2 * 10**6),
            "htr": recipe(args.hh_train, 3 * 10**6, reflectors="mix"),
            "hho": recipe(args.hh_heldout, 4 * 10**6, reflectors="mix")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200000)
    ap.add_argument("--heldout", type=int, default=10000)
    ap.add_argument("--hh-train", type=int, default=40000,
                    help="extra training matrices with Householder-product eigenvectors")
    ap.add_argument("--hh-heldout", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None)
    ap.add_argument("--build", default=None, metavar="SET:START:STOP:FILE",
                    help="only build items START..STOP-1 of set tr/ho/htr/hho into FILE (npz)")
    ap.add_argument("--shards", nargs="*", default=None,
                    help="npz files written by --build: train from them instead of building")
    args = ap.parse_args()
    ipr.load()
    device = torch.device("cuda:0")
    t0 = time.time()
    sets = sets_of(args)
    if args.build:
        key, a, b, path = args.build.split(":")
        a, b = int(a), int(b)
        log(f"building set {key} items {a}..{b - 1}")
        d = build_dataset(sets[key][a:b], device)
        np.savez(path, set=key, start=a, stop=b, **d)
        log(f"wrote {path} in {time.time() - t0:.0f} s")
        return
    data = {}
    if args.shards:
        parts = {}
        for f in args.shards:
            with np.load(f, allow_pickle=False) as z:
                parts.setdefault(str(z["set"]), []).append(
                    (int(z["start"]), int(z["stop"]),
                     {k: z[k] for k in z.files if k not in ("set", "start", "stop")}))
        for key, lst in parts.items():
            lst.sort(key=lambda t: t[0])
            assert lst[0][0] == 0 and all(lst[i][1] == lst[i + 1][0] for i in range(len(lst) - 1))
            assert lst[-1][1] == len(sets[key]), (key, lst[-1][1], len(sets[key]))
            data[key] = {k: np.concatenate([t[2][k] for t in lst]) for k in lst[0][2]}
        log(f"loaded {len(args.shards)} shards: " + ", ".join(f"{k} {len(v['feats'])}"
                                                              for k, v in data.items()))
    else:
        for key, items in sets.items():
            log(f"building set {key} ({len(items)} items)")
            data[key] = build_dataset(items, device)
    t1 = time.time()
    train_set = {k: np.concatenate([data["tr"][k], data["htr"][k]]) for k in data["tr"]}
    theta, final_loss = train(train_set, device, epochs=args.epochs)
    t2 = time.time()
    report = {"train_items": len(sets["tr"]), "train_items_householder": len(sets["htr"]),
              "heldout_items": len(sets["ho"]), "heldout_items_householder": len(sets["hho"]),
              "final_loss": final_loss, "seconds_data": t1 - t0, "seconds_train": t2 - t1,
              "train": evaluate(theta, sets["tr"][:20000],
                                {k: v[:20000] for k, v in data["tr"].items()}, device),
              "heldout": evaluate(theta, sets["ho"], data["ho"], device),
              "heldout_householder": evaluate(theta, sets["hho"], data["hho"], device)}
    np.savez(args.out, theta=theta, report=json.dumps(report))
    log(json.dumps(report, indent=1))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


def load_weights(path=WEIGHTS):
    """The stored network parameters (float32, IPR_MLP_NPARAM) or None."""
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return z["theta"].astype(np.float32)


if __name__ == "__main__":
    main()
