"""The learned (p, q) selector: training data, labels, GPU training and evaluation.

The paper picks the oversampling by a rule of thumb (Section 4: p = 10) and
the number of power steps by experience (Section 8: q = 1 or 2).  Here a small
network reads the singular values of a 16-column probe sketch (one thin pass
over A) and predicts, for each (p, q) of a grid, whether the plain method
meets the tolerance; the library then takes the cheapest point it trusts,
and the Section 14 certificate with the Figure 12 fallback covers misses.

Every step runs in the HIP library through its C ABI:
  features  rsvd_probe_sigma (probe sketch, FP64 CholeskyQR + Jacobi, input map)
  labels    rsvd_prefix_bounds (one Stage A run per q labels every p: the
            first k+p columns of the basis are the basis the plain method
            builds with k+p columns)
  training  rsvd_mlp_forward / rsvd_mlp_backward / rsvd_mlp_adam
  use       rsvd_factor on a plan with p = q = -1 after rsvd_selector_set
Matrices of the stream: workloads.gen.selector_matrix (m, n uniform in
[1000, 8000], sigma_j = j^-alpha exp(-(j-1)/tau), k = the 1e-3 rank).

Command line (GPU):
  python -m paper_1607_01649_amd.selector train --items 1500 --out W.npy
  python -m paper_1607_01649_amd.selector eval --weights W.npy --items 100
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

from . import (RSVD, RSVD_MLP_NPARAM, RSVD_RETURN_RANK_L, RSVD_SEL_NQ, RSVD_SEL_P, make_desc, rsvd_mlp_adam,
               rsvd_mlp_backward, rsvd_mlp_forward, rsvd_plan, rsvd_prefix_bounds, rsvd_probe_sigma,
               rsvd_workspace_size, selector_grid_cap)
from . import _aligned_workspace

EPS = 1e-3                 # relative spectral tolerance of the stream
SEED_TRAIN, SEED_TEST, SEED_COST = 1, 2, 3
N_OUT = 40
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.npy")
# training record next to the weights: threshold tau chosen on the validation items, data sizes, accuracy
WEIGHTS_META = WEIGHTS[:-4] + ".json"


def load_weights(path: str = WEIGHTS):
    """(theta as float32 numpy, tau)."""
    theta = np.load(path).astype(np.float32)
    meta = path[:-4] + ".json"
    tau = json.load(open(meta))["tau"] if os.path.exists(meta) else 0.3
    return theta, float(tau)


def simulated_time(prob, Y, M, meta, tau):
    """Modelled total time of the decision rule on labelled items: the chosen
    point's cost, plus (on a miss) the cost of the cheapest certified point as
    the price of the fallback."""
    tot = 0.0
    for pr, y, mk, (i, m, n, k) in zip(prob, Y, M, meta):
        pts = grid(m, n, k)
        ok = [(cost_ms(m, n, k, p, q) * (2.0 - pr[o]), o, p, q) for o, p, q in pts if pr[o] >= tau]
        o, p, q = (min(ok)[1:] if ok else max(pts, key=lambda t: (pr[t[0]], -t[0])))
        c = cost_ms(m, n, k, p, q)
        if y[o] < 0.5:
            feas = [cost_ms(m, n, k, pp, qq) for oo, pp, qq in pts if y[oo] > 0.5]
            c += min(feas) if feas else c
        tot += c
    return tot


def grid(m: int, n: int, k: int):
    """(o, p, q) for the grid points with k + p <= min(m, n, 1024)."""
    cap = selector_grid_cap(m, n)
    return [(iq * len(RSVD_SEL_P) + ip, p, iq) for iq in range(RSVD_SEL_NQ) for ip, p in enumerate(RSVD_SEL_P)
            if k + p <= cap]


# Coefficients of the modelled time (ms), fitted by `costfit` to measured plain-method times (eps = 0) on
# items of the stream: fixed part, ms per TFLOP of the 2q+2 passes, per CholeskyQR, per Jacobi unit.
COST_COEF = (0.081, 20.9, 0.104, 1.08)


def cost_terms(m, n, k, p, q):
    """The four terms of the modelled time (their coefficients in COST_COEF)."""
    l = min(k + p, m, n)
    return (1.0, (2 * q + 2) * 2.0 * m * n * l / 1e12, (2 * q + 1) * max(l / 128.0, 1.0) ** 1.5, (l / 95.0) ** 1.5)


def cost_ms(m, n, k, p, q) -> float:
    """The library's modelled time of (p, q) (include/rsvd.h)."""
    return float(sum(c * t for c, t in zip(COST_COEF, cost_terms(m, n, k, p, q))))


def _plan(m, n, k, p, q, device, **kw):
    d = make_desc(m, n, k, p, q, a_dtype="f32", **kw)
    ws = _aligned_workspace(rsvd_workspace_size(d), device)
    return rsvd_plan(d, ws), ws


def item_features(A: torch.Tensor, k: int, seed: int) -> torch.Tensor:
    """Network input (16 floats, device) from the probe sketch of A."""
    m, n = A.shape
    plan, ws = _plan(m, n, k, max(16 - k, 0), 0, A.device, seed=seed)
    try:
        sig = torch.empty(16, dtype=torch.float64, device=A.device)
        x = torch.empty(16, dtype=torch.float32, device=A.device)
        rsvd_probe_sigma(plan, A, sig, x)
        torch.cuda.synchronize(A.device)
        return x
    finally:
        from . import rsvd_destroy
        rsvd_destroy(plan)


def item_labels(A: torch.Tensor, k: int, seed: int, eps: float = EPS, sigma1: float = 1.0):
    """Labels (40) and mask (40): 1 where the plain method at (p, q) returns a
    rank-(k+p) result whose certificate is <= eps * sigma1."""
    from . import rsvd_destroy
    m, n = A.shape
    y = np.zeros(N_OUT, np.float32)
    mask = np.zeros(N_OUT, np.float32)
    pts = grid(m, n, k)
    ps = sorted({p for _, p, _ in pts})
    pmax = ps[-1]
    bounds = {}
    for q in range(RSVD_SEL_NQ):
        plan, ws = _plan(m, n, k, pmax, q, A.device, seed=seed, eps=eps)
        try:
            b = rsvd_prefix_bounds(plan, A, [k + p for p in ps])
        finally:
            rsvd_destroy(plan)
        for p, bb in zip(ps, b):
            o = q * len(RSVD_SEL_P) + RSVD_SEL_P.index(p)
            y[o] = 1.0 if bb <= eps * sigma1 else 0.0
            mask[o] = 1.0
            bounds[(p, q)] = bb
    return y, mask, bounds


def make_dataset(seed: int, items: int, device, log=None, start: int = 0):
    """Features, labels and masks of items start .. start+items-1 of the stream with this seed."""
    from workloads import gen
    X, Y, M, meta = [], [], [], []
    t0 = time.perf_counter()
    for i in range(start, start + items):
        A, k = gen.selector_matrix(seed, i, str(device))
        m, n = A.shape
        if k > selector_grid_cap(m, n):
            continue                      # target rank beyond the largest basis the library builds
        x = item_features(A, k, seed).cpu().numpy()
        y, mk, _ = item_labels(A, k, seed)
        X.append(x)
        Y.append(y)
        M.append(mk)
        meta.append((i, m, n, k))
        del A
        if log and (i - start + 1) % 100 == 0:
            log(f"items {i - start + 1}/{items}  {time.perf_counter() - t0:.1f} s")
    return np.array(X, np.float32), np.array(Y, np.float32), np.array(M, np.float32), meta


def init_theta(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    g = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((64, 16), (64, 64), (40, 64)):
        b = math.sqrt(6.0 / cols)
        parts.append(g.uniform(-b, b, size=rows * cols))
        parts.append(np.zeros(rows))
    th = np.concatenate(parts).astype(np.float32)
    assert th.size == RSVD_MLP_NPARAM
    return th


class Trainer:
    """Mini-batch Adam on the GPU with the library's network kernels."""

    def __init__(self, theta0: np.ndarray, device):
        self.dev = torch.device(device)
        self.theta = torch.from_numpy(np.asarray(theta0, np.float32)).to(self.dev)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.loss = torch.zeros(2, dtype=torch.float32, device=self.dev)
        self.t = 0

    def _bufs(self, B):
        f = dict(dtype=torch.float32, device=self.dev)
        return (torch.empty(B, 64, **f), torch.empty(B, 64, **f), torch.empty(B, N_OUT, **f),
                torch.empty(B * 168, **f))

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        H1, H2, Z, _ = self._bufs(X.shape[0])
        rsvd_mlp_forward(self.theta, X, H1, H2, Z)
        return Z

    def step(self, X, Y, M, lr) -> float:
        H1, H2, Z, scr = self._bufs(X.shape[0])
        rsvd_mlp_forward(self.theta, X, H1, H2, Z)
        rsvd_mlp_backward(self.theta, X, H1, H2, Z, Y, M, self.grad, self.loss, scr)
        self.t += 1
        rsvd_mlp_adam(self.theta, self.grad, self.m, self.v, lr, self.t)
        return float(self.loss[0])

    def fit(self, X, Y, M, epochs=300, batch=256, lr=2e-3, seed=0, log=None):
        g = np.random.default_rng(seed)
        Xd = torch.from_numpy(X).to(self.dev)
        Yd = torch.from_numpy(Y).to(self.dev)
        Md = torch.from_numpy(M).to(self.dev)
        N = X.shape[0]
        hist = []
        for ep in range(epochs):
            perm = torch.from_numpy(g.permutation(N)).to(self.dev)
            tot = 0.0
            for s in range(0, N, batch):
                idx = perm[s:s + batch]
                tot += self.step(Xd[idx].contiguous(), Yd[idx].contiguous(), Md[idx].contiguous(), lr)
            hist.append(tot / max(1, (N + batch - 1) // batch))
            if log and (ep + 1) % 50 == 0:
                log(f"epoch {ep + 1}: loss {hist[-1]:.4f}")
        return hist


def _solver(m, n, k, p, q, device, seed, theta=None, tau=0.5, sketch="f32"):
    """The stream's solver; sketch = "bf16" takes the sketches A Omega and the power steps' products in bf16 (the
    projection B = Q^T A stays FP32, so the residual the certificate measures carries no bf16 rounding of A)."""
    cap = selector_grid_cap(m, n)
    s = RSVD(m, n, k, p, q, dtype="f32", device=device, seed=seed, eps=EPS, max_rank=cap, fallback_block=32,
             flags=RSVD_RETURN_RANK_L, sketch_dtype=sketch, proj_dtype="f32")
    if theta is not None:
        s.set_selector(theta, tau)
    return s


def _timed(solver, A):
    torch.cuda.synchronize(A.device)
    t0 = time.perf_counter()
    U, S, V, info = solver(A)
    torch.cuda.synchronize(A.device)
    return (time.perf_counter() - t0) * 1e3, info


def evaluate(theta: torch.Tensor, seed: int, items: int, device, tau: float = 0.3, start: int = 0, log=None,
             with_best: bool = True, sketch: str = "f32"):
    """Time-to-eps on the items of a stream under four strategies: the paper's
    defaults (p = 10, q = 2) with fallback, the fallback alone (p = q = 0),
    the learned selector with fallback, and the per-item cheapest certified
    grid point (an upper bound on what a selector can gain)."""
    from workloads import gen
    rows = []
    warm = False
    for i in range(start, start + items):
        A, k = gen.selector_matrix(seed, i, str(device))
        m, n = A.shape
        if k > selector_grid_cap(m, n):
            continue
        strategies = {"default": (10, 2), "fallback_only": (0, 0), "learned": (-1, -1)}
        if with_best:
            y, mk, _ = item_labels(A, k, seed)
            feas = [(cost_ms(m, n, k, p, q), p, q) for o, p, q in grid(m, n, k) if y[o] > 0]
            pts = grid(m, n, k)
            strategies["best"] = min(feas)[1:] if feas else (pts[-1][1], pts[-1][2])
        row = {"item": i, "m": m, "n": n, "k": k}
        for name, (p, q) in strategies.items():
            if k + max(p, 0) > selector_grid_cap(m, n):
                p = 0
            sol = _solver(m, n, k, p, q, device, seed, theta if p == -1 else None, tau, sketch)
            if not warm:
                _timed(sol, A)
            ms, info = _timed(sol, A)
            row[name] = {"ms": ms, "status": int(info.status), "p": int(info.p_used), "q": int(info.q_used),
                         "rank": int(info.rank_out), "steps": int(info.fallback_steps),
                         "bound_rel": float(info.err_bound / max(info.sigma1, 1e-300))}
            del sol
        warm = True
        rows.append(row)
        del A
        if log and len(rows) % 10 == 0:
            log(f"eval items {len(rows)}")
    return rows


def summarize(rows):
    """Per strategy: totals over all items and over the items the paper's
    defaults certify (the others end at the rank cap under every strategy)."""
    out = {}
    cert = [r for r in rows if r["default"]["status"] == 0]
    for name in rows[0]:
        if name in ("item", "m", "n", "k"):
            continue
        ms = [r[name]["ms"] for r in rows]
        out[name] = {"total_ms": float(np.sum(ms)), "mean_ms": float(np.mean(ms)),
                     "certifiable_items": len(cert),
                     "certifiable_total_ms": float(np.sum([r[name]["ms"] for r in cert])),
                     "certified": float(np.mean([r[name]["status"] == 0 for r in rows])),
                     "no_fallback": float(np.mean([r[name]["steps"] == 0 and r[name]["status"] == 0
                                                   for r in rows]))}
    for name in out:
        if name == "default":
            continue
        d = np.array([r[name]["ms"] - r["default"]["ms"] for r in rows])
        half = 1.96 * float(np.std(d, ddof=1)) * math.sqrt(len(d)) if len(d) > 1 else float("nan")
        out[name]["vs_default_total_ms"] = {"diff": float(np.sum(d)), "ci95_half_width": half}
    return out


def costfit(seed: int, items: int, device, per_item: int = 3, log=None):
    """Times the plain method (eps = 0: no certificate, no fallback) at per_item random grid points of each of
    `items` stream items (one warm-up call, then the median of three), and fits the coefficients of the
    modelled time by non-negative least squares on the relative error."""
    from scipy.optimize import nnls
    from workloads import gen
    g = np.random.default_rng(seed)
    rows = []
    for i in range(items):
        A, k = gen.selector_matrix(seed, i, str(device))
        m, n = A.shape
        if k > selector_grid_cap(m, n):
            continue
        pts = grid(m, n, k)
        for j in g.choice(len(pts), size=min(per_item, len(pts)), replace=False):
            _, p, q = pts[j]
            sol = RSVD(m, n, k, p, q, dtype="f32", device=device, seed=seed)
            _timed(sol, A)
            ms = float(np.median([_timed(sol, A)[0] for _ in range(3)]))
            rows.append({"item": i, "m": m, "n": n, "k": k, "p": p, "q": q, "ms": ms})
            del sol
        del A
        if log and (i + 1) % 10 == 0:
            log(f"costfit items {i + 1}/{items}")
    T = np.array([cost_terms(r["m"], r["n"], r["k"], r["p"], r["q"]) for r in rows])
    t = np.array([r["ms"] for r in rows])
    coef, _ = nnls(T / t[:, None], np.ones(len(t)))
    old = np.array([sum(c * x for c, x in zip(COST_COEF, row)) for row in T])
    new = T @ coef
    return {"coef": coef.tolist(), "points": len(rows),
            "rel_err_old": {"median": float(np.median(np.abs(old / t - 1))), "max": float(np.max(np.abs(old / t - 1)))},
            "rel_err_new": {"median": float(np.median(np.abs(new / t - 1))), "max": float(np.max(np.abs(new / t - 1)))},
            "rows": rows}


def retune(theta: np.ndarray, val: int, start: int, device, log=None):
    """The threshold tau of least modelled time on labelled validation items of the training stream (items
    start .. start+val-1), under the current cost model."""
    Xv, Yv, Mv, metav = make_dataset(SEED_TRAIN, val, device, log, start=start)
    tr = Trainer(theta, device)
    Zv = tr.forward(torch.from_numpy(Xv).to(torch.device(device))).cpu().numpy()
    pv = 1.0 / (1.0 + np.exp(-Zv))
    taus = [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8]
    sim = {t: simulated_time(pv, Yv, Mv, metav, t) for t in taus}
    return min(sim, key=sim.get), sim, len(Xv)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval", "costfit", "retune"])
    ap.add_argument("--start", type=int, default=0, help="first item of the stream (eval, retune)")
    ap.add_argument("--sketch", choices=["f32", "bf16"], default="f32",
                    help="eval: precision of the sketches and power steps (the projection stays FP32)")
    ap.add_argument("--items", type=int, default=1500)
    ap.add_argument("--val", type=int, default=150)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--tau", type=float, default=None, help="default: the value stored with the weights")
    ap.add_argument("--json", default=None)
    ap.add_argument("--data", default=None, help="save the labelled items (npz)")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")

    def log(msg):
        print(msg, flush=True)
    if args.cmd == "train":
        X, Y, M, meta = make_dataset(SEED_TRAIN, args.items, dev, log)
        Xv, Yv, Mv, metav = make_dataset(SEED_TRAIN, args.val, dev, log, start=args.items)
        if args.data:
            np.savez(args.data, X=X, Y=Y, M=M, meta=np.array(meta), Xv=Xv, Yv=Yv, Mv=Mv, metav=np.array(metav))
        log(f"train items {len(X)}, positives {Y[M > 0].mean():.3f}")
        tr = Trainer(init_theta(0), dev)
        hist = tr.fit(X, Y, M, epochs=args.epochs, log=log)
        Zv = tr.forward(torch.from_numpy(Xv).to(dev)).cpu().numpy()
        pv = 1.0 / (1.0 + np.exp(-Zv))
        acc = float(((pv >= 0.5) == (Yv > 0.5))[Mv > 0].mean())
        taus = [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8]
        sim = {t: simulated_time(pv, Yv, Mv, metav, t) for t in taus}
        tau = min(sim, key=sim.get)
        np.save(args.out, tr.theta.cpu().numpy())
        res = {"train_items": len(X), "val_items": len(Xv), "final_loss": hist[-1], "val_accuracy": acc,
               "tau": tau, "val_modelled_ms": {str(t): v for t, v in sim.items()}, "epochs": args.epochs,
               "eps": EPS}
        json.dump(res, open(args.out[:-4] + ".json", "w"), indent=1)
        log(json.dumps(res))
        if args.json:
            json.dump({"summary": res, "loss": hist}, open(args.json, "w"))
    elif args.cmd == "costfit":
        res = costfit(SEED_COST, args.items, dev, log=log)
        log(json.dumps({k: v for k, v in res.items() if k != "rows"}))
        if args.json:
            json.dump(res, open(args.json, "w"))
    elif args.cmd == "retune":
        th, _ = load_weights(args.weights)
        tau, sim, nval = retune(th, args.val, args.start, dev, log)
        meta_path = args.weights[:-4] + ".json"
        meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
        meta.update({"tau": tau, "val_modelled_ms": {str(t): v for t, v in sim.items()}, "val_items": nval,
                     "cost_coef": list(COST_COEF)})
        json.dump(meta, open(args.out[:-4] + ".json", "w"), indent=1)
        log(json.dumps({"tau": tau, "val_modelled_ms": sim, "val_items": nval}))
    else:
        th, tau = load_weights(args.weights)
        theta = torch.from_numpy(th).to(dev)
        rows = evaluate(theta, SEED_TEST, args.items, dev, tau if args.tau is None else args.tau, start=args.start,
                        log=log, with_best=args.sketch == "f32", sketch=args.sketch)
        summ = summarize(rows)
        log(json.dumps(summ))
        if args.json:
            json.dump({"summary": summ, "rows": rows}, open(args.json, "w"))


if __name__ == "__main__":
    main()
