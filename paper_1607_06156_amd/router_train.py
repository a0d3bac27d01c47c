"""Train the route-selection MLP from measured route times, and evaluate it.

Dataset: graphs from the G(n,m), R-MAT (with and without per-level noise) and
thinned-lattice generators at log2 n ~ U[lo, hi], seeds 10^7 + i.  For each
graph the library computes the router features (64-bin log-degree histogram
/ n, log2 n, log2 m) and times the three routes (BFS then SV, SV, SV with
bounded link retries) with one warm-up and the median of three runs; the
label is the fastest route.  Training runs the library's FP32 SGD kernels;
the input standardisation is folded into the first layer so the exported
weights take raw features.

Held-out evaluation: new seeds from the same families plus graphs from the
power-law component-forest generator (a family the router never saw), timed
end to end with the router and with the degree heuristic.

    python -m paper_1607_06156_amd.router_train --n-train 3000 --out weights.txt

Large datasets can be built in pieces (--start, --dataset-out, --build-only)
and merged when training (--dataset-in).
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

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gen  # noqa: E402
import paper_1607_06156_amd as ccmi  # noqa: E402

FAMILIES = ["gnm", "rmat", "rmat-noisy", "grid"]


def make_graph(family: str, lg: float, deg: float, seed: int):
    if family == "gnm":
        n = int(round(2 ** lg))
        return gen.gnm(n, int(round(n * deg / 2)), seed)
    if family == "rmat":
        return gen.rmat(int(round(lg)), deg / 2, seed)
    if family == "rmat-noisy":
        return gen.rmat(int(round(lg)), deg / 2, seed, noise=0.1)
    if family == "grid":
        L = max(2, int(round(math.sqrt(2 ** lg))))
        return gen.grid(L, 0.5 + 0.4 * ((seed * 2654435761) % 1000) / 1000.0, seed)
    if family == "plcomp":
        return gen.plcomp(int(round(2 ** lg)), seed)
    raise KeyError(family)


def features(u, v, n, m):
    deg = ccmi.degree(u, v, n)
    h64, _, _, _, _ = ccmi.degree_histograms(deg)
    f = np.zeros(66, np.float64)
    f[:64] = h64.cpu().numpy().astype(np.float64) / max(n, 1)
    f[64] = math.log2(max(n, 1))
    f[65] = math.log2(max(m, 1))
    return f.astype(np.float32)


def time_route(u, v, n, route, reps=3):
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    ccmi.label(u, v, n, route=route, out=out)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ccmi.label(u, v, n, route=route, out=out)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def draw(seed0, i, lg_lo, lg_hi):
    """Scale and mean degree of graph i (a function of i alone, so datasets
    built in separate runs over disjoint index ranges concatenate)."""
    rng = np.random.default_rng([seed0, i])
    return float(rng.uniform(lg_lo, lg_hi)), float(rng.uniform(2, 32))


def build_dataset(count, seed0, lg_lo, lg_hi, families, log=None, start=0):
    X, T, meta = [], [], []
    for i in range(start, start + count):
        fam = families[i % len(families)]
        lg, deg = draw(seed0, i, lg_lo, lg_hi)
        g = make_graph(fam, lg, deg, seed0 + i)
        if g.m == 0:
            continue
        u = torch.from_numpy(g.u).cuda()
        v = torch.from_numpy(g.v).cuda()
        x = features(u, v, g.n, g.m)
        t = [time_route(u, v, g.n, r) for r in ("bfs+sv", "sv", "sv-theta")]
        X.append(x)
        T.append(t)
        meta.append({"family": fam, "n": g.n, "m": g.m})
        if log and (i % 100 == 0):
            log(f"[router] {i}/{count} {fam} n={g.n} m={g.m} times_ms={[round(a * 1e3, 3) for a in t]}")
    return np.array(X, np.float32), np.array(T, np.float64), meta


def init_params(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for fin, fout in [(66, 64), (64, 64), (64, 3)]:
        lim = math.sqrt(6.0 / fin)
        parts.append(rng.uniform(-lim, lim, (fout, fin)).astype(np.float32).reshape(-1))
        parts.append(np.zeros(fout, np.float32))
    return np.concatenate(parts)


def fit(X, y, epochs=300, batch=128, lr=0.05, seed=0, log=None):
    """SGD on standardised features with the library's kernels; returns raw-feature weights."""
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[sd < 1e-6] = 1.0
    Xs = ((X - mu) / sd).astype(np.float32)
    P = torch.from_numpy(init_params(seed)).cuda()
    Xd = torch.from_numpy(Xs).cuda()
    yd = torch.from_numpy(y.astype(np.int32)).cuda()
    rng = np.random.default_rng(seed)
    N = X.shape[0]
    for ep in range(epochs):
        order = rng.permutation(N)
        tot = 0.0
        for s in range(0, N, batch):
            idx = torch.from_numpy(order[s:s + batch]).cuda()
            loss, _ = ccmi.mlp_sgd_step(P, Xd[idx].contiguous(), yd[idx].contiguous(), lr)
            tot += loss * idx.numel()
        if log and (ep % 50 == 0 or ep == epochs - 1):
            log(f"[router] epoch {ep} loss {tot / N:.4f}")
    w = P.cpu().numpy().astype(np.float64)
    # fold x' = (x - mu) / sd into layer 1: W1' = W1 / sd, b1' = b1 - W1' mu
    W1 = w[: 64 * 66].reshape(64, 66) / sd[None, :]
    b1 = w[64 * 66: 64 * 66 + 64] - W1 @ mu
    w[: 64 * 66] = W1.reshape(-1)
    w[64 * 66: 64 * 66 + 64] = b1
    return w.astype(np.float32)


def accuracy(w, X, y):
    logits = ccmi.mlp_forward(torch.from_numpy(w).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    return float(np.mean(np.argmax(logits, axis=1) == y)), np.argmax(logits, axis=1)


def evaluate(w, count, seed0, lg_lo, lg_hi, log=None):
    """End-to-end time with the router vs the degree heuristic on held-out graphs."""
    ccmi.router_set(w)
    fams = FAMILIES + ["plcomp"]
    rows = []
    for i in range(count):
        fam = fams[i % len(fams)]
        lg, deg = draw(seed0, i, lg_lo, lg_hi)
        g = make_graph(fam, lg, deg, seed0 + i)
        if g.m == 0:
            continue
        u = torch.from_numpy(g.u).cuda()
        v = torch.from_numpy(g.v).cuda()
        tr = time_route(u, v, g.n, "router")
        th = time_route(u, v, g.n, "heuristic")
        _, st_r = ccmi.label(u, v, g.n, route="router", stats=True)
        _, st_h = ccmi.label(u, v, g.n, route="heuristic", stats=True)
        best = min(time_route(u, v, g.n, r) for r in ("bfs+sv", "sv", "sv-theta"))
        rows.append({"family": fam, "n": g.n, "m": g.m, "router_s": tr, "heuristic_s": th, "best_forced_s": best,
                     "router_route": st_r["route_name"], "heuristic_route": st_h["route_name"]})
        if log and (i % 100 == 0):
            log(f"[router] eval {i}/{count} {fam} n={g.n} m={g.m} router {tr * 1e3:.3f} ms "
                f"heuristic {th * 1e3:.3f} ms")
    ccmi.router_set(None)
    out = {"graphs": len(rows)}
    for key in ["router_s", "heuristic_s", "best_forced_s"]:
        out[key] = sum(r[key] for r in rows)
    by = {}
    for r in rows:
        f = by.setdefault(r["family"], {"graphs": 0, "router_s": 0.0, "heuristic_s": 0.0})
        f["graphs"] += 1
        f["router_s"] += r["router_s"]
        f["heuristic_s"] += r["heuristic_s"]
    out["by_family"] = by
    out["router_no_slower"] = out["router_s"] <= out["heuristic_s"]
    return out, rows


def load(path):
    """Weights written by save(): the parameters in order, comments skipped."""
    with open(path) as f:
        vals = [float(x) for line in f if not line.lstrip().startswith("#") for x in line.split()]
    w = np.asarray(vals, dtype=np.float32)
    if w.size != ccmi.ROUTER_NPARAMS:
        raise ValueError(f"{path}: {w.size} parameters, expected {ccmi.ROUTER_NPARAMS}")
    return w


def save(w, path, note):
    with open(path, "w") as f:
        f.write("# route-selection MLP 66-64-64-3, FP32, row-major [out][in]: W1 b1 W2 b2 W3 b3\n")
        for line in note.splitlines():
            f.write("# " + line + "\n")
        for i in range(0, w.size, 8):
            f.write(" ".join(f"{x:.9g}" for x in w[i:i + 8]) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=3000)
    ap.add_argument("--n-eval", type=int, default=300)
    ap.add_argument("--lg-lo", type=float, default=10.0)
    ap.add_argument("--lg-hi", type=float, default=20.0)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--out", default="router_weights.txt")
    ap.add_argument("--report", default="router_report.json")
    ap.add_argument("--start", type=int, default=0, help="index of the first training graph to build")
    ap.add_argument("--dataset-in", action="append", default=[], help="earlier dataset (.npz) to prepend")
    ap.add_argument("--dataset-out", default=None, help="save the dataset built here (.npz)")
    ap.add_argument("--build-only", action="store_true", help="build (and save) the dataset, do not train")
    ap.add_argument("--eval-weights", default=None,
                    help="only evaluate these saved weights on the held-out graphs (no training)")
    args = ap.parse_args()

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    t0 = time.time()
    if args.eval_weights:
        w = load(args.eval_weights)
        rep, rows = evaluate(w, args.n_eval, 20_000_000, args.lg_lo, args.lg_hi, log)
        rep.update({"weights": args.eval_weights, "seconds": time.time() - t0})
        log(f"[router] evaluation: router {rep['router_s'] * 1e3:.1f} ms vs heuristic "
            f"{rep['heuristic_s'] * 1e3:.1f} ms (best forced {rep['best_forced_s'] * 1e3:.1f} ms) "
            f"over {rep['graphs']} graphs")
        with open(args.report, "w") as f:
            json.dump({"summary": rep, "rows": rows}, f, indent=1)
        print(json.dumps(rep))
        return
    X, T, meta = build_dataset(args.n_train, 10_000_000, args.lg_lo, args.lg_hi, FAMILIES, log, start=args.start)
    if args.dataset_out:
        np.savez(args.dataset_out, X=X, T=T, n=np.array([r["n"] for r in meta], np.int64),
                 m=np.array([r["m"] for r in meta], np.int64),
                 family=np.array([FAMILIES.index(r["family"]) for r in meta], np.int8))
        log(f"[router] saved {len(T)} graphs to {args.dataset_out}")
    if args.build_only:
        return
    for path in args.dataset_in:
        d = np.load(path)
        X = np.concatenate([d["X"], X]) if len(X) else d["X"]
        T = np.concatenate([d["T"], T]) if len(T) else d["T"]
        log(f"[router] loaded {len(d['T'])} graphs from {path}")
    y = np.argmin(T, axis=1)
    log(f"[router] dataset {len(y)} graphs in {time.time() - t0:.0f}s; label counts {np.bincount(y, minlength=3)}")
    ntr = int(0.9 * len(y))
    w = fit(X[:ntr], y[:ntr], epochs=args.epochs, log=log)
    acc_tr, _ = accuracy(w, X[:ntr], y[:ntr])
    acc_va, pred = accuracy(w, X[ntr:], y[ntr:])
    # time regret on the validation split: chosen route time / best time
    Tv = T[ntr:]
    regret = float(np.sum(Tv[np.arange(len(pred)), pred]) / np.sum(Tv.min(axis=1)))
    log(f"[router] train acc {acc_tr:.3f} val acc {acc_va:.3f} val time / best {regret:.4f}")
    note = (f"trained on {ntr} graphs (families {', '.join(FAMILIES)}, log2 n in [{args.lg_lo}, {args.lg_hi}], "
            f"seeds 1e7+i), labels = fastest measured route; train acc {acc_tr:.3f}, val acc {acc_va:.3f}; "
            f"held-out {len(y) - ntr} graphs")
    save(w, args.out, note)
    rep, rows = evaluate(w, args.n_eval, 20_000_000, args.lg_lo, args.lg_hi, log)
    rep.update({"train_graphs": ntr, "val_acc": acc_va, "train_acc": acc_tr, "val_time_over_best": regret,
                "label_counts": np.bincount(y, minlength=3).tolist(), "seconds": time.time() - t0})
    log(f"[router] evaluation: router {rep['router_s'] * 1e3:.1f} ms vs heuristic {rep['heuristic_s'] * 1e3:.1f} ms "
        f"(best forced {rep['best_forced_s'] * 1e3:.1f} ms) over {rep['graphs']} graphs")
    with open(args.report, "w") as f:
        json.dump({"summary": rep, "rows": rows}, f, indent=1)
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
