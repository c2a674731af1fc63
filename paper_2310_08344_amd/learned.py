"""Learned spectral bound and sweep budget for batched phi actions.

The plain method takes each instance's spectral bound from power iteration
(Listing 7 of the paper) and runs the Leja loop until its stop rule passes.
Here a small MLP (lx_predictor, trained by the library's own kernels)
predicts log(1.05 rho_hat) and log(sweeps) from 8 instance features; the
predicted bound replaces power iteration and the predicted sweep count
becomes a budget.  A prediction is accepted only when the instance's Leja
loop converges within its budget; every other instance falls back to the
plain method (power iteration, then the loop without a budget).

Everything numerical runs in the HIP library; this module moves data and
orchestrates calls.

    python -m paper_2310_08344_amd.learned records --count N --seed S --out R.npz
    python -m paper_2310_08344_amd.learned train --records R1.npz [R2.npz ...] --out P.bin --summary S.json
    python -m paper_2310_08344_amd.learned evaluate --predictor P.bin --out E.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import binding as B
from . import workloads as W

SAFETY = 1.05
POWER_ITERS = 20
RTOL = 1e-8
MAX_ITERS = 400
PREDICTOR_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "predictor.bin")


def _log(*a):
    print("[learned]", *a, file=sys.stderr, flush=True)


def _instance_args(items, dev):
    import torch
    args, keep = [], []
    for p, u, v in items:
        tv = torch.as_tensor(v).to(dev)
        tu = torch.as_tensor(u).to(dev) if u is not None else None
        out = torch.empty_like(tv)
        a = dict(op=B.make_operator(p), v=tv, out=out, l=p.meta["l"], h=p.h)
        if tu is not None:
            a["u"] = tu
        args.append(a)
        keep.append((tv, tu, out))
    return args, keep


def features(ctx, args):
    import torch
    X = torch.empty(len(args), 8, dtype=torch.float32, device="cuda:0")
    ctx.features(args, X)
    return X


# --------------------------------------------------------------------------
# records
# --------------------------------------------------------------------------

def generate_records(ctx, count: int, seed0: int, batch: int = 512, sizes=(64, 128, 256)):
    """Runs the plain batched method (power iteration + Leja at rtol 1e-8)
    on `count` seeded instances and returns (X [n, 8] float32 features,
    Y [n, 2] float32 targets log(1.05 rho_hat), log(sweeps), kinds [n]);
    instances that do not converge within MAX_ITERS sweeps are dropped."""
    import torch
    Xs, Ys, kinds = [], [], []
    t0 = time.perf_counter()
    for b0 in range(0, count, batch):
        items = [W.learned_instance(i, seed0, sizes) for i in range(b0, min(count, b0 + batch))]
        args, keep = _instance_args(items, "cuda:0")
        X = features(ctx, args)
        st, res = ctx.phi_leja_batched(args, power_iters=POWER_ITERS, safety=SAFETY, rtol=RTOL,
                                       max_iters=MAX_ITERS, raise_on_error=False)
        Xh = X.cpu().numpy()
        for (p, _, _), x, r in zip(items, Xh, res):
            if r["status"] != B.LX_OK or not (r["rho_hat"] > 0):
                continue
            Xs.append(x)
            Ys.append([math.log(SAFETY * r["rho_hat"]), math.log(r["iters"])])
            kinds.append(0 if p.kind == W.DIFFADV else 1)
        del keep
        _log(f"records {min(count, b0 + batch)}/{count}, kept {len(Xs)}, {time.perf_counter() - t0:.1f} s")
    return (np.asarray(Xs, dtype=np.float32), np.asarray(Ys, dtype=np.float32), np.asarray(kinds, dtype=np.int8))


# --------------------------------------------------------------------------
# training
# --------------------------------------------------------------------------

def train_predictor(ctx, X, Y, steps=20000, batch=512, lr=1e-3, seed=1, val_frac=0.1):
    """Standardises, trains on (1 - val_frac) of the records and measures the
    validation residuals.  Returns (predictor, summary dict).  The summary's
    margins are the 99th percentile of log(rho) underestimation and the
    95th percentile of log(sweeps) underestimation on the validation set."""
    import torch
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    nv = max(1, int(n * val_frac))
    iv, it = perm[:nv], perm[nv:]
    mx, sx = X[it].mean(axis=0), X[it].std(axis=0) + 1e-6
    my, sy = Y[it].mean(axis=0), Y[it].std(axis=0) + 1e-6
    p = ctx.predictor(seed=seed)
    p.set_scaling(mx, sx, my, sy)
    Xt = torch.as_tensor(np.ascontiguousarray(X[it])).to("cuda:0")
    Yt = torch.as_tensor(np.ascontiguousarray(Y[it])).to("cuda:0")
    t0 = time.perf_counter()
    losses = []
    chunk = max(1, steps // 10)
    for k in range(0, steps, chunk):
        frac = k / steps
        lr_k = lr * (0.1 ** frac)     # geometric decay to lr/10
        losses.append(p.train(Xt, Yt, min(chunk, steps - k), min(batch, len(it)), lr_k, seed=seed + k))
        _log(f"train step {k + chunk}/{steps} loss {losses[-1]:.4g}")
    train_s = time.perf_counter() - t0
    Xv = torch.as_tensor(np.ascontiguousarray(X[iv])).to("cuda:0")
    out = torch.empty(len(iv), 2, dtype=torch.float32, device="cuda:0")
    p.infer(Xv, out)
    pred = out.cpu().numpy().astype(np.float64)
    res = Y[iv].astype(np.float64) - pred          # > 0: the network underestimates
    summary = {
        "records": int(n), "train": int(len(it)), "validation": int(nv),
        "steps": int(steps), "batch": int(batch), "lr": lr, "train_seconds": round(train_s, 2),
        "final_minibatch_loss": losses[-1],
        "val_rmse_log_rho": float(np.sqrt(np.mean(res[:, 0] ** 2))),
        "val_rmse_log_sweeps": float(np.sqrt(np.mean(res[:, 1] ** 2))),
        "margin_log_rho": float(max(0.0, np.quantile(res[:, 0], 0.99))),
        "margin_log_sweeps": float(max(0.0, np.quantile(res[:, 1], 0.95))),
    }
    return p, summary


# --------------------------------------------------------------------------
# solving with the predictor
# --------------------------------------------------------------------------

def solve_plain(ctx, args):
    st, res = ctx.phi_leja_batched(args, power_iters=POWER_ITERS, safety=SAFETY, rtol=RTOL, max_iters=MAX_ITERS,
                                   raise_on_error=False)
    return res


def solve_learned(ctx, predictor, args, margin_log_rho, margin_log_sweeps):
    """Predicted bound and budget; instances that do not converge within their
    budget are solved again by the plain method.  Returns (results,
    fallback indices)."""
    import torch
    X = features(ctx, args)
    Y = torch.empty(len(args), 2, dtype=torch.float32, device="cuda:0")
    predictor.infer(X, Y)
    pred = Y.cpu().numpy().astype(np.float64)
    largs = []
    for a, (lr, ls) in zip(args, pred):
        lam = -math.exp(lr + margin_log_rho)          # lambda = -(1.05 rho_hat), inflated
        budget = int(min(MAX_ITERS, math.ceil(math.exp(ls + margin_log_sweeps)) + 2))
        q = dict(a)
        q.update(c=lam / 2.0, gamma=-lam / 4.0, budget=max(budget, 1))
        largs.append(q)
    st, res = ctx.phi_leja_batched(largs, power_iters=0, rtol=RTOL, max_iters=MAX_ITERS, raise_on_error=False)
    fb = [i for i, r in enumerate(res) if r["status"] != B.LX_OK]
    if fb:
        st2, res2 = ctx.phi_leja_batched([args[i] for i in fb], power_iters=POWER_ITERS, safety=SAFETY, rtol=RTOL,
                                         max_iters=MAX_ITERS, raise_on_error=False)
        for i, r in zip(fb, res2):
            r["fallback"] = True
            res[i] = r
    return res, fb


def solve_plain_single(ctx, args):
    """The plain path instance by instance: lx_spectrum then lx_phi_leja."""
    res = []
    for a in args:
        _, c, g = ctx.spectrum(a["op"], u=a.get("u"), iters=POWER_ITERS, safety=SAFETY)
        r = ctx.phi_leja(a["op"], a["v"], [a["out"]], [a["l"]], a["h"], c, g, u=a.get("u"), rtol=RTOL,
                         max_iters=MAX_ITERS, raise_on_error=False)
        res.append({"status": r.status, "iters": r.iters[0]})
    return res


def evaluate(ctx, predictor, margins, count=1024, seed0=900000, size=256, repeats=2):
    """Time-to-solution of the learned + batched path against the plain
    batched path and the plain single-instance path on `count` instances
    (half diffusion-advection, half Burgers) at size^2."""
    import torch
    items = [W.learned_instance(i, seed0, (size,)) for i in range(count)]
    args, keep = _instance_args(items, "cuda:0")
    outs_plain = [torch.empty_like(a["out"]) for a in args]
    pargs = [dict(a, out=o) for a, o in zip(args, outs_plain)]

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    solve_plain(ctx, pargs)                       # warm-up
    solve_learned(ctx, predictor, args, *margins)
    t_plain = t_learn = 0.0
    for _ in range(repeats):
        res_p, t = timed(lambda: solve_plain(ctx, pargs))
        t_plain += t / repeats
        (res_l, fb), t = timed(lambda: solve_learned(ctx, predictor, args, *margins))
        t_learn += t / repeats
    res_s, t_single = timed(lambda: solve_plain_single(ctx, pargs))
    # agreement of the accepted learned results with the plain ones
    diffs = []
    for a, o in zip(args, outs_plain):
        d = torch.linalg.vector_norm(a["out"] - o) / torch.clamp(torch.linalg.vector_norm(o), min=1e-300)
        diffs.append(float(d))
    sweeps_p = sum(r["iters"] for r in res_p) + POWER_ITERS * count
    sweeps_l = sum(r["iters"] for r in res_l) + POWER_ITERS * len(fb)
    return {
        "instances": count, "grid": size, "rtol": RTOL,
        "plain_batched_ms": round(t_plain * 1e3, 3), "learned_batched_ms": round(t_learn * 1e3, 3),
        "plain_single_ms": round(t_single * 1e3, 3),
        "speedup_learned_vs_plain_batched": round(t_plain / t_learn, 3),
        "speedup_learned_vs_plain_single": round(t_single / t_learn, 3),
        "accepted": count - len(fb), "fallbacks": len(fb),
        "all_converged": all(r["status"] == B.LX_OK for r in res_l),
        "sweeps_plain_incl_power": int(sweeps_p), "sweeps_learned_incl_fallback_power": int(sweeps_l),
        "max_rel_diff_learned_vs_plain": max(diffs), "median_rel_diff_learned_vs_plain": float(np.median(diffs)),
    }


def load_predictor(ctx, path=PREDICTOR_FILE):
    """The committed predictor and its margins."""
    p = ctx.predictor()
    p.load(path)
    with open(os.path.splitext(path)[0] + ".json") as f:
        meta = json.load(f)
    return p, (meta["margin_log_rho"], meta["margin_log_sweeps"]), meta


# --------------------------------------------------------------------------
# command line
# --------------------------------------------------------------------------

def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2310_08344_amd.learned")
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("records")
    r.add_argument("--count", type=int, required=True)
    r.add_argument("--seed", type=int, default=100000)
    r.add_argument("--batch", type=int, default=512)
    r.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--records", nargs="+", required=True)
    t.add_argument("--steps", type=int, default=20000)
    t.add_argument("--batch", type=int, default=512)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", required=True)
    t.add_argument("--summary", required=True)
    e = sub.add_parser("evaluate")
    e.add_argument("--predictor", default=PREDICTOR_FILE)
    e.add_argument("--count", type=int, default=1024)
    e.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    lib = B.Library.load()
    ctx = lib.context(n_max=1 << 16, k_max=1)
    if args.cmd == "records":
        X, Y, K = generate_records(ctx, args.count, args.seed, args.batch)
        np.savez(args.out, X=X, Y=Y, kind=K)
        _log("wrote", args.out, X.shape)
    elif args.cmd == "train":
        parts = [np.load(f) for f in args.records]
        X = np.concatenate([q["X"] for q in parts])
        Y = np.concatenate([q["Y"] for q in parts])
        p, summary = train_predictor(ctx, X, Y, args.steps, args.batch, args.lr)
        p.save(args.out)
        with open(args.summary, "w") as f:
            json.dump(summary, f, indent=1)
        _log("wrote", args.out, summary)
    else:
        p, margins, meta = load_predictor(ctx, args.predictor)
        res = evaluate(ctx, p, margins, count=args.count)
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
        _log(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
