"""Learned spectral bound and sweep budget for batched phi actions.

The plain method takes each instance's spectral bound from power iteration
(Listing 7 of the paper) and runs the Leja loop until its stop rule passes.
Here a small MLP (lx_predictor, trained by the library's own kernels)
predicts log(1.05 rho_hat) and log(sweeps) from 8 instance features; the
predicted bound replaces power iteration and the predicted sweep count
becomes a budget.  A prediction is accepted only when the instance's Leja
loop converges within its budget; every other instance falls back to the
plain method (power iteration, then the loop without a budget).

Everything numerical runs in the HIP library; this module draws instances
(through the workloads module), moves data and orchestrates calls.

    python -m paper_2310_08344_amd.learned all --records 100000 --out-dir DIR
    python -m paper_2310_08344_amd.learned evaluate --predictor P.bin --out E.json

`all` generates the records with the plain method, trains, calibrates the
budget margin on held-out instances, writes DIR/predictor.bin and
DIR/predictor.json, and evaluates on 1024 instances at 256^2.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import workloads as W

SAFETY = 1.05
POWER_ITERS = 20
RTOL = 1e-8
MAX_ITERS = 400
DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
PREDICTOR_FILE = os.path.join(DATA_DIR, "predictor.bin")

# seeds of the instance streams: training records, budget calibration, evaluation
SEED_RECORDS, SEED_CALIBRATION, SEED_EVALUATION = 100000, 500000, 900000


def _log(*a):
    print("[learned]", *a, file=sys.stderr, flush=True)


def _draw(job):
    index, seed0, sizes = job
    return W.learned_instance(index, seed0, sizes)


def draw_instances(indices, seed0, sizes, pool=None):
    """learned_instance for each index (in a process pool when given)."""
    jobs = [(int(i), seed0, tuple(sizes)) for i in indices]
    if pool is None:
        return [_draw(j) for j in jobs]
    return pool.map(_draw, jobs, chunksize=16)


def _instance_args(items, dev):
    import torch
    from . import binding as B
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

def generate_records(ctx, count: int, seed0: int = SEED_RECORDS, batch: int = 1024, sizes=(64, 128, 256),
                     pool=None):
    """Runs the plain batched method (power iteration + Leja at rtol 1e-8)
    on `count` seeded instances and returns (X [n, 8] float32 features,
    Y [n, 2] float32 targets log(1.05 rho_hat), log(sweeps), kinds [n]);
    instances that do not converge within MAX_ITERS sweeps are dropped."""
    from . import binding as B
    Xs, Ys, kinds = [], [], []
    t0 = time.perf_counter()
    for b0 in range(0, count, batch):
        items = draw_instances(range(b0, min(count, b0 + batch)), seed0, sizes, pool)
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
    """Standardises, trains on (1 - val_frac) of the records with Adam (the
    step size decays geometrically to lr/10) and measures the validation
    residuals.  Returns (predictor, summary dict); the summary's
    margin_log_rho is the 99th percentile of the validation underestimates
    of log(1.05 rho_hat)."""
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
    loss = float("nan")
    chunk = max(1, steps // 10)
    for k in range(0, steps, chunk):
        lr_k = lr * (0.1 ** (k / steps))
        loss = p.train(Xt, Yt, min(chunk, steps - k), min(batch, len(it)), lr_k, seed=seed + k)
        _log(f"train step {min(k + chunk, steps)}/{steps} minibatch loss {loss:.4g}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    Xv = torch.as_tensor(np.ascontiguousarray(X[iv])).to("cuda:0")
    out = torch.empty(len(iv), 2, dtype=torch.float32, device="cuda:0")
    p.infer(Xv, out)
    pred = out.cpu().numpy().astype(np.float64)
    res = Y[iv].astype(np.float64) - pred          # > 0: the network underestimates
    summary = {
        "records": int(n), "train": int(len(it)), "validation": int(nv),
        "steps": int(steps), "batch": int(batch), "lr": lr, "train_seconds": round(train_s, 2),
        "final_minibatch_loss": loss,
        "val_rmse_log_rho": float(np.sqrt(np.mean(res[:, 0] ** 2))),
        "val_rmse_log_sweeps": float(np.sqrt(np.mean(res[:, 1] ** 2))),
        "margin_log_rho": float(max(0.0, np.quantile(res[:, 0], 0.99))),
    }
    return p, summary


def calibrate_budget(ctx, predictor, margin_log_rho, count=4096, seed0=SEED_CALIBRATION, sizes=(64, 128, 256),
                     pool=None, quantile=0.98):
    """Runs held-out instances with the predicted (inflated) interval and no
    budget, and returns the `quantile` of log(sweeps needed) - predicted
    log(sweeps): the margin that makes the budget cover that share of
    instances."""
    import torch
    from . import binding as B
    r_all = []
    for b0 in range(0, count, 1024):
        items = draw_instances(range(b0, min(count, b0 + 1024)), seed0, sizes, pool)
        args, keep = _instance_args(items, "cuda:0")
        X = features(ctx, args)
        Yp = torch.empty(len(args), 2, dtype=torch.float32, device="cuda:0")
        predictor.infer(X, Yp)
        pred = Yp.cpu().numpy().astype(np.float64)
        largs = []
        for a, (lr_, _) in zip(args, pred):
            lam = -math.exp(lr_ + margin_log_rho)
            largs.append(dict(a, c=lam / 2.0, gamma=-lam / 4.0))
        st, res = ctx.phi_leja_batched(largs, power_iters=0, rtol=RTOL, max_iters=MAX_ITERS, raise_on_error=False)
        for r, (_, ls) in zip(res, pred):
            r_all.append(math.log(r["iters"]) - ls if r["status"] == B.LX_OK else float("inf"))
        del keep
    r_all = np.asarray(r_all)
    finite = np.isfinite(r_all)
    margin = float(max(0.0, np.quantile(r_all[finite], quantile))) if finite.any() else 1.0
    return margin, {"calibration_instances": int(count), "calibration_unconverged": int((~finite).sum()),
                    "budget_quantile": quantile, "margin_log_sweeps": margin}


# --------------------------------------------------------------------------
# solving with the predictor
# --------------------------------------------------------------------------

def solve_plain(ctx, args):
    """The plain batched method: power iteration, then the Leja loop."""
    st, res = ctx.phi_leja_batched(args, power_iters=POWER_ITERS, safety=SAFETY, rtol=RTOL, max_iters=MAX_ITERS,
                                   raise_on_error=False)
    return res


def solve_learned(ctx, predictor, args, margin_log_rho, margin_log_sweeps):
    """Predicted bound and budget (lx_phi_leja_learned, one library call):
    instances that do not converge within their budget are solved again by
    the plain method.  Returns (results, fallback indices)."""
    st, res, nf = ctx.phi_leja_learned(args, predictor, margin_log_rho, margin_log_sweeps,
                                       power_iters=POWER_ITERS, safety=SAFETY, rtol=RTOL, max_iters=MAX_ITERS,
                                       raise_on_error=False)
    return res, [i for i, r in enumerate(res) if r["fallback"]]


def solve_plain_single(ctx, args):
    """The plain path instance by instance: lx_spectrum then lx_phi_leja."""
    res = []
    for a in args:
        _, c, g = ctx.spectrum(a["op"], u=a.get("u"), iters=POWER_ITERS, safety=SAFETY)
        r = ctx.phi_leja(a["op"], a["v"], [a["out"]], [a["l"]], a["h"], c, g, u=a.get("u"), rtol=RTOL,
                         max_iters=MAX_ITERS, raise_on_error=False)
        res.append({"status": r.status, "iters": r.iters[0]})
    return res


def evaluate(ctx, predictor, margins, count=1024, seed0=SEED_EVALUATION, size=256, repeats=10, warmups=3, pool=None,
             tune=True):
    """Time-to-solution of the learned + batched path against the plain
    batched path and the plain single-instance path on `count` instances
    (half diffusion-advection, half Burgers) at size^2, inputs resident on
    the GPU; the three timings cover the whole solve, predictor and
    fallbacks included."""
    import torch
    from . import binding as B
    items = draw_instances(range(count), seed0, (size,), pool)
    args, keep = _instance_args(items, "cuda:0")
    outs_plain = [torch.empty_like(a["out"]) for a in args]
    pargs = [dict(a, out=o) for a, o in zip(args, outs_plain)]
    outs_single = [torch.empty_like(a["out"]) for a in args]
    sargs = [dict(a, out=o) for a, o in zip(args, outs_single)]

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    # descriptors are built once per instance set, for both paths; the
    # batch launch shape of this instance class comes from the autotuner
    # (timed on the plain batched path; the learned path shares the class)
    pb, lb = ctx.prepare(pargs), ctx.prepare(args)
    tuned = (ctx.tune_batched(pb, power_iters=POWER_ITERS, safety=SAFETY, rtol=RTOL, max_iters=MAX_ITERS, repeats=3)
             if tune else [])
    best = min(tuned, key=lambda r: r[3]) if tuned else (0, 0, 0, None)
    for _ in range(warmups):
        solve_plain(ctx, pb)
        solve_learned(ctx, predictor, lb, *margins)
    tp, tl = [], []
    for _ in range(repeats):
        res_p, t = timed(lambda: solve_plain(ctx, pb))
        tp.append(t)
        (res_l, fb), t = timed(lambda: solve_learned(ctx, predictor, lb, *margins))
        tl.append(t)
    t_plain, t_learn = float(np.median(tp)), float(np.median(tl))
    res_s, t_single = timed(lambda: solve_plain_single(ctx, sargs))
    ok_p = [r["status"] == B.LX_OK for r in res_p]
    diffs, idx = [], []
    for i, (a, o, okp) in enumerate(zip(args, outs_plain, ok_p)):
        if okp:
            d = torch.linalg.vector_norm(a["out"] - o) / torch.clamp(torch.linalg.vector_norm(o), min=1e-300)
            diffs.append(float(d))
            idx.append(i)
    order = np.argsort(diffs)[::-1][:3] if diffs else []
    largest = [{"index": int(idx[j]), "seed": int(seed0 + idx[j]), "kind": items[idx[j]][0].kind,
                "l": int(items[idx[j]][0].meta["l"]), "rel_diff": diffs[j],
                "sweeps_learned_plain": [int(res_l[idx[j]]["iters"]), int(res_p[idx[j]]["iters"])],
                "fallback": bool(res_l[idx[j]]["fallback"])} for j in order]
    sweeps_p = sum(r["iters"] for r in res_p) + POWER_ITERS * count
    sweeps_l = sum(r["iters"] for r in res_l) + POWER_ITERS * len(fb)
    kinds = np.array([0 if p.kind == W.DIFFADV else 1 for p, _, _ in items])
    fb_kinds = kinds[fb] if fb else np.array([], dtype=int)
    return {
        "instances": count, "grid": size, "rtol": RTOL,
        "timing": f"median of {repeats} after {warmups} warm-ups (plain and learned batched, alternating); one "
                  "run of the per-instance path; inputs resident on the GPU and instance descriptors prepared "
                  "once for either path",
        "plain_batched_ms": round(t_plain * 1e3, 3), "learned_batched_ms": round(t_learn * 1e3, 3),
        "plain_single_ms": round(t_single * 1e3, 3),
        "speedup_learned_vs_plain_batched": round(t_plain / t_learn, 3),
        "speedup_learned_vs_plain_single": round(t_single / t_learn, 3),
        "accepted": count - len(fb), "fallbacks": len(fb),
        "fallbacks_diffadv_burgers": [int((fb_kinds == 0).sum()), int((fb_kinds == 1).sum())],
        "plain_converged": int(sum(ok_p)),
        "learned_converged": int(sum(r["status"] == B.LX_OK for r in res_l)),
        "single_converged": int(sum(r["status"] == B.LX_OK for r in res_s)),
        "sweeps_plain_incl_power": int(sweeps_p), "sweeps_learned_incl_fallback_power": int(sweeps_l),
        "max_rel_diff_learned_vs_plain": max(diffs) if diffs else None,
        "median_rel_diff_learned_vs_plain": float(np.median(diffs)) if diffs else None,
        "largest_rel_diffs": largest,
        "tuned_shape": {"iterations_per_launch": best[0], "tile_rows": best[1], "points_per_workgroup": best[2]},
    }


def load_predictor(ctx, path=PREDICTOR_FILE):
    """A saved predictor and its margins (path and path with .json)."""
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
    a_all = sub.add_parser("all")
    a_all.add_argument("--records", type=int, default=100000)
    a_all.add_argument("--steps", type=int, default=20000)
    a_all.add_argument("--batch", type=int, default=512)
    a_all.add_argument("--lr", type=float, default=1e-3)
    a_all.add_argument("--calibration", type=int, default=4096)
    a_all.add_argument("--evaluate", type=int, default=1024)
    a_all.add_argument("--workers", type=int, default=12)
    a_all.add_argument("--out-dir", required=True)
    e = sub.add_parser("evaluate")
    e.add_argument("--predictor", default=PREDICTOR_FILE)
    e.add_argument("--count", type=int, default=1024)
    e.add_argument("--workers", type=int, default=12)
    e.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    # the pool forks before this process touches the GPU
    pool = mp.get_context("fork").Pool(args.workers) if args.workers > 1 else None
    from . import binding as B
    lib = B.Library.load()
    ctx = lib.context(n_max=1 << 16, k_max=1)
    if args.cmd == "all":
        os.makedirs(args.out_dir, exist_ok=True)
        t0 = time.perf_counter()
        X, Y, K = generate_records(ctx, args.records, SEED_RECORDS, pool=pool)
        t_rec = time.perf_counter() - t0
        np.savez(os.path.join(args.out_dir, "records.npz"), X=X, Y=Y, kind=K)
        p, summary = train_predictor(ctx, X, Y, args.steps, args.batch, args.lr)
        margin_s, cal = calibrate_budget(ctx, p, summary["margin_log_rho"], args.calibration, pool=pool)
        summary.update(cal)
        summary["records_seconds"] = round(t_rec, 1)
        summary["records_kept_diffadv_burgers"] = [int((K == 0).sum()), int((K == 1).sum())]
        summary["target_ranges"] = {"log_rho": [float(Y[:, 0].min()), float(Y[:, 0].max())],
                                    "log_sweeps": [float(Y[:, 1].min()), float(Y[:, 1].max())]}
        path = os.path.join(args.out_dir, "predictor.bin")
        p.save(path)
        summary["command"] = ("python -m paper_2310_08344_amd.learned all " +
                              " ".join(f"--{k.replace('_', '-')} {v}" for k, v in vars(args).items()
                                       if k != "cmd"))
        res = evaluate(ctx, p, (summary["margin_log_rho"], margin_s), count=args.evaluate, pool=pool)
        summary["evaluation"] = res
        with open(os.path.splitext(path)[0] + ".json", "w") as f:
            json.dump(summary, f, indent=1)
        _log(json.dumps(summary))
    else:
        p, margins, meta = load_predictor(ctx, args.predictor)
        res = evaluate(ctx, p, margins, count=args.count, pool=pool)
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
        _log(json.dumps(res))
    ctx.close()
    if pool is not None:
        pool.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
