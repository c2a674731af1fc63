#!/usr/bin/env python
"""Benchmark of the Leja phi-action hot path on one MI355X.

One step = power iteration (20 sweeps) for the spectral bound, then the
phi_1, phi_2, phi_3 actions of a seeded N(0,1) vector from one Newton basis
on the periodic 4096^2 diffusion-advection grid (D = 1, cell Peclet 1,
h = 50 x CFL, rtol 1e-8), all through the C ABI.  Inputs are resident in
HBM before the timed region.  Before it, the launch shapes of this grid are
autotuned (lx_tune) and the practical bandwidth is calibrated with plain
copy and z = a x + b y kernels on vectors larger than the Infinity Cache.

Prints one JSON line on stdout:
  value         phi-action solves/s (3 solves per step)
  roofline      HBM roofline of the dominant kernel (the fused Leja sweep):
                algorithmic bytes per launch / average launch duration, both
                from HIP events recorded on the library's stream around
                every sweep of the timed steps; traffic from the committed
                rocprofv3 counter summary when it was taken on the current
                kernel source, else null
  small_configs the 64^2 exp workload (rtol 1e-10) and the 1024^2 phi_1..phi_3
                workload (rtol 1e-8): solves/s, time to solution
  batched_256   256 uneven instances in one batched call against the plain
                per-instance path (both with power iteration), the tuned
                batch shape, a whole-call roofline
  learned_1024  the learned + batched form against plain batched and plain
                per-instance solves on 1024 instances at 256^2
  exprb42_2048  one EXPRB42 step of the 2048^2 Burgers workload, FP64 and
                FP32 sweeps
  paper_problems_8192
                the paper's linear test problems (Sec. 3, Problems I and II:
                nu = 10, third-order upwind gradient, tolerance 1e-12) at
                8192^2 for h = 1, 10, 100 x CFL to the paper's final times,
                with the algorithmic bandwidth over the whole time loop as a
                fraction of the practical peak measured in the same run
  cpu_baseline  the CPU oracle on a bounded sample of the same 4096^2 solve
                (a few power sweeps, the full planner, the Leja loop forced
                to a few iterations with three outputs and with one), scaled
                to the GPU run's iteration counts; one thread and all cores

Usage: python bench.py [--steps K] [--warmup W] [--no-tune] [--no-calibrate] [--no-batched] [--no-learned]
                       [--no-exprb] [--no-paper] [--no-small] [--no-cpu-baseline] [--window-kernel 0|1|2]
                       [--depth D] [--tune-sweeps S]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of the dominant kernel from rocprofv3 counters, per kernel family
TRAFFIC_FILES = {"leja_stream": os.path.join(ROOT, "profiles", "leja_stream_phi123_4096_traffic.json")}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def committed_traffic(launch_bytes: float, family: str, depth: int):
    """HBM bytes per launch of the sweep from the committed counter summary,
    if it was taken on the current kernel source at the same depth."""
    if family not in TRAFFIC_FILES:
        return None
    try:
        with open(TRAFFIC_FILES[family]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2310_08344_amd.profsummary import sweep_source_hash
    if t.get("sweep_source_sha256") != sweep_source_hash() or t.get("depth") != depth:
        return None
    return {"bytes_per_launch": t["hbm_bytes_per_launch"], "ratio_to_algorithmic":
            round(t["hbm_bytes_per_launch"] / launch_bytes, 4) if launch_bytes else None}


def cpu_baseline(n: int, gpu_iters, power_iters: int = 20, power_sample: int = 4, leja_sample: int = 8) -> dict:
    """The oracle as it stands, timed on this host at the benchmarked grid
    (n^2, the same seeded v and operator), once on one thread and once with
    every visible core allowed to its thread pools.

    Bounded sample: power_sample power sweeps, the planner for the full
    run's 301 coefficients per output, and two runs of the Leja loop forced
    to leja_sample iterations, one with all three outputs taking terms and
    one with only phi_1 (phi_2 and phi_3 stop after their first term).  Per
    iteration the loop then costs a + b k with k outputs taking terms; the
    full solve is power_iters sweeps + the planner + the sum over the GPU
    run's iterations of a + b k(m) (k(m) from its per-output counts)."""
    from threadpoolctl import threadpool_limits

    from oracle.leja import leja_points, newton_coeffs
    from oracle.operators import make_apply
    from oracle.phi_action import leja_phi, power_iteration, shift_scale
    from paper_2310_08344_amd import workloads as W

    p, v = W.config2(n=n)
    x0 = W.start_vector(p.n)
    A = make_apply(p)
    outs = [(1, 1.0, 1.0), (2, 1.0, 1.0), (3, 1.0, 1.0)]
    max_iters = 300
    cores = len(os.sched_getaffinity(0))
    leja_points(max_iters + 1)   # the Leja table, built once (as the library does per context)

    def sample(threads):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            rho, _ = power_iteration(A, x0, power_sample)
            t_pw = (time.perf_counter() - t0) / power_sample
            c, g = shift_scale(rho)
            t0 = time.perf_counter()
            for (l, a, sg) in outs:
                newton_coeffs(l, p.h, c, g, max_iters + 1, alpha=a, sigma=sg)
            t_plan = time.perf_counter() - t0
            t0 = time.perf_counter()
            leja_phi(A, v, outs, p.h, c, g, 1e-8, 0.0, max_iters, force_iters=[leja_sample] * 3)
            t3 = time.perf_counter() - t0 - t_plan
            t0 = time.perf_counter()
            leja_phi(A, v, outs, p.h, c, g, 1e-8, 0.0, max_iters, force_iters=[leja_sample, 1, 1])
            t1 = time.perf_counter() - t0 - t_plan
        b = max(0.0, (t3 - t1) / (2.0 * (leja_sample - 1)))
        a = max(0.0, t3 / leja_sample - 3.0 * b)
        loop = sum(a + b * sum(1 for it in gpu_iters if m < it) for m in range(max(gpu_iters)))
        total = power_iters * t_pw + t_plan + loop
        return {"seconds_per_solve_set": round(total, 3), "power_sweep_s": round(t_pw, 4),
                "planner_s": round(t_plan, 3), "iteration_s_base_per_output": [round(a, 4), round(b, 4)]}

    one = sample(1)
    allc = sample(cores)
    return {"value": round(3.0 / one["seconds_per_solve_set"], 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"the oracle on this workload at {n}^2 (same operator and seeded v): {power_sample} power "
                       f"sweeps, the planner for 301 coefficients per output, and the Leja loop forced to "
                       f"{leja_sample} iterations with three outputs and with one; scaled to {power_iters} power "
                       f"sweeps and the GPU run's iteration counts {list(gpu_iters)} (no grid scaling)"),
            "one_thread": one,
            "all_cores": dict(allc, threads_allowed=cores,
                              value=round(3.0 / allc["seconds_per_solve_set"], 4),
                              note="numpy runs the oracle's elementwise stencil arithmetic on one thread; only "
                                   "library calls (norms) may use the wider pool")}


def bench_small_configs(lib, repeats: int = 20, warmups: int = 3) -> dict:
    """The two other single-instance workloads, time to solution (power
    iteration 20 sweeps + planner + Leja loop), median of `repeats` after
    `warmups`: exp(hA)u on the 64^2 Gaussian workload at rtol 1e-10 (1 solve
    per step) and phi_1..phi_3 of a seeded N(0,1) v on 1024^2 at rtol 1e-8
    (3 solves per step; launch shapes tuned first).  Both working sets fit
    in the 256 MB Infinity Cache, so `effective_gbs` (algorithmic bytes of
    the power and Leja launches over the step's time) is not an HBM rate."""
    import torch

    from paper_2310_08344_amd import binding as B
    from paper_2310_08344_amd import workloads as W

    dev = torch.device("cuda:0")
    res = {}
    for name, (p, v_h), ls, rtol in (("c1_64_exp", W.config1(), [0], 1e-10),
                                     ("c2_1024_phi123", W.config2(n=1024), [1, 2, 3], 1e-8)):
        ctx = lib.context(n_max=p.N, k_max=len(ls))
        try:
            op = B.make_operator(p)
            if len(ls) > 1:
                ctx.tune(op, K=len(ls), sweeps=8)
            v = torch.as_tensor(v_h).to(dev)
            x0 = torch.as_tensor(W.start_vector(p.n)).to(dev)
            outs = [torch.empty_like(v) for _ in ls]
            stats = []

            def step():
                _, c, g = ctx.spectrum(op, x0=x0, iters=20)
                sp = ctx.stats()
                r = ctx.phi_leja(op, v, outs, ls, p.h, c, g, rtol=rtol, max_iters=300)
                if r.status != B.LX_OK:
                    raise RuntimeError(f"phi_leja status {r.status}: {ctx.last_error()}")
                stats.append((sp["bytes"], r.stats["bytes"], r.iters))

            for _ in range(warmups):
                step()
            ts = []
            for _ in range(repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                step()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            t = float(np.median(ts))
            pb, lb, its = stats[-1]
            res[name] = {"grid": p.n, "rtol": rtol, "outputs": len(ls), "solves_per_s": round(len(ls) / t, 1),
                         "ms_per_step": round(t * 1e3, 4), "sweeps": list(its)[:len(ls)],
                         "effective_gbs": round((pb + lb) / t / 1e9, 1),
                         "timing": f"median of {repeats} after {warmups} warm-ups, wall time of the whole step"}
            log(name, res[name])
        finally:
            ctx.close()
    return res


def bench_batched(lib, repeats: int = 10, warmups: int = 3, tune: bool = True) -> dict:
    """256 uneven diffusion-advection instances (sides 64..512), exp action
    at rtol 1e-8 with 20 power-iteration sweeps each: one batched call
    against the plain path (lx_spectrum + lx_phi_leja per instance)."""
    import torch

    from paper_2310_08344_amd import binding as B
    from paper_2310_08344_amd import workloads as W

    items = W.batched_instances()
    dev = torch.device("cuda:0")
    vs = [torch.as_tensor(u0).to(dev) for _, u0 in items]
    outs = [torch.empty_like(v) for v in vs]
    ops = [B.make_operator(p) for p, _ in items]
    ctx = lib.context(n_max=max(p.N for p, _ in items), k_max=1)
    args = [dict(op=op, v=v, out=o, l=0, h=p.h) for op, v, o, (p, _) in zip(ops, vs, outs, items)]

    def plain():
        for op, v, o, (p, _) in zip(ops, vs, outs, items):
            _, c, g = ctx.spectrum(op, iters=20)
            ctx.phi_leja(op, v, [o], [0], p.h, c, g, rtol=1e-8, max_iters=300)

    def batched():
        st, res = ctx.phi_leja_batched(args, power_iters=20, rtol=1e-8, max_iters=300)
        if st != B.LX_OK:
            raise RuntimeError(f"batched status {st}")
        return res

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    # the batch's launch shape from the autotuner (this batch class: 256
    # diffusion-advection instances with sides 64..512)
    # (without tuning: the shape LX_TUNE_CACHE holds for this class, else the default rule)
    tuned = ctx.tune_batched(args, power_iters=20, rtol=1e-8, max_iters=300, repeats=3) if tune else []
    best = min(tuned, key=lambda r: r[3]) if tuned else (0, 0, 0, None)
    log("batch tuner:", " ".join(f"{d}/{th}/{ppw}:{ms:.2f}" for d, th, ppw, ms in tuned))
    for _ in range(warmups):
        plain()
        res = batched()
    tp, tb = [], []
    for _ in range(repeats):
        tp.append(timed(plain)[1])
        res, t = timed(batched)
        tb.append(t)
    t_plain, t_batch = float(np.median(tp)), float(np.median(tb))
    st = ctx.stats()
    ctx.close()
    iters = sorted(r["iters"] for r in res)
    return {"workload": "256 diffusion-advection instances, sides uniform in {64,128,256,512}, D ~ LogU(0.1,10), "
                        "|v| ~ U(0,5), h = s x CFL with s ~ LogU(1,50), exp action, rtol 1e-8, 20 power sweeps",
            "points": int(sum(p.N for p, _ in items)),
            "batched_solves_per_s": round(len(items) / t_batch, 1),
            "plain_solves_per_s": round(len(items) / t_plain, 1),
            "batched_ms": round(t_batch * 1e3, 3), "plain_ms": round(t_plain * 1e3, 3),
            "speedup_batched_vs_plain": round(t_plain / t_batch, 2),
            "timing": f"median of {repeats} after {warmups} warm-ups, each path timed whole (power iteration, "
                      "planner and Leja loop)",
            "tuned_shape": {"iterations_per_launch": best[0], "tile_rows": best[1], "points_per_workgroup": best[2],
                            "tuner_median_ms": best[3], "candidates": len(tuned)},
            "captured_graph_replayed": bool(st["batch_graph"]),
            "roofline": {"bound": "hbm", "achieved": round(st["bytes"] / t_batch / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(st["bytes"] / t_batch / 1e9 / HBM_PEAK_GBS, 4),
                         "bytes_per_call": st["bytes"],
                         "note": "algorithmic bytes of the whole batched call (power sweeps 16 B/pt each, windows "
                                 "as the single-instance kernel) over its median wall time, planner and host "
                                 "polling included; the per-kernel rates are in the committed profiles"},
            "sweeps_min_median_max": [iters[0], iters[len(iters) // 2], iters[-1]]}


def bench_learned(lib, count: int = 1024, tune: bool = True) -> dict:
    """The learned + batched form against the plain batched and plain
    single-instance paths on 1024 instances at 256^2 (half
    diffusion-advection, half Burgers), with the committed predictor."""
    from paper_2310_08344_amd import learned as L

    ctx = lib.context(n_max=1 << 16, k_max=1)
    p, margins, meta = L.load_predictor(ctx)
    res = L.evaluate(ctx, p, margins, count=count, tune=tune)
    ctx.close()
    res["predictor"] = {"records": meta.get("records"), "val_rmse_log_rho": meta.get("val_rmse_log_rho"),
                        "val_rmse_log_sweeps": meta.get("val_rmse_log_sweeps"),
                        "margins": [round(margins[0], 4), round(margins[1], 4)]}
    return res


# final times of the paper's 2^13 runs for h = 1, 10, 100 x CFL (Sec. 3,
# table of Problems I and II)
PAPER_RUNS_8192 = ((1.0, 2e-7), (10.0, 2e-6), (100.0, 2e-5))


# the paper's time-to-solution runs on one A100 (Sec. 3, table of speedups):
# 2^14 grid, T_f = 2e-6, h = 100 x CFL; its GPU seconds for Problems I and II
PAPER_RUNS_16384 = ((100.0, 2e-6),)
PAPER_A100_SECONDS_16384 = {"I": 4.76, "II": 4.14}


def bench_paper_problems(lib, n: int = 8192, axpby_gbs=None, tune: bool = True, runs=PAPER_RUNS_8192) -> dict:
    """Problems I (exp action) and II (phi_1 with a source) on n^2 with the
    third-order upwind operator: for each step size, power iteration once
    (A is constant), then the time loop to the paper's final time, timed as
    a whole.  Bytes are the kernels' algorithmic bytes: the spectrum
    (16 B/pt per sweep), the Leja loops (lx_stats.bytes), and for Problem II
    the right-hand side h (A u + S) (24 B/pt) and the sum u + phi (24 B/pt)."""
    import torch

    from paper_2310_08344_amd import binding as B
    from paper_2310_08344_amd import workloads as W

    dev = torch.device("cuda:0")
    ctx = lib.context(n_max=n * n, k_max=1)
    res = {"grid": n, "tolerance": 1e-12, "runs": []}
    try:
        p0, u0_h, S_h = W.paper_linear(n, 1.0, True)
        op = B.make_operator(p0)
        if tune:
            best = min(ctx.tune(op, K=1, sweeps=8), key=lambda r: r[6])
            res["tuned"] = {"depth": best[0], "rows": best[3], "workgroups": best[5],
                            "us_per_iteration": round(best[6], 2)}
        u0 = torch.as_tensor(u0_h).to(dev)
        S = torch.as_tensor(S_h).to(dev)
        del u0_h, S_h
        x0 = torch.as_tensor(W.start_vector(n)).to(dev)
        ua, ub = torch.empty_like(u0), torch.empty_like(u0)
        N = float(n * n)
        for source in (False, True):
            for cfl, t_final in runs:
                h = cfl * p0.h   # p0.h is one CFL step
                steps = max(1, round(t_final / h))
                # untimed warm-up step (planner tables, code paths)
                _, c, g = ctx.spectrum(op, x0=x0, iters=20)
                ctx.linear_step(op, u0, ua, h, c, g, source=S if source else None, rtol=1e-12, max_iters=1000)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, c, g = ctx.spectrum(op, x0=x0, iters=20)
                nbytes = 16.0 * N * 20
                nbytes1 = 16.0 * N * 20   # the same iterations one per launch
                iters = []
                cur, nxt = u0, ua
                for k in range(steps):
                    r = ctx.linear_step(op, cur, nxt, h, c, g, source=S if source else None, rtol=1e-12,
                                        max_iters=1000)
                    if r.status != B.LX_OK:
                        raise RuntimeError(f"linear_step status {r.status}: {ctx.last_error()}")
                    iters.append(r.iters[0])
                    nbytes += r.stats["bytes"] + (48.0 * N if source else 0.0)
                    nbytes1 += N * (24.0 + 32.0 * (r.iters[0] - 1)) + (48.0 * N if source else 0.0)
                    cur, nxt = nxt, (ub if nxt is ua else ua)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                gbs = nbytes / dt / 1e9
                run = {"problem": "II" if source else "I", "h_cfl": cfl, "t_final": t_final, "steps": steps,
                       "iters_first_last": [iters[0], iters[-1]], "seconds": round(dt, 4),
                       "ms_per_step": round(dt * 1e3 / steps, 3), "gbs": round(gbs, 1),
                       "frac_of_8tbs": round(gbs / HBM_PEAK_GBS, 4),
                       "gbs_one_iteration_bytes": round(nbytes1 / dt / 1e9, 1)}
                if axpby_gbs:
                    run["frac_of_practical_axpby"] = round(gbs / axpby_gbs, 4)
                    run["one_iteration_bytes_frac_of_practical_axpby"] = round(nbytes1 / dt / 1e9 / axpby_gbs, 4)
                if n == 16384 and cfl == 100.0:
                    run["paper_a100_seconds"] = PAPER_A100_SECONDS_16384[run["problem"]]
                res["runs"].append(run)
                log("paper problem", run)
    finally:
        ctx.close()
    res["note"] = ("gbs: this library's algorithmic bytes (several Leja iterations per launch read and write the "
                   "basis and the output once) over the wall time of the whole loop; gbs_one_iteration_bytes: the "
                   "bytes the same iterations move one per launch (32 B/pt each), over the same time; the paper's "
                   "A100 figures (0.87-0.92 of its practical z = ax + by bandwidth at 2^13, and its seconds at "
                   "2^14, Sec. 3) are context, not a like-for-like ratio")
    return res


def bench_exprb42(lib, n: int = 2048, repeats: int = 5, tune: bool = True) -> dict:
    """One EXPRB42 step of the 2048^2 Burgers workload (nu = 1e-3, four
    Fourier modes, h = 10 x CFL of the Jacobian, tolerance 1e-8), power
    iteration included: FP64 sweeps (windows after tuning) and FP32 sweeps;
    the FP32 update's relative difference from the FP64 one."""
    import torch

    from paper_2310_08344_amd import binding as B
    from paper_2310_08344_amd import workloads as W

    p, u0_h = W.config3(n=n)
    dev = torch.device("cuda:0")
    u0 = torch.as_tensor(u0_h).to(dev)
    x0 = torch.as_tensor(W.start_vector(n)).to(dev)
    out64, out32 = torch.empty_like(u0), torch.empty_like(u0)
    ctx = lib.context(n_max=n * n, k_max=2)
    res = {"workload": f"periodic viscous Burgers {n}^2, nu = 1e-3, u0 = 4 seeded Fourier modes, one EXPRB42 step "
                       "h = 10 x CFL, tolerance 1e-8, 20 power sweeps", "grid": n}
    try:
        op = B.make_operator(p)
        op32 = B.make_operator(p)
        op32.prec = B.LX_FP32_SWEEP
        for K in (2, 1) if tune else ():
            ctx.tune(op, K=K, sweeps=24)
            ctx.tune(op32, K=K, sweeps=24)

        def step(o, out):
            _, c, g = ctx.spectrum(o if o.prec == B.LX_FP64 else op, u=u0, x0=x0, iters=20)
            r = ctx.exprb_step(o, u0, out, p.h, c, g, rtol=1e-8, max_iters=300)
            if r.status != B.LX_OK:
                raise RuntimeError(f"exprb_step status {r.status}: {ctx.last_error()}")
            return r

        for name, o, out in (("fp64", op, out64), ("fp32_sweeps", op32, out32)):
            r = step(o, out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(repeats):
                r = step(o, out)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / repeats
            res[name] = {"ms_per_step": round(dt * 1e3, 3), "iters_phi1_phi3": list(r.iters),
                         "depth": r.stats["depth"], "register_marching": bool(r.stats["marching"]),
                         "fp32_levels": r.stats["n_fp32"]}
        du64 = out64 - u0
        res["fp32_update_rel_diff_vs_fp64"] = float(torch.linalg.norm(out32 - out64) / torch.linalg.norm(du64))
    finally:
        ctx.close()
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096, help="grid side of the phi_1..phi_3 workload")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-calibrate", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-shaped 8192^2 problems")
    ap.add_argument("--no-small", action="store_true", help="skip the 64^2 and 1024^2 workloads")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned + batched comparison")
    ap.add_argument("--no-exprb", action="store_true", help="skip the EXPRB42 Burgers step")
    ap.add_argument("--window-kernel", type=int, default=0, choices=(0, 1, 2),
                    help="kernel of the windows: 0 tuned, 1 LDS tiles, 2 register marching")
    ap.add_argument("--depth", type=int, default=0, help="Leja iterations per launch (0: tuned)")
    ap.add_argument("--tune-sweeps", type=int, default=24, help="Leja iterations each tuning candidate is timed on")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the phi-action path is single-GPU (--gpus {args.gpus} "
              "is not supported; the design notes describe how it would shard)", file=sys.stderr)
        return 2

    import torch

    from paper_2310_08344_amd import binding as B
    from paper_2310_08344_amd import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    lib = B.Library.load()
    p, v_h = W.config2(n=args.n)
    log("workload n", p.n, "h", p.h)
    dev = torch.device("cuda:0")
    v = torch.as_tensor(v_h).to(dev)
    x0 = torch.as_tensor(W.start_vector(p.n)).to(dev)
    outs = [torch.empty_like(v) for _ in range(3)]
    ctx = lib.context(n_max=max(p.N, 1 << 22), k_max=4)
    op = B.make_operator(p)
    ls = [1, 2, 3]
    torch.cuda.synchronize()

    extra = {}
    if not args.no_calibrate:
        n_cal = 1 << 26   # 512 MiB per vector: beyond the 256 MB Infinity Cache
        extra["practical_copy_gbs"] = round(ctx.bandwidth_probe(0, n_cal, 10), 1)
        extra["practical_axpby_gbs"] = round(ctx.bandwidth_probe(1, n_cal, 10), 1)
        log("calibration copy", extra["practical_copy_gbs"], "axpby", extra["practical_axpby_gbs"], "GB/s")
    if not args.no_tune:
        for K in (3, 2, 1):
            best = min(ctx.tune(op, K=K, sweeps=args.tune_sweeps), key=lambda r: r[6])
            log(f"tuned K={K}: depth {best[0]} tx {best[1]} ty {best[2]} rows {best[3]} vec {best[4]} "
                f"workgroups {best[5]} {best[6]:.1f} us per iteration")

    if args.window_kernel or args.depth:
        ctx.set_window_kernel(args.window_kernel)
        ctx.set_depth(args.depth)
        log("forced window kernel", args.window_kernel, "depth", args.depth)

    def step():
        rho, c, g = ctx.spectrum(op, x0=x0, iters=20)
        sp = ctx.stats()
        r = ctx.phi_leja(op, v, outs, ls, p.h, c, g, rtol=1e-8, max_iters=300)
        if r.status != B.LX_OK:
            raise RuntimeError(f"phi_leja status {r.status}: {ctx.last_error()}")
        return sp, r.stats

    for i in range(args.warmup):
        step()
        log("warmup step", i + 1, "done")
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for i in range(args.steps):
        recs.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_timing(False)
    log("timed steps done")
    dt = (t1 - t0) / args.steps
    value = 3.0 / dt

    launches = sum(r["n_launch"] for _, r in recs)
    sweep_ms = sum(r["sweep_ms"] for _, r in recs)
    leja_bytes = sum(r["bytes"] for _, r in recs)
    achieved = leja_bytes / (sweep_ms * 1e-3) / 1e9
    pw_ms = sum(s["sweep_ms"] for s, _ in recs)
    pw_bytes = sum(s["bytes"] for s, _ in recs)
    last = recs[-1][1]
    per_launch = leja_bytes / launches
    depth = last["depth"]
    # the bytes the same iterations move one per launch (y in and out, and
    # each output still iterating in and out; the first sweep only writes p)
    n_pts = float(p.n) ** 2
    one_iter_bytes = 0.0
    for _, r in recs:
        its = r["iters"][:3]
        for m in range(max(its)):
            one_iter_bytes += n_pts * (16.0 + sum((8.0 if m == 0 else 16.0) for i in its if m < i))
    traffic = committed_traffic(per_launch, "leja_stream" if last["marching"] else
                                ("leja_block" if depth >= 3 else "other"), depth)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "kernel": (f"{'leja_stream_deep' if depth >= 7 else 'leja_stream'} (diffusion-advection, K=3, FP64, "
                       f"register-marching windows of {depth} iterations)" if last["marching"] else
                       {2: "leja_pair (diffusion-advection, K=3, FP64, two iterations per launch)",
                        3: "leja_block (diffusion-advection, K=3, FP64, windows of three iterations)",
                        4: "leja_block (diffusion-advection, K=3, FP64, windows of four iterations)",
                        6: "leja_block (diffusion-advection, K=3, FP64, windows of six iterations)"}.get(
                           depth, "leja_sweep (diffusion-advection, K=3, FP64)")),
            "launches": launches, "avg_launch_us": round(sweep_ms * 1e3 / launches, 2),
            "iterations_per_launch": depth,
            "one_iteration_equivalent_gbs": round(one_iter_bytes / (sweep_ms * 1e-3) / 1e9, 1),
            "cache_note": "the outputs stream with nontemporal hints and the basis vector a launch reads (8 of the "
                          "64 bytes per point of a window) is mostly served by the 256 MB Infinity Cache; the L2 "
                          "traffic counters count it as memory traffic",
            "bytes_per_launch": per_launch}
    if traffic:
        roof["traffic_ratio_to_algorithmic"] = traffic["ratio_to_algorithmic"]
    out = {
        "metric": "phi-action solves/s at tol 1e-8",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"periodic diffusion-advection {p.n}^2, phi_1..phi_3 of seeded N(0,1) v from one "
                               f"Newton basis, h = 50 x CFL, rtol 1e-8, power iteration 20 sweeps",
                   "grid": p.n, "outputs": 3, "rtol": 1e-8, "power_iters": 20},
        "hbm_gbs_leja": round(achieved, 1),
        "hbm_gbs_power": round(pw_bytes / (pw_ms * 1e-3) / 1e9, 1) if pw_ms > 0 else None,
        "sweeps": last["iters"][:3],
        "plan_ms": round(last["plan_ms"], 3),
        "roofline": roof,
    }
    out.update({k: v for k, v in extra.items() if v is not None})
    ctx.close()
    if not args.no_small:
        log("64^2 exp and 1024^2 phi_1..phi_3 workloads")
        out["small_configs"] = bench_small_configs(lib)
    if not args.no_batched:
        log("batched 256-instance comparison")
        out["batched_256"] = bench_batched(lib, tune=not args.no_tune)
    if not args.no_batched and not args.no_learned:
        log("learned + batched on 1024 instances at 256^2")
        out["learned_1024"] = bench_learned(lib, tune=not args.no_tune)
    if not args.no_exprb:
        log("EXPRB42 step on the 2048^2 Burgers workload")
        out["exprb42_2048"] = bench_exprb42(lib, tune=not args.no_tune)
    if not args.no_paper:
        log("paper-shaped problems I and II at 8192^2")
        out["paper_problems_8192"] = bench_paper_problems(lib, axpby_gbs=extra.get("practical_axpby_gbs"),
                                                          tune=not args.no_tune)
        log("paper-shaped problems I and II at 16384^2 (time to solution)")
        out["paper_problems_16384"] = bench_paper_problems(lib, n=16384, axpby_gbs=extra.get("practical_axpby_gbs"),
                                                           tune=not args.no_tune, runs=PAPER_RUNS_16384)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(p.n, last["iters"][:3])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
