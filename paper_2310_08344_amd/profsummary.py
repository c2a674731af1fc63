"""Summaries of rocprofv3 output for the sweep kernels.

Reads the CSV files that `rocprofv3 --kernel-trace --stats --output-format
csv -o run` and `rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE --output-format csv
-o run` write, and prints or writes:

* per-kernel call counts and durations, with the working launches of one
  kernel (duration above a threshold) separated from its early-exit launches;
* HBM bytes per working launch of one kernel from FETCH_SIZE and WRITE_SIZE
  (KiB per dispatch), each scaled by what the counter reads for the library's
  copy kernel of known size in the same run (`lx_bandwidth_probe`, 2^26 FP64
  elements: 512 MiB read and 512 MiB written).

    python -m paper_2310_08344_amd.profsummary stats DIR [--kernel leja_sweep] [--exit-us 20] [--max-us T]
    python -m paper_2310_08344_amd.profsummary traffic FETCH_DIR WRITE_DIR --points N
        [--kernel leja_sweep] [--algorithmic BYTES] [--max-bpp B] [--json OUT]
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics as st
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_08344_amd", "csrc")
# the sources the FP64 Leja kernels (one, two and more iterations per launch) are compiled from
SWEEP_SOURCES = ("kernels.hip", "pair.hip", "block.hip", "stream.hip", "tile_device.h", "sweep_device.h",
                 "window_device.h", "lx_device.h")
COPY_ELEMS = 1 << 26


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    s = name
    for pre in ("void ", "lx::(anonymous namespace)::", "lx::"):
        s = s.replace(pre, "")
    return s.split("(")[0]


def kernel_stats(d: str):
    rows = []
    with open(os.path.join(d, "run_kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append({"kernel": _short(r["Name"]), "calls": int(r["Calls"]),
                         "avg_us": float(r["AverageNs"]) / 1e3, "min_us": float(r["MinNs"]) / 1e3,
                         "max_us": float(r["MaxNs"]) / 1e3, "share": float(r["Percentage"])})
    return rows


def trace(d: str, kernel: str):
    """(start_ns, duration_ns) of every dispatch whose name contains `kernel`."""
    out = []
    with open(os.path.join(d, "run_kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            if kernel in r["Kernel_Name"]:
                s, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
                out.append((s, e - s))
    out.sort()
    return out


def split_launches(d: str, kernel: str, exit_us: float, max_us: float = float("inf")):
    t = trace(d, kernel)
    work = [x / 1e3 for _, x in t if exit_us <= x / 1e3 < max_us]
    idle = [x / 1e3 for _, x in t if x / 1e3 < exit_us]
    return work, idle


def _counter(d: str, cname: str):
    """{dispatch id: (kernel name, value summed over instances)}."""
    out = {}
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != cname:
                continue
            k = int(r["Dispatch_Id"])
            name, v = out.get(k, (r["Kernel_Name"], 0.0))
            out[k] = (name, v + float(r["Counter_Value"]))
    return out


def _values(c, kernel):
    return [v for _, (n, v) in sorted(c.items()) if kernel in n]


def traffic(fetch_dir: str, write_dir: str, kernel: str, points: int, exit_bytes_per_point: float = 1.0,
            max_bytes_per_point: float = float("inf")):
    f = _counter(fetch_dir, "FETCH_SIZE")
    w = _counter(write_dir, "WRITE_SIZE")
    cf, cw = _values(f, "copy_kernel"), _values(w, "copy_kernel")
    if not cf or not cw:
        raise SystemExit("no copy_kernel dispatch in the counter runs: cannot scale the counters")
    scale_f = COPY_ELEMS * 8 / (st.median(cf) * 1024)
    scale_w = COPY_ELEMS * 8 / (st.median(cw) * 1024)
    kf = [v * 1024 * scale_f for v in _values(f, kernel)]
    kw = [v * 1024 * scale_w for v in _values(w, kernel)]
    if len(kf) != len(kw):
        raise SystemExit(f"{kernel}: {len(kf)} FETCH dispatches but {len(kw)} WRITE dispatches")
    # working launches: those that moved at least exit_bytes_per_point bytes per point
    pairs = [(a, b) for a, b in zip(kf, kw) if exit_bytes_per_point * points <= a + b < max_bytes_per_point * points]
    return {
        "counter_scale": {"FETCH_SIZE": round(scale_f, 4), "WRITE_SIZE": round(scale_w, 4)},
        "working_launches": len(pairs),
        "hbm_bytes_per_launch": round(st.mean(a + b for a, b in pairs)) if pairs else None,
        "fetch_bytes_per_point": [round(a / points, 2) for a, _ in pairs],
        "write_bytes_per_point": [round(b / points, 2) for _, b in pairs],
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2310_08344_amd.profsummary")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--kernel", default="leja_sweep")
    s.add_argument("--exit-us", type=float, default=20.0)
    s.add_argument("--max-us", type=float, default=float("inf"),
                   help="count only working launches shorter than this (separates grid sizes)")
    s.add_argument("--list", action="store_true", help="also list the working launches' durations in order")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--points", type=int, required=True)
    t.add_argument("--kernel", default="leja_sweep")
    t.add_argument("--algorithmic", type=float, default=None, help="algorithmic bytes per working launch")
    t.add_argument("--max-bpp", type=float, default=float("inf"),
                   help="count only launches below this many bytes per point (separates grid sizes)")
    t.add_argument("--depth", type=int, default=None, help="iterations per launch of the profiled kernel")
    t.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print("| Kernel | Calls | Avg (us) | Min (us) | Max (us) | Share |")
        print("|---|---|---|---|---|---|")
        for r in kernel_stats(a.dir):
            print(f"| `{r['kernel']}` | {r['calls']} | {r['avg_us']:.2f} | {r['min_us']:.2f} | "
                  f"{r['max_us']:.2f} | {r['share']:.1f}% |")
        work, idle = split_launches(a.dir, a.kernel, a.exit_us, a.max_us)
        if work:
            band = f" below {a.max_us:g} us" if a.max_us != float("inf") else ""
            print(f"\n{a.kernel}: {len(work)} working launches{band}, average {st.mean(work):.2f} us, "
                  f"median {st.median(work):.2f} us; {len(idle)} early-exit launches"
                  + (f", average {st.mean(idle):.2f} us" if idle else ""))
            if a.list:
                print("durations (us, in launch order): " + " ".join(f"{x:.1f}" for x in work))
    else:
        r = traffic(a.fetch_dir, a.write_dir, a.kernel, a.points, max_bytes_per_point=a.max_bpp)
        r["kernel"] = a.kernel
        if a.depth is not None:
            r["depth"] = a.depth
        r["sweep_source_sha256"] = sweep_source_hash()
        if a.algorithmic and r["hbm_bytes_per_launch"]:
            r["algorithmic_bytes_per_launch"] = a.algorithmic
            r["ratio"] = round(r["hbm_bytes_per_launch"] / a.algorithmic, 4)
        txt = json.dumps(r, indent=1)
        if a.json:
            with open(a.json, "w") as f:
                f.write(txt + "\n")
        print(txt)
    return 0


if __name__ == "__main__":
    sys.exit(main())
