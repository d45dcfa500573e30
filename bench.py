"""Benchmark of the bidirectional subset-BFS hot path on one MI355X.

A step is one pass of the whole hot path (expand, dedup, compact, transpose,
meet, traceback, verify) over one batch of seeded synthetic automata.  The
default workload is n=256, k=2 random automata (10 seeds) plus the Černý
automata C_16..C_32, solved together through srw_solve_batch.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  `value` is subsets expanded per second (k * |list|
per expansion step, summed over all automata) of the batched path; the same
line carries automata/s of the batched and of the one-at-a-time path,
per-solve latency percentiles, the roofline of the dominant kernel (timed
with HIP events on the library's stream) and the CPU oracle baseline.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2207_05495_amd import inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0
# int32 VALU lane-ops/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

CLASSES = ("expand", "insert", "compact", "prep", "meet", "trace", "setup")


def workload(name, srw):
    """List of (n, k, delta, label)."""
    out = []
    if name == "config2":
        for i in range(10):
            d, _ = I.first_synchronizing(256, 2, I.member_seed(I.BASE_SEED, i), srw.check_sync)
            out.append((256, 2, d, f"rand256#{i}"))
        for n in range(16, 33):
            out.append((n, 2, I.cerny(n), f"cerny{n}"))
    elif name == "config1":
        for i in range(100):
            d, _ = I.first_synchronizing(64, 2, I.member_seed(I.BASE_SEED, i), srw.check_sync)
            out.append((64, 2, d, f"rand64#{i}"))
    elif name == "config4":
        d, _ = I.first_synchronizing(450, 2, I.member_seed(I.BASE_SEED, 0), srw.check_sync)
        out.append((450, 2, d, "rand450#0"))
    else:
        raise SystemExit(f"unknown workload {name}")
    return out


def oracle_one(path):
    """Child process: solve one automaton with the oracle, print its stats."""
    from oracle import oracle as O
    z = np.load(path)
    n, k, d = int(z["n"]), int(z["k"]), z["d"]
    t = time.perf_counter()
    r, _, info = O.bidir(n, k, d)
    print(json.dumps({"r": r, "candidates": info["candidates"], "s": time.perf_counter() - t}))


def cpu_baseline(probs, budget_s):
    """The oracle (single-threaded C, Alg. 2 meet) on a bounded sample of the
    workload: the random members in order, then the Černý ones, each in
    a child process that is stopped when the budget runs out (a stopped
    member is left out of the sample).  Runs before the GPU is touched."""
    import subprocess
    import tempfile
    order = sorted(range(len(probs)), key=lambda i: probs[i][3].startswith("cerny"))
    t0 = time.perf_counter()
    cand, busy = 0, 0.0
    solved = []
    with tempfile.TemporaryDirectory() as tmp:
        for i in order:
            left = budget_s - (time.perf_counter() - t0)
            if left <= 0.5:
                break
            n, k, d, label = probs[i]
            path = os.path.join(tmp, f"m{i}.npz")
            np.savez(path, n=n, k=k, d=d)
            try:
                res = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one", path],
                                     capture_output=True, text=True, timeout=left, check=True)
            except subprocess.TimeoutExpired:
                break
            out = json.loads(res.stdout.strip().splitlines()[-1])
            cand += out["candidates"]
            busy += out["s"]
            solved.append(label)
    return {"value": cand / busy if busy else None, "unit": "subsets expanded/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{len(solved)} of {len(probs)} automata solved one by one in "
                      f"{busy:.1f} s of oracle time ({', '.join(solved[:3])}, ..., {solved[-1]})"
                      if solved else "none finished within the budget",
            "automata_per_s": len(solved) / busy if busy else None}


def roofline(stats, probs):
    """Roofline of the kernel class with the most time in the timed region."""
    ms = stats["ms"]
    launches = stats["launches"]
    dom = max(CLASSES[:6], key=lambda c: ms[c])
    t = ms[dom] / max(1, launches[dom]) / 1e3     # seconds per launch
    nl = max(1, launches[dom])
    if dom == "meet":
        # algorithmic unit: pair-word tests |L_f| * |L_b| * W (brute force);
        # one test is two 32-bit lane-ops
        ops = 2.0 * stats["pair_words"] / nl
        ach = ops / t / 1e12
        return {"kernel": "k_meet", "bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS,
                "unit": "TOP/s", "frac": ach / VALU_PEAK_TOPS, "traffic": None,
                "per_launch_ms": t * 1e3, "launches": launches[dom]}
    byts = {"expand": stats["bytes_expand"], "insert": stats["bytes_insert"],
            "compact": stats["bytes_compact"]}.get(dom)
    if byts is None:
        return {"kernel": dom, "bound": "latency", "achieved": None, "peak": None,
                "unit": None, "frac": None, "traffic": None, "per_launch_ms": t * 1e3}
    ach = byts / nl / t / 1e9
    return {"kernel": "k_" + dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
            "per_launch_ms": t * 1e3, "launches": launches[dom]}


def class_table(stats):
    out = {}
    for c in CLASSES:
        nl = stats["launches"][c]
        if nl:
            out[c] = {"ms": round(stats["ms"][c], 3), "launches": nl}
    gb = {"expand": stats["bytes_expand"], "insert": stats["bytes_insert"],
          "compact": stats["bytes_compact"]}
    for c, b in gb.items():
        if c in out and stats["ms"][c] > 0:
            out[c]["GBps"] = round(b / (stats["ms"][c] / 1e3) / 1e9, 1)
            out[c]["hbm_frac"] = round(b / (stats["ms"][c] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config2")
    ap.add_argument("--cpu-budget", type=float, default=40.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--oracle-one", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_one:
        oracle_one(args.oracle_one)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the search of one automaton is not sharded "
              "across GPUs in this library (see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2207_05495_amd import srw
    probs = workload(args.workload, srw)          # host-only calls so far
    cpu = None if args.no_cpu else cpu_baseline(probs, args.cpu_budget)

    import torch
    torch.cuda.set_device(0)
    srw.use_torch(0)
    batch = [(n, k, d) for n, k, d, _ in probs]
    print(f"workload {args.workload}: {len(probs)} automata", file=sys.stderr, flush=True)

    if args.calib_copy_mb:
        a = torch.empty(args.calib_copy_mb << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    srw.set_option("profile", 0)
    for _ in range(args.warmup):
        res = srw.solve_batch(batch)
        assert all(st == 0 for st, _, _ in res), res
    srw.reset_stats()
    srw.set_option("profile", 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        res = srw.solve_batch(batch)
        print(f"step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    srw.set_option("profile", 0)
    for st, r, w in res:
        assert st == 0
    stats = srw.get_stats()
    per_step = dt / args.steps
    cand = stats["candidates"] / args.steps
    out = {
        "metric": "subsets expanded/s + automata solved/s (batched vs plain, 1 GPU), p99 latency",
        "value": cand / per_step,
        "unit": "subsets expanded/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": per_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload,
                   "automata": len(probs),
                   "sizes": sorted({(n, k) for n, k, _, _ in probs if n > 40})
                   if args.workload != "config2" else
                   "10 x random n=256 k=2 (uniform delta, seeded SplitMix64) + Cerny C_16..C_32",
                   "path": "srw_solve_batch"},
        "automata_per_s": len(probs) / per_step,
        "subsets_per_step": cand,
        "pairs_per_step": stats["pairs"] / args.steps,
        "kernels": class_table(stats),
        "roofline": roofline(stats, probs),
    }
    if not args.no_plain:
        lat = []
        srw.reset_stats()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for n, k, d in batch:
            a = time.perf_counter()
            srw.solve(n, k, d)
            lat.append((time.perf_counter() - a) * 1e3)
        torch.cuda.synchronize()
        plain = time.perf_counter() - t1
        out["plain"] = {"automata_per_s": len(batch) / plain,
                        "subsets_per_s": srw.get_stats()["candidates"] / plain,
                        "p50_ms": float(np.percentile(lat, 50)),
                        "p99_ms": float(np.percentile(lat, 99))}
        out["batched_over_plain"] = out["automata_per_s"] / out["plain"]["automata_per_s"]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
