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


def workload(name, srw, count=None, nmax=None):
    """List of (n, k, delta, label)."""
    out = []
    if name == "mix4096-n32-320-k2-3":
        # the seeded 4096-member batch: n uniform in [32, 320], k in {2, 3};
        # optionally only its first `count` members and those with n <= nmax
        for m in I.mixed_batch(count or 4096, 32, 320, (2, 3), srw.check_sync):
            if nmax is None or m["n"] <= nmax:
                out.append((m["n"], m["k"], m["delta"], f"mix{m['n']}k{m['k']}"))
        return out
    if name in ("n256k2x10+cerny16-32", "n256k2x10"):
        for i in range(10):
            d, _ = I.first_synchronizing(256, 2, I.member_seed(I.BASE_SEED, i), srw.check_sync)
            out.append((256, 2, d, f"rand256#{i}"))
        if name == "n256k2x10+cerny16-32":
            for n in range(16, 33):
                out.append((n, 2, I.cerny(n), f"cerny{n}"))
    elif name == "n64k2x100":
        for i in range(100):
            d, _ = I.first_synchronizing(64, 2, I.member_seed(I.BASE_SEED, i), srw.check_sync)
            out.append((64, 2, d, f"rand64#{i}"))
    elif name == "sink26-k25":
        # the member of Rystsov's sink series with 26 states and 25 letters
        # (r = 325), the hard instance the paper times
        out.append((26, 25, I.sink_series(26), "sink26"))
    elif name == "n450k2":
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


def oracle_steps(path, max_steps):
    """Child process: the oracle's search of one automaton, stopped after
    1, 2, 3, ... expansion steps (each run from the start); one JSON line per
    run.  With max_steps > 0 only that many steps, once."""
    from oracle import oracle as O
    z = np.load(path)
    n, k, d = int(z["n"]), int(z["k"]), z["d"]
    for st in ([max_steps] if max_steps > 0 else range(1, 1 << 20)):
        t = time.perf_counter()
        done, info = O.bidir_steps(n, k, d, st)
        print(json.dumps({"steps": info["steps"], "candidates": info["candidates"], "done": done,
                          "s": time.perf_counter() - t}), flush=True)
        if done:
            break


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return model, cores


def cpu_baseline_steps(prob, budget_s, max_procs=16):
    """The oracle (single-threaded C, Alg. 2 meet) on one automaton too large
    for it to finish: its search stopped after S expansion steps, S the
    largest step count whose run fits the budget (the runs for 1, 2, ...
    steps go one after another in a child process, each from the start).
    Then the same S-step run in as many processes at once as the host has
    cores (at most max_procs), for the all-cores rate.  Runs before the GPU
    is touched."""
    import subprocess
    import tempfile
    n, k, d, label = prob
    model, ncpu = host_cpu()
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "m.npz")
        np.savez(path, n=n, k=k, d=d)
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-steps", path]
        proc = subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True)
        last, t0 = None, time.perf_counter()
        # each run takes about 1.5-2x the one before: stop starting runs
        # once the next one would likely overrun the budget
        for line in proc.stdout:
            rec = json.loads(line)
            last = rec
            if rec["done"] or time.perf_counter() - t0 + 2.5 * rec["s"] > budget_s:
                break
        proc.kill()
        proc.wait()
        if last is None:
            return None
        procs = max(1, min(max_procs, ncpu or 1))
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-steps", path,
               "--oracle-max-steps", str(last["steps"])]
        t1 = time.perf_counter()
        outs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True) for _ in range(procs)]
        cand = 0
        for p_ in outs:
            out, _ = p_.communicate()
            cand += json.loads(out.strip().splitlines()[-1])["candidates"]
        wall = time.perf_counter() - t1
    return {"value": last["candidates"] / last["s"], "unit": "subsets expanded/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{label}: the oracle's search stopped after its first {last['steps']} "
                      f"expansion steps ({last['candidates']} subsets expanded in {last['s']:.1f} s, "
                      f"one thread); the whole search does not finish within minutes on a CPU",
            "cpu_model": model, "host_cores": ncpu,
            "all_cores": {"value": cand / wall, "unit": "subsets expanded/s", "cores": procs,
                          "sample": f"the same {last['steps']}-step run in {procs} processes at once, "
                                    f"{wall:.1f} s wall"}}


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
            "automata_per_s": len(solved) / busy if busy else None,
            "cpu_model": host_cpu()[0], "host_cores": host_cpu()[1]}


def kernel_short_name(name):
    """'void srw::k_meet<4>(srw::StepDesc const*, ...)' -> 'k_meet<4>'."""
    name = name.split("(")[0].strip()
    if name.startswith("void "):
        name = name[5:]
    return name.replace("srw::", "")


KERNEL_SRC = os.path.join(ROOT, "paper_2207_05495_amd", "csrc", "srw_kernels.hip")


def source_sha1(path=KERNEL_SRC):
    """SHA-1 of the kernel source without its comments and blank lines: the
    code the counters describe (an edit of comments alone leaves it)."""
    import hashlib
    import re
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = [ln.rstrip() for ln in text.splitlines() if ln.strip()]
    return hashlib.sha1("\n".join(lines).encode()).hexdigest()


def pmc_summary(fetch_csv, write_csv, workload, out_path, src=KERNEL_SRC):
    """HBM bytes per launch of every kernel from two rocprofv3 --pmc runs of
    the same command (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch).  The
    command first runs three device copies of 256 MiB (--calib-copy-mb 256);
    each counter is scaled by the bytes one copy moves over what the counter
    read for it.  The kernel source the counters were taken with is recorded
    by its SHA-1, so that a later change to it voids the figures."""
    import csv
    import collections

    def load(path):
        d = collections.defaultdict(list)
        with open(path) as f:
            for row in csv.DictReader(f):
                d[kernel_short_name(row["Kernel_Name"])].append(float(row["Counter_Value"]))
        return d
    fe, wr = load(fetch_csv), load(write_csv)
    copy = "__amd_rocclr_copyBuffer"
    moved = 256.0 * 1024                          # KiB read (and written) by one copy
    f_fac = moved / (sum(fe[copy][:3]) / 3)
    w_fac = moved / (sum(wr[copy][:3]) / 3)
    per = {}
    print(f"calibration: 256 MiB copy -> FETCH_SIZE {fe[copy][0]:.0f} KiB, WRITE_SIZE "
          f"{wr[copy][0]:.0f} KiB; factors fetch {f_fac:.3f}, write {w_fac:.3f}")
    print("| kernel | dispatches | fetch MiB | write MiB | MiB per dispatch |")
    print("|---|---|---|---|---|")
    for k in sorted(fe, key=lambda k: -sum(fe[k])):
        if k == copy:
            continue
        n = len(fe[k])
        F = sum(fe[k]) * f_fac / 1024
        Wm = sum(wr.get(k, [0.0])) * w_fac / 1024
        per[k] = (F + Wm) * 2 ** 20 / n
        print(f"| `{k}` | {n} | {F:.1f} | {Wm:.1f} | {(F + Wm) / n:.2f} |")
    if out_path:
        with open(out_path, "w") as f:
            json.dump({workload: per, "_factors": {"fetch": f_fac, "write": w_fac},
                       "_kernel_source_sha1": source_sha1(src)}, f, indent=1)


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload`, from the rocprofv3
    FETCH_SIZE / WRITE_SIZE passes recorded in profiles/hbm_traffic.json
    (None when no counters were taken for this kernel and workload, or when
    the kernel source changed since)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("_kernel_source_sha1") != source_sha1():
        return None
    return rec.get(workload, {}).get(kernel)


def roofline(stats, cls_stats, workload):
    """Roofline of the kernel class with the most time (per-class times of
    `cls_stats`, a pass with every class timed); for the meet, its per-width
    launch times and operation counts come from `stats`, the timed region."""
    ms = cls_stats["ms"]
    launches = cls_stats["launches"]
    dom = max(CLASSES[:6], key=lambda c: ms[c])
    t = ms[dom] / max(1, launches[dom]) / 1e3     # seconds per launch
    nl = max(1, launches[dom])
    if dom == "meet" and stats["meet_w"]:
        # the meet launches one kernel per set width: take the one with the
        # most time.  Unit: the set operations of the chunked meet as the
        # counting build of the kernel counts them in the extra pass (32-bit
        # lane-ops: 2 per 64-bit column AND, 4 per word of a row subset
        # test), over the launch time of the timed region's kernel, against
        # the chip's 32-bit VALU rate.  The brute-force pair-word count
        # |L_f| * |L_b| * W is reported beside it: its ratio to the ops
        # performed is what the chunking prunes.
        W, m = max(stats["meet_w"].items(), key=lambda kv: kv[1]["ms"])
        mc = cls_stats.get("meet_w", {}).get(W, m)
        # the meet against inverse levels in buckets is its own kernel, with
        # its own events and counters; it is the one when it has most of the
        # width's time
        if m.get("b_launches", 0) and m["b_ms"] * 2 > m["ms"]:
            name, nl, t_ms = f"k_meet_b<{W}, false>", m["b_launches"], m["b_ms"]
            ops = mc.get("b_ops", 0) / max(1, mc.get("b_launches", 0))
        else:
            name, nl, t_ms = f"k_meet<{W}, false, false>", m["launches"], m["ms"]
            ops = (mc["ops"] - mc.get("b_ops", 0)) / max(1, mc["launches"] - mc.get("b_launches", 0))
            t_ms -= m.get("b_ms", 0.0)
            nl -= m.get("b_launches", 0)
        t = t_ms / max(1, nl) / 1e3
        ach = ops / t / 1e12
        return {"kernel": name, "bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS,
                "unit": "TOP/s", "frac": ach / VALU_PEAK_TOPS,
                "traffic": measured_traffic(workload, name),
                "ops_per_launch": ops,
                "brute_force_lane_ops_per_launch": 2.0 * m["pair_words"] / m["launches"],
                "per_launch_ms": t * 1e3, "launches": nl}
    byts = {"expand": cls_stats["bytes_expand"], "insert": cls_stats["bytes_insert"],
            "compact": cls_stats["bytes_compact"]}.get(dom)
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
    # candidates over the time of the kernels that expand, insert (hash
    # probes: at least one per candidate) and compact them; one-block steps
    # are timed with the expansion class
    t_exp = sum(stats["ms"][c] for c in ("expand", "insert", "compact"))
    if t_exp > 0:
        out["expansion_candidates_per_s"] = stats["candidates"] / (t_exp / 1e3)
    # hash inserts: one probe sequence and one compare-and-swap or atomicMin
    # per candidate, over the insertion class alone
    if "insert" in out and stats["ms"]["insert"] > 0:
        out["insert"]["hash_inserts_per_s"] = stats["candidates"] / (stats["ms"]["insert"] / 1e3)
    if "meet" in out and stats["ms"]["meet"] > 0:
        out["meet"]["pairs_per_s"] = stats["pairs"] / (stats["ms"]["meet"] / 1e3)
    return out


def serve_requests(count, nmax, kmax, srw):
    """Request mix of the serving workload (inputs.serve_mix): 90% random
    automata (n uniform in [64, nmax], k uniform in 2..kmax), 10% Černý C_n
    with n uniform in [8, 40]."""
    return [(m["n"], m["k"], m["delta"], m["label"])
            for m in I.serve_mix(count, nmax, kmax, srw.check_sync)]


def serve_bench(args, srw):
    """Poisson arrivals into one srw_server (continuous batching): latency
    percentiles and completed solves per second."""
    reqs = serve_requests(args.requests, args.serve_nmax, args.serve_kmax, srw)
    rng = np.random.default_rng(7)
    last = [time.perf_counter()]

    def progress(msg):
        if time.perf_counter() - last[0] > 10:
            last[0] = time.perf_counter()
            print(msg, file=sys.stderr, flush=True)

    rate = args.rate
    if rate <= 0:
        # capacity: a closed-loop pass of the first 64 requests
        m = min(64, len(reqs))
        with srw.Server(deadline_ms=args.deadline_ms) as s:
            t = time.perf_counter()
            for i, (n, k, d, _) in enumerate(reqs[:m]):
                s.submit(n, k, d, i)
            got = 0
            while got < m and time.perf_counter() - t < args.serve_seconds:
                got += len(s.poll(100000))
                progress(f"capacity pass: {got}/{m} done")
            cap = got / (time.perf_counter() - t)
        # the closed server's memory goes back to PyTorch's cache; hand it to
        # the driver so that the next server's budget (a share of the free
        # device memory) is not cut by it
        import torch
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        rate = 0.7 * cap
        print(f"capacity ~{cap:.2f}/s; arrival rate {rate:.2f}/s", file=sys.stderr, flush=True)
    gaps = rng.exponential(1.0 / rate, size=len(reqs))
    done = {}
    with srw.Server(deadline_ms=args.deadline_ms) as s:
        t0 = time.perf_counter()
        nxt = t0
        for i, (n, k, d, _) in enumerate(reqs):
            nxt += gaps[i]
            while True:
                for x in s.poll(0):
                    done[x["tag"]] = x
                progress(f"submitted {i}/{len(reqs)}, completed {len(done)}")
                if time.perf_counter() >= nxt:
                    break
                time.sleep(min(0.002, max(0.0, nxt - time.perf_counter())))
            s.submit(n, k, d, i)
        t_sub = time.perf_counter()
        while len(done) < len(reqs) and time.perf_counter() - t_sub < args.serve_seconds:
            for x in s.poll(100000):
                done[x["tag"]] = x
            progress(f"all submitted, completed {len(done)}/{len(reqs)}")
        elapsed = time.perf_counter() - t0
        pending = s.pending()
        print(f"closing the server with {pending} requests pending (each lane ends its running step)",
              file=sys.stderr, flush=True)
    ok = [x for x in done.values() if x["status"] == srw.OK]
    lat = np.array([x["latency_ms"] for x in ok]) if ok else np.zeros(1)
    per = {}
    for cls in sorted({r[3] for r in reqs}):
        idx = [i for i, r in enumerate(reqs) if r[3] == cls]
        fin = [done[i] for i in idx if i in done]
        ls = [x["latency_ms"] for x in fin if x["status"] == srw.OK]
        ent = {"requests": len(idx), "unfinished": len(idx) - len(fin),
               "status_counts": {srw.STATUS_NAMES.get(st, st): sum(1 for x in fin if x["status"] == st)
                                 for st in sorted({x["status"] for x in fin})}}
        if ls:
            ent.update({"p50_ms": float(np.percentile(ls, 50)), "p99_ms": float(np.percentile(ls, 99))})
        # the admission estimate against the device memory the solve held
        ratio = [x["dev_bytes"] / x["est_bytes"] for x in fin
                 if x["status"] == srw.OK and x["est_bytes"] > 0 and x["dev_bytes"] > 0]
        if ratio:
            ent["dev_over_estimate"] = {"p50": float(np.percentile(ratio, 50)),
                                        "min": float(min(ratio)), "max": float(max(ratio))}
        per[cls] = ent
    return {
        "metric": "subsets expanded/s + automata solved/s (batched vs plain, 1 GPU), p99 latency",
        "value": len(ok) / elapsed, "unit": "automata solved/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": elapsed * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "serve-mix", "requests": len(reqs), "rate_per_s": rate,
                   "mix": f"90% random n~U[64,{args.serve_nmax}] k~U{{2..{args.serve_kmax}}}, "
                          "10% Cerny n~U[8,40]", "path": "srw_server (continuous batching)"},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "completed": len(ok), "failed": len(done) - len(ok), "unfinished": int(pending),
        "status_counts": {srw.STATUS_NAMES.get(st, st): sum(1 for x in done.values() if x["status"] == st)
                          for st in sorted({x["status"] for x in done.values()})},
        "deadline_ms": args.deadline_ms,
        "per_class": per,
    }


def beam_bench(args, srw):
    """Beam-search upper bounds (srw_beam_batch) of 64 seeded random n = 450,
    k = 2 automata (the first is the default workload's), width ceil(n ln n)
    as in the paper's large-n runs (Section 3); beside it the oracle's beam
    search of the first automata, single-threaded."""
    import math
    import torch
    from oracle import oracle as O
    n, k, count = 450, 2, 64
    width = int(math.ceil(n * math.log(n)))
    probs = []
    for i in range(count):
        d, _ = I.first_synchronizing(n, k, I.member_seed(I.BASE_SEED, i), srw.check_sync)
        probs.append((n, k, d, width))
    # the oracle's beam, on as many automata as fit the CPU budget
    cpu, t_cpu, same = 0, 0.0, 0
    want = []
    while cpu < count and t_cpu < args.cpu_budget / 4:
        t = time.perf_counter()
        R, w, _ = O.beam(n, k, probs[cpu][2], width)
        t_cpu += time.perf_counter() - t
        want.append((R, w))
        cpu += 1
    res = srw.beam_batch(probs)                   # warmup
    for _ in range(args.warmup):
        res = srw.beam_batch(probs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = srw.beam_batch(probs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    for (R, w), (st, Rg, wg) in zip(want, res):
        exp = (srw.OK, R, list(w)) if R is not None else (srw.ENOBOUND, -1, None)
        if (st, Rg, wg) != exp:
            raise SystemExit(f"beam result {(st, Rg)} differs from the oracle's R={R}")
        same += 1
    Rs = [R for st, R, _ in res if st == srw.OK]
    stored = stored_oracle_values()
    r0 = stored.get(np.asarray(probs[0][2], dtype=np.int32).tobytes())
    return {
        "metric": "beam-search upper bounds/s (1 GPU)", "value": count / dt, "unit": "automata/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "beam-n450k2x64", "automata": count, "width": width,
                   "sizes": f"{count} x random n={n} k={k} (uniform delta, seeded SplitMix64, first "
                            "synchronizing draw)", "path": "srw_beam_batch"},
        "R_min": min(Rs) if Rs else None, "R_max": max(Rs) if Rs else None,
        "R_first": res[0][1], "r_first_exact": r0[0] if r0 else None,
        "oracle_checked": f"{same} of {count} (R and word) equal the oracle's beam search",
        "cpu_baseline": {"value": cpu / t_cpu if t_cpu else None, "unit": "automata/s", "cores": 1,
                         "kind": "oracle", "sample": f"the first {cpu} automata, orc_beam, one core",
                         "cpu": host_cpu()},
    }


def eppstein_bench(args, srw):
    """Eppstein upper bounds (srw_eppstein_batch) of 1,024 seeded random
    n = 450, k = 2 automata (the first 64 are those of the beam workload);
    beside it the oracle's Eppstein heuristic on the first automata,
    single-threaded, and a check of every word against it."""
    import torch
    from oracle import oracle as O
    n, k, count = 450, 2, 1024
    probs = []
    for i in range(count):
        d, _ = I.first_synchronizing(n, k, I.member_seed(I.BASE_SEED, i), srw.check_sync)
        probs.append((n, k, d))
    cpu, t_cpu = 0, 0.0
    want = []
    while cpu < count and t_cpu < args.cpu_budget:
        t = time.perf_counter()
        want.append(O.eppstein(n, k, probs[cpu][2])[0])
        t_cpu += time.perf_counter() - t
        cpu += 1
    res = srw.eppstein_batch(probs, word_cap=4096)        # warmup
    for _ in range(args.warmup):
        res = srw.eppstein_batch(probs, word_cap=4096)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = srw.eppstein_batch(probs, word_cap=4096)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    for i, (w, (st, ln, wg)) in enumerate(zip(want, res)):
        if (st, ln, wg) != (srw.OK, len(w), w):
            raise SystemExit(f"Eppstein result {i} ({st}, {ln}) differs from the oracle's ({len(w)})")
    lens = [ln for _, ln, _ in res]
    stored = stored_oracle_values()
    r0 = stored.get(np.asarray(probs[0][2], dtype=np.int32).tobytes())
    return {
        "metric": "Eppstein upper bounds/s (1 GPU)", "value": count / dt, "unit": "automata/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "eppstein-n450k2x1024", "automata": count,
                   "sizes": f"{count} x random n={n} k={k} (uniform delta, seeded SplitMix64, first "
                            "synchronizing draw)", "path": "srw_eppstein_batch"},
        "len_min": min(lens), "len_max": max(lens), "len_mean": float(np.mean(lens)),
        "len_first": lens[0], "r_first_exact": r0[0] if r0 else None,
        "oracle_checked": f"{cpu} of {count} words equal the oracle's",
        "cpu_baseline": {"value": cpu / t_cpu if t_cpu else None, "unit": "automata/s", "cores": 1,
                         "kind": "oracle", "sample": f"the first {cpu} automata, orc_eppstein, one core",
                         "cpu": host_cpu()},
    }


def bound_bench(args, srw):
    """The upper bound of Section 2.1.3 (srw_bound_batch: Eppstein, the beam
    of width n, the beam of the adaptive width) of 64 seeded random n = 450,
    k = 2 automata (those of the beam workload); beside it the oracle's
    composition of the same three on the first automata, single-threaded."""
    import torch
    from oracle import bounds as Bd
    n, k, count = 450, 2, 64
    probs = []
    for i in range(count):
        d, _ = I.first_synchronizing(n, k, I.member_seed(I.BASE_SEED, i), srw.check_sync)
        probs.append((n, k, d))
    cpu, t_cpu = 0, 0.0
    want = []
    while cpu < count and t_cpu < args.cpu_budget / 2:
        t = time.perf_counter()
        want.append(Bd.upper_bound(n, k, probs[cpu][2]))
        t_cpu += time.perf_counter() - t
        cpu += 1
    res = srw.bound_batch(probs)                   # warmup
    for _ in range(args.warmup):
        res = srw.bound_batch(probs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = srw.bound_batch(probs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    for i, ((R, w, w1, _), (st, Rg, wg, word)) in enumerate(zip(want, res)):
        if (st, Rg, wg, word) != (srw.OK, R, w1, w):
            raise SystemExit(f"bound {i}: ({st}, {Rg}, {wg}) differs from the oracle's ({R}, {w1})")
    Rs = [R for st, R, _, _ in res if st == srw.OK]
    widths = [wd for st, _, wd, _ in res if st == srw.OK]
    stored = stored_oracle_values()
    r0 = stored.get(np.asarray(probs[0][2], dtype=np.int32).tobytes())
    return {
        "metric": "upper bounds (Eppstein + adaptive beam)/s (1 GPU)", "value": count / dt,
        "unit": "automata/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "bound-n450k2x64", "automata": count,
                   "sizes": f"{count} x random n={n} k={k} (uniform delta, seeded SplitMix64, first "
                            "synchronizing draw)", "path": "srw_bound_batch"},
        "R_min": min(Rs), "R_max": max(Rs), "R_mean": float(np.mean(Rs)),
        "width_min": min(widths), "width_max": max(widths),
        "R_first": res[0][1], "r_first_exact": r0[0] if r0 else None,
        "oracle_checked": f"{cpu} of {count} (R, width and word) equal the oracle's",
        "cpu_baseline": {"value": cpu / t_cpu if t_cpu else None, "unit": "automata/s", "cores": 1,
                         "kind": "oracle", "sample": f"the first {cpu} automata, oracle/bounds.py "
                                                     "(orc_eppstein, orc_beam_sizes), one core",
                         "cpu": host_cpu()},
    }


def stored_oracle_values():
    """(r, word) the oracle stored under tests/golden for seeded random
    automata, keyed by the bytes of the transition table (rebuilt from each
    entry's seed and attempt)."""
    import glob
    out = {}
    for path in glob.glob(os.path.join(ROOT, "tests", "golden", "*.json")):
        with open(path) as f:
            rec = json.load(f)
        for c in rec.get("cases", []):
            if "r" not in c or "seed" not in c or "attempt" not in c:
                continue
            d = I.random_automaton(c["n"], c["k"], c["seed"], c["attempt"])
            w = c["word"]
            w = [int(x) for x in w] if isinstance(w, str) else list(w)
            out[d.tobytes()] = (c["r"], w)
    return out


def check_against_oracle(probs, res, stored, words=True):
    """Every result with a stored oracle value must equal it (r and word;
    r alone with words=False, for the list reductions, which keep r but may
    return another shortest word); returns how many were checked."""
    checked = 0
    for (n, k, d, label), (st, r, w) in zip(probs, res):
        want = stored.get(np.asarray(d, dtype=np.int32).tobytes())
        if want is None:
            continue
        if st != 0 or r != want[0] or (words and w != want[1]):
            raise SystemExit(f"{label}: GPU result {(st, r)} differs from the stored oracle value r={want[0]}")
        checked += 1
    return checked


def batched_vs_plain(args, srw, stored):
    """Automata solved per second by one srw_solve_batch call over a seeded
    batch against srw_solve one automaton at a time, with the latency of the
    single solves."""
    import torch
    probs = workload(args.batch_workload, srw, None, args.batch_nmax)
    batch = [(n, k, d) for n, k, d, _ in probs]
    res = srw.solve_batch(batch)                  # warmup
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = srw.solve_batch(batch)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    assert all(st == 0 for st, _, _ in res)
    checked = check_against_oracle(probs, res, stored)
    print(f"batched pass over {len(batch)} automata: {tb * 1e3:.0f} ms", file=sys.stderr, flush=True)
    lat = []
    t = time.perf_counter()
    for n, k, d in batch:
        a = time.perf_counter()
        srw.solve(n, k, d)
        lat.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    sizes = sorted({n for n, _, _, _ in probs})
    return {"workload": args.batch_workload, "automata": len(batch),
            "members": f"the members with n <= {args.batch_nmax} of the seeded 4096-member batch "
                       f"(n~U[32,320], k~U{{2,3}}; here n in [{sizes[0]}, {sizes[-1]}])"
                       if args.batch_nmax else "all members",
            "batched_automata_per_s": len(batch) / tb, "batched_ms": tb * 1e3,
            "plain_automata_per_s": len(batch) / tp, "plain_ms": tp * 1e3,
            "batched_over_plain": tp / tb,
            "plain_p50_ms": float(np.percentile(lat, 50)), "plain_p99_ms": float(np.percentile(lat, 99)),
            "oracle_checked": checked}


def tuning_note(tuned):
    """The autotuner's values in force ({W: {key: value}}), or None."""
    if not tuned:
        return None
    return {"table": "paper_2207_05495_amd/tuning.json",
            "per_width": {str(w): v for w, v in sorted(tuned.items())}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n450k2")
    ap.add_argument("--batch-workload", default="mix4096-n32-320-k2-3",
                    help="batched-vs-plain comparison: this workload ...")
    ap.add_argument("--batch-nmax", type=int, default=160,
                    help="... its members with n <= BATCH_NMAX (0: all)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--set", action="append", default=[], metavar="KEY=VALUE",
                    help="library option (srw_set_option) for the whole run; repeatable")
    ap.add_argument("--no-tuning", action="store_true",
                    help="leave out the autotuner's per-width table (paper_2207_05495_amd/tuning.json); "
                         "its values take precedence over --set values of the same keys")
    ap.add_argument("--cpu-budget", type=float, default=40.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--oracle-one", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--oracle-steps", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--oracle-max-steps", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="summarize rocprofv3 FETCH_SIZE / WRITE_SIZE counter files of a run "
                         "with --calib-copy-mb 256 and exit (no GPU)")
    ap.add_argument("--pmc-out", default=None, help="with --pmc-summary: write the JSON here")
    ap.add_argument("--pmc-src", default=KERNEL_SRC,
                    help="with --pmc-summary: the kernel source the counters were taken with")
    ap.add_argument("--count", type=int, default=None,
                    help="mix4096-n32-320-k2-3: first COUNT members of the seeded 4096-member batch")
    ap.add_argument("--nmax", type=int, default=None,
                    help="mix4096-n32-320-k2-3: keep only members with n <= NMAX")
    ap.add_argument("--requests", type=int, default=400, help="serve-mix: requests")
    ap.add_argument("--deadline-ms", type=int, default=20000,
                    help="serve-mix: per-request deadline on the device (0: none)")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serve-mix: Poisson arrivals per second (0: 0.7 x measured capacity)")
    ap.add_argument("--serve-nmax", type=int, default=400, help="serve-mix: largest random n")
    ap.add_argument("--serve-kmax", type=int, default=4, help="serve-mix: largest alphabet")
    ap.add_argument("--serve-seconds", type=float, default=90.0,
                    help="serve-mix: stop waiting for completions after this long")
    args = ap.parse_args()
    if args.oracle_one:
        oracle_one(args.oracle_one)
        return
    if args.oracle_steps:
        oracle_steps(args.oracle_steps, args.oracle_max_steps)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.workload, args.pmc_out,
                    args.pmc_src)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the search of one automaton is not sharded "
              "across GPUs in this library; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2207_05495_amd import srw
    if args.workload == "beam-n450k2x64":
        import torch
        torch.cuda.set_device(0)
        srw.use_torch(0)
        print(json.dumps(beam_bench(args, srw)))
        return
    if args.workload == "bound-n450k2x64":
        import torch
        torch.cuda.set_device(0)
        srw.use_torch(0)
        print(json.dumps(bound_bench(args, srw)))
        return
    if args.workload == "eppstein-n450k2x1024":
        import torch
        torch.cuda.set_device(0)
        srw.use_torch(0)
        print(json.dumps(eppstein_bench(args, srw)))
        return
    if args.workload == "serve-mix":
        import torch
        torch.cuda.set_device(0)
        srw.use_torch(0)
        tuned = {} if args.no_tuning else srw.apply_tuning()
        out = serve_bench(args, srw)
        out["config"]["tuning"] = tuning_note(tuned)
        print(json.dumps(out))
        return
    probs = workload(args.workload, srw, args.count, args.nmax)   # host-only calls so far
    stored = stored_oracle_values()
    cpu = None
    if not args.no_cpu:
        cpu = (cpu_baseline_steps(probs[0], args.cpu_budget) if len(probs) == 1
               else cpu_baseline(probs, args.cpu_budget))

    import torch
    torch.cuda.set_device(0)
    srw.use_torch(0)
    tuned = {} if args.no_tuning else srw.apply_tuning()
    for kv in args.set:
        key, val = kv.split("=", 1)
        srw.set_option(key, int(val))
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
    words = all(kv.split("=", 1)[0] != "reduce" or kv.split("=", 1)[1] == "0" for kv in args.set)
    checked = check_against_oracle(probs, res, stored, words) if args.warmup else 0
    # timed region: only the meet launches carry HIP events (profile 2); the
    # per-class events of profile 1 serialize the queue between kernels
    srw.reset_stats()
    srw.set_option("profile", 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = []
    for s in range(args.steps):
        a = time.perf_counter()
        res = srw.solve_batch(batch)
        step_ms.append((time.perf_counter() - a) * 1e3)
        print(f"step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    srw.set_option("profile", 0)
    for st, r, w in res:
        assert st == 0
    stats = srw.get_stats()
    # one more pass, outside the timed region, with every kernel class timed
    srw.reset_stats()
    srw.set_option("profile", 1)
    srw.solve_batch(batch)
    torch.cuda.synchronize()
    srw.set_option("profile", 0)
    cls_stats = srw.get_stats()
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
                   "options": dict(kv.split("=", 1) for kv in args.set),
                   "automata": len(probs),
                   "sizes": {
                       "n64k2x100": "100 x random n=64 k=2",
                       "n256k2x10": "10 x random n=256 k=2",
                       "n256k2x10+cerny16-32": "10 x random n=256 k=2 + Cerny C_16..C_32",
                       "mix4096-n32-320-k2-3": f"first {len(probs)} of the 4096-member batch, "
                                  "n~U[32,320], k~U{2,3}",
                       "n450k2": "1 x random n=450 k=2",
                       "sink26-k25": "Rystsov's sink series, n=26 k=25 (r=325)"}[args.workload]
                   + ("" if args.workload.startswith("sink") else
                      " (uniform delta, seeded SplitMix64, first synchronizing draw)"),
                   "path": "srw_solve_batch",
                   "tuning": tuning_note(tuned)},
        "automata_per_s": len(probs) / per_step,
        "step_p50_ms": float(np.percentile(step_ms, 50)),
        "step_p99_ms": float(np.percentile(step_ms, 99)),
        "oracle_checked": f"{checked} of {len(probs)} results equal stored oracle values "
                          f"({'r and word' if words else 'r'})",
        "subsets_per_step": cand,
        "pairs_per_step": stats["pairs"] / args.steps,
        "kernels": class_table(cls_stats),
        "meet_work": cls_stats["meet_work"],
        "kernels_note": "per-class times of one extra pass with every class timed (and the "
                        "meet's counting build: meet_work)",
        "roofline": roofline(stats, cls_stats, args.workload),
    }
    if not args.no_plain and len(batch) > 1:
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
    if not args.no_batch:
        out["batched_vs_plain"] = batched_vs_plain(args, srw, stored)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
