"""Autotuner of the batched solve, per set width W = ceil(n/64).

For each width class it draws a seeded sample of random automata of that
width (uniform delta, as everywhere else), times ``srw_solve_batch`` on the
sample under candidate values of the library's tuning options, and keeps,
one option at a time (coordinate descent, in the order of ``GRID``), the
value with the least time.  A value replaces the current one only when it is
faster by more than ``--margin`` (timing noise).  Every run of a class must
give the same r and word for every automaton: the options change how the
search runs, never what it finds, and a difference stops the tuner with an
error.  A value under which some automaton of the sample does not finish
(out of device memory, say) is left out.

What it tunes, per width:
  schedule     the direction schedule: 0 smaller frontier first, 3 the
               cost model of Section 2.1.2
  meet_groups  tile groups of 64 inverse sets per chunked-meet work item
  meet_rows    candidate rows above which a tile group ANDs columns staged in
               LDS instead of testing sets one by one
  bucket       inverse-level size from which levels are kept in buckets
  small_cand   candidates up to which a step runs in one block (and the
               first steps of an automaton in one launch)

The set width itself is not a choice: a wider bitset than ceil(n/64) words
only adds words to every operation.

The table it writes (``tuning.json`` beside this file by default) is applied
with ``srw.apply_tuning()``; each value becomes the library option
"<key>@<W>".

Usage (on the GPU, from the repository root):
    python -m paper_2207_05495_amd.autotune --widths 1,2,3,4,5,8
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

from paper_2207_05495_amd import inputs as I
from paper_2207_05495_amd import srw

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning.json")

# option -> candidate values, in the order they are tuned; the first value
# listed is not the start: every option starts at the library default
GRID = (
    ("schedule", (0, 3)),
    ("meet_groups", (8, 16, 32, 64)),
    ("meet_rows", (128, 256, 512)),
    ("bucket", (0, 4096, 16384, 65536)),
    ("small_cand", (512, 2048, 8192)),
)
DEFAULTS = {"schedule": 0, "meet_groups": 16, "meet_rows": 512, "bucket": 16384, "small_cand": 2048}

# per width: (automata in the sample, n range, letter counts); sized so that
# one batched run of a class takes a fraction of a second to a few seconds
SAMPLES = {
    1: (256, (32, 64), (2, 3)),
    2: (128, (65, 128), (2, 3)),
    3: (48, (129, 192), (2, 3)),
    4: (16, (193, 256), (2,)),
    5: (8, (257, 320), (2,)),
    6: (4, (321, 384), (2,)),
    7: (1, (385, 448), (2,)),
    8: (1, (449, 452), (2,)),
}
SAMPLE_BASE = I.BASE_SEED ^ 0xA770


def sample(W, count=None):
    """The seeded sample of width class W: list of (n, k, delta)."""
    cnt, (lo, hi), ks = SAMPLES[W]
    members = I.mixed_batch(count or cnt, lo, hi, ks, srw.check_sync, base=SAMPLE_BASE + W)
    return [(m["n"], m["k"], m["delta"]) for m in members]


def _set(W, values):
    for key, v in values.items():
        srw.set_option(f"{key}@{W}", v)


def _clear(W):
    for key, _ in GRID:
        srw.set_option(f"{key}@{W}", -1)


def time_class(W, probs, values, repeat):
    """Least wall time of `repeat` batched runs of the sample, and their
    results (status, r, word per automaton)."""
    _set(W, values)
    best, res = None, None
    for _ in range(repeat):
        t0 = time.perf_counter()
        out = srw.solve_batch(probs)
        dt = time.perf_counter() - t0
        if res is not None and out != res:
            raise RuntimeError(f"width {W}: two runs under {values} gave different results")
        res = out
        best = dt if best is None else min(best, dt)
    return best, res


def tune_class(W, probs, repeat=2, margin=0.02, log=print):
    cur = dict(DEFAULTS)
    t_cur, want = time_class(W, probs, cur, repeat)
    if any(st != srw.OK for st, _, _ in want):
        raise RuntimeError(f"width {W}: a sample member did not solve ({[st for st, _, _ in want]})")
    t_default = t_cur
    trials = [{"values": dict(cur), "s": round(t_cur, 5)}]
    log(f"W={W}: {len(probs)} automata (n {sorted(n for n, _, _ in probs)[:8]}...), "
        f"r {[r for _, r, _ in want][:8]}..., defaults {t_cur * 1e3:.1f} ms")
    for key, cands in GRID:
        for v in cands:
            if v == cur[key]:
                continue
            trial = dict(cur, **{key: v})
            t, res = time_class(W, probs, trial, repeat)
            failed = [(i, st) for i, (st, _, _) in enumerate(res) if st != srw.OK]
            wrong = [(i, want[i][1], res[i][1]) for i in range(len(res))
                     if res[i][0] == srw.OK and res[i][1:] != want[i][1:]]
            if wrong:
                raise RuntimeError(f"width {W}: {trial} changed r or word of members {wrong[:4]}")
            if failed:
                trials.append({"values": trial, "s": None,
                               "failed": [[i, srw.STATUS_NAMES.get(st, st)] for i, st in failed]})
                log(f"  {key}={v}: {len(failed)} member(s) did not finish "
                    f"({srw.STATUS_NAMES.get(failed[0][1], failed[0][1])}); left out")
                continue
            trials.append({"values": trial, "s": round(t, 5)})
            log(f"  {key}={v}: {t * 1e3:.1f} ms")
            if t < t_cur * (1 - margin):
                cur, t_cur = trial, t
    _clear(W)
    return {"values": cur, "s": round(t_cur, 5), "default_s": round(t_default, 5),
            "automata": len(probs), "trials": trials}


def tune(widths, repeat=2, margin=0.02, log=print):
    srw.use_torch(0)
    table = {}
    for W in widths:
        probs = sample(W)
        # one run of a class of the widest sets takes about a second or more
        table[str(W)] = tune_class(W, probs, repeat if W <= 5 else 1, margin, log)
    return table


def write_table(table, path, argv):
    import torch
    rec = {"device": torch.cuda.get_device_name(0),
           "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", ""),
           "host": platform.node(),
           "made_by": "python -m paper_2207_05495_amd.autotune " + " ".join(argv),
           "made_at": time.strftime("%Y-%m-%d %H:%M:%S"),
           "defaults": DEFAULTS,
           "widths": table}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    os.replace(tmp, path)


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--widths", default="1,2,3,4,5,8")
    ap.add_argument("--repeat", type=int, default=2)
    ap.add_argument("--margin", type=float, default=0.02)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    a = ap.parse_args(argv)
    widths = [int(x) for x in a.widths.split(",") if x]
    if any(w not in SAMPLES for w in widths):
        ap.error("widths are 1..8")

    def log(*x):
        print(*x, flush=True)

    table = tune(widths, a.repeat, a.margin, log)
    write_table(table, a.out, argv)
    log("wrote", a.out)


if __name__ == "__main__":
    main()
