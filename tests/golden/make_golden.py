"""Writes expected (r, word) of full-size workloads with the CPU oracle.

Calls only oracle/ and the shared input generator: the stored values never
come from the GPU path.  Each entry records the generator seed and attempt,
so a test can rebuild the exact automaton.

    python tests/golden/make_golden.py rand256     # n=256, k=2, 10 seeds
    python tests/golden/make_golden.py mixed       # smaller mixed sizes
    python tests/golden/make_golden.py mix4096     # members with n <= 160 among the
                                                   # first 300 of the 4096-member batch
    python tests/golden/make_golden.py n450        # the n=450, k=2 automaton (hours of CPU)
    python tests/golden/make_golden.py gpucases 1   # larger cases of the GPU parity tests
    python tests/golden/make_golden.py serve5 2 120
                                                   # random requests among the first 120
                                                   # of the serving mix, 120 s each at most
    python tests/golden/make_golden.py mix4096big 4 900
                                                   # members with n > 160 among the first
                                                   # 300 of the batch, at most 900 s of
                                                   # oracle time each (the rest recorded
                                                   # as unpinned)
    python tests/golden/make_golden.py serve5 5 900 --resume
                                                   # only the entries of the stored set
                                                   # recorded as unpinned, with the new
                                                   # budget; the others are kept
"""

import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2207_05495_amd import inputs as I  # noqa: E402


def solve_one(args):
    n, k, seed = args
    d, attempt = I.first_synchronizing(n, k, seed, O.is_synchronizing)
    t = time.time()
    r, w, info = O.bidir(n, k, d, meet=O.MEET_MARK)
    return {"n": n, "k": k, "seed": seed, "attempt": attempt, "r": r,
            "word": "".join(str(x) for x in w) if k <= 10 else w,
            "visited_f": info["visited_f"], "visited_b": info["visited_b"],
            "pairs": info["pairs"], "oracle_s": round(time.time() - t, 2)}


def solve_bounded(args):
    """solve_one in a child process, stopped after `budget` seconds."""
    n, k, seed, budget = args
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--one", str(n), str(k), str(seed)]
    try:
        res = subprocess.run(cmd, capture_output=True, text=True, timeout=budget, check=True)
    except subprocess.TimeoutExpired:
        return {"n": n, "k": k, "seed": seed, "unpinned": f"oracle over {budget} s"}
    except subprocess.CalledProcessError as e:
        return {"n": n, "k": k, "seed": seed, "unpinned": f"oracle failed: {e.stderr[-200:]}"}
    return json.loads(res.stdout.strip().splitlines()[-1])


def jobs(which):
    if which == "rand256":
        return [(256, 2, I.member_seed(I.BASE_SEED, i)) for i in range(10)]
    if which == "mixed":
        out = []
        for i, (n, k) in enumerate([(160, 2), (192, 2), (224, 2), (96, 3), (128, 3),
                                    (160, 3), (80, 4), (100, 4), (300, 2), (320, 2)]):
            out.append((n, k, I.member_seed(I.BASE_SEED ^ 0xABCDEF, i)))
        return out
    if which == "mix4096":
        # the seeded 4096-member batch (n uniform in [32, 320], k in {2, 3}):
        # its first 300 members, those with n <= 160
        return [(m["n"], m["k"], m["seed"])
                for m in I.mixed_batch(300, 32, 320, (2, 3), O.is_synchronizing) if m["n"] <= 160]
    if which == "mix4096big":
        # the same first 300 members, those with n > 160, cheapest first
        ms = [m for m in I.mixed_batch(300, 32, 320, (2, 3), O.is_synchronizing) if m["n"] > 160]
        ms.sort(key=lambda m: (m["k"], m["n"]))
        return [(m["n"], m["k"], m["seed"]) for m in ms]
    if which == "gpucases":
        # the larger random cases of the GPU parity tests (seed base, index)
        spec = [(200, 3, 5, 1)]
        spec += [(n, k, 61, j) for j, (n, k) in enumerate([(64, 2), (150, 2), (200, 3), (129, 2),
                                                            (40, 4), (255, 2), (90, 3)])]
        spec += [(n, k, 79, i) for i, (n, k) in enumerate([(40, 2), (64, 3), (100, 2), (150, 2),
                                                               (200, 3)])]
        spec += [(n, k, 97, i) for i, (n, k) in enumerate([(20, 2), (64, 2), (65, 3), (128, 2),
                                                               (190, 3), (257, 2)])]
        return [(n, k, I.member_seed(b, i)) for n, k, b, i in spec]
    if which == "serve5":
        # the random requests among the first 120 of the serving mix (n uniform
        # in [64, 400], k uniform in 2..4); its Černý requests are fixed by the
        # closed form instead
        return [(m["n"], m["k"], m["seed"]) for m in I.serve_mix(120, 400, 4, O.is_synchronizing)
                if "seed" in m]
    if which == "n450":
        # the single hard instance: n = 450, k = 2, seed of member 0
        return [(450, 2, I.member_seed(I.BASE_SEED, 0))]
    raise SystemExit(f"unknown set {which}")


def main():
    if sys.argv[1:2] == ["--one"]:
        print(json.dumps(solve_one(tuple(int(x) for x in sys.argv[2:5]))), flush=True)
        return
    resume = "--resume" in sys.argv
    args = [a for a in sys.argv[1:] if a != "--resume"]
    which = args[0] if args else "rand256"
    procs = int(args[1]) if len(args) > 1 else 6
    budget = float(args[2]) if len(args) > 2 else None
    path = os.path.join(HERE, f"{which}.json")
    js = jobs(which)
    old = {}
    if resume:
        with open(path) as f:
            old = {(c["n"], c["k"], c["seed"]): c for c in json.load(f)["cases"]}
        todo = [j for j in js if "unpinned" in old.get(j, {"unpinned": 1})]
    else:
        todo = js
    got = {}

    def write():
        res = [got[j] if j in got else old[j] for j in js if j in got or j in old]
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"generator": "paper_2207_05495_amd.inputs (SplitMix64, first synchronizing attempt)",
                       "oracle": "oracle/srw_oracle.c orc_bidir, Alg. 2 meet",
                       "cases": res}, f, indent=1)
        os.replace(tmp, path)
        return res

    # results are written as they come (a long run can be stopped and resumed)
    with Pool(procs) as p:
        if budget is None:
            it = p.imap_unordered(solve_one, todo, chunksize=1)
        else:
            it = p.imap_unordered(solve_bounded, [j + (budget,) for j in todo], chunksize=1)
        for c in it:
            got[(c["n"], c["k"], c["seed"])] = c
            if resume:
                write()
            print(c["n"], c["k"], c.get("r"), c.get("oracle_s", c.get("unpinned")), flush=True)
    res = write()
    print(path, [(c["n"], c["k"], c.get("r"), c.get("oracle_s")) for c in res])


if __name__ == "__main__":
    main()
