"""Writes expected (r, word) of full-size workloads with the CPU oracle.

Calls only oracle/ and the shared input generator: the stored values never
come from the GPU path.  Each entry records the generator seed and attempt,
so a test can rebuild the exact automaton.

    python tests/golden/make_golden.py rand256     # n=256, k=2, 10 seeds
    python tests/golden/make_golden.py mixed       # smaller mixed sizes
    python tests/golden/make_golden.py mix4096     # members with n <= 160 among the
                                                   # first 300 of the 4096-member batch
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
    raise SystemExit(f"unknown set {which}")


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "rand256"
    procs = int(sys.argv[2]) if len(sys.argv) > 2 else 6
    js = jobs(which)
    with Pool(procs) as p:
        res = p.map(solve_one, js, chunksize=1)
    path = os.path.join(HERE, f"{which}.json")
    with open(path, "w") as f:
        json.dump({"generator": "paper_2207_05495_amd.inputs (SplitMix64, first synchronizing attempt)",
                   "oracle": "oracle/srw_oracle.c orc_bidir, Alg. 2 meet",
                   "cases": res}, f, indent=1)
    print(path, [(c["n"], c["k"], c["r"], c["oracle_s"]) for c in res])


if __name__ == "__main__":
    main()
