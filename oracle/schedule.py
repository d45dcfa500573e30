"""The paper's cost-model step choice, restricted to the plain search.

TEST INFRASTRUCTURE ONLY.  Only the test suite may import this module; the
library never does.

Section 2.1.2 prices each possible next step by the subset tests it is
expected to make, using ExpMark, an estimate of the tests of one
MarkSupersets call, and picks the cheapest.  The plain search has two of the
paper's five step types, BFS and IBFS, both with their history (an exact
visited set); it has no BFS^NH / IBFS^NH and no DFS phase.  Their costs are
taken as infinite, as the paper does for a step that cannot be made, and the
paper then compares the single-step costs of BFS and IBFS greedily.  Of the
four terms of Eq. 1-4 two price inclusion reductions (self-reduction, Eq. 2;
reduction by history, Eq. 3) that the plain search does not make, so they
are zero; what remains is the set cost (Eq. 1) and the meet test (Eq. 4).

Readings where the paper is silent:
  - the fraction r^dupl a side's duplicate removal takes away is that of its
    last step: 1 - |new level| / (k |previous level|); 0 before its first step;
  - densities are clamped to [1/(2n), 1 - 1/(2n)] (ExpMark divides by A_d,
    B_d and 1 - B_d);
  - ties go forward.

Parity unpinned beyond the checks of tests/test_schedule_oracle.py: the paper
gives no worked value of ExpMark or of a step choice.
"""

from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

SET_COST = 512.0          # the constant SetCost of Section 2.1.2


def exp_mark(a_s, b_s, a_d, b_d):
    """ExpMark(A_s, B_s, A_d, B_d) of Section 2.1.2: the estimated subset
    tests of marking the sets of a list B (B_s sets, density B_d) that are
    supersets of a set of a list A (A_s sets, density A_d)."""
    if a_s <= 0 or b_s <= 0:
        return 0.0
    w = (1.0 + b_d) / (1.0 + a_d * b_d - a_d)
    exponent = math.log(1.0 + b_d) / math.log(w)     # log base w of (1 + B_d)
    return b_s * ((1.0 + b_d) / b_d + 1.0 / (a_d - a_d * b_d)) * a_s ** exponent


def density(rows, n):
    """density(L) = sum of |S| over S in L, divided by n |L|."""
    if len(rows) == 0:
        return 0.0
    bits = np.unpackbits(np.ascontiguousarray(rows).view(np.uint8)).sum()
    return float(bits) / (n * len(rows))


def step_costs(n, k, levels):
    """(BFS cost, IBFS cost) of the next step, given the lists of both sides
    (levels[side] = [(rows, keys), ...], the current level last)."""
    lo, hi = 0.5 / n, 1.0 - 0.5 / n

    def clamp(x):
        return min(hi, max(lo, x))

    def side(s):
        cur = levels[s][-1][0]
        size = len(cur)
        if len(levels[s]) >= 2 and len(levels[s][-2][0]) > 0:
            r_dupl = 1.0 - size / (k * len(levels[s][-2][0]))
        else:
            r_dupl = 0.0
        return size, r_dupl, clamp(density(cur, n) if size else lo)

    lf, rf, df = side(0)
    lb, rb, db = side(1)
    bfs = SET_COST * k * lf + exp_mark(k * (1.0 - rf) * lf, lb, df, db)
    ibfs = SET_COST * k * lb + exp_mark(lf, k * (1.0 - rb) * lb, df, db)
    return bfs, ibfs


def cost_sides(n, k, delta, max_steps=10_000):
    """The sides the cost model picks, step by step, until the searches meet
    (the plain bidirectional search, run by the oracle after each choice)."""
    sched = []
    while True:
        met, levels = O.levels_after(n, k, delta, sched)
        if met:
            return sched
        if len(sched) >= max_steps:
            raise RuntimeError("step limit")
        bfs, ibfs = step_costs(n, k, levels)
        sched.append(1 if ibfs < bfs else 0)
