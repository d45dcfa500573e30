"""Pins of the oracle's cost-model step choice (Section 2.1.2): ExpMark's
special cases and limits, the density of a list, and that the search it
steers finds the same r and word as any other schedule."""

import numpy as np
import pytest

from oracle import oracle as O
from oracle import schedule as S
from paper_2207_05495_amd import inputs as I


@pytest.mark.parametrize("b_s,a_d,b_d", [(1.0, 0.3, 0.4), (1e6, 0.05, 0.5), (77.0, 0.9, 0.1)])
def test_exp_mark_of_one_set(b_s, a_d, b_d):
    # A_s = 1: the power of A_s is 1 whatever the exponent
    want = b_s * ((1 + b_d) / b_d + 1 / (a_d * (1 - b_d)))
    assert S.exp_mark(1.0, b_s, a_d, b_d) == pytest.approx(want, rel=1e-12)


def test_exp_mark_is_linear_in_a_for_sparse_a():
    # A_d -> 0: w -> 1 + B_d, the exponent -> 1 (every A-set is tested)
    for b_d in (0.1, 0.4, 0.8):
        r = S.exp_mark(2e6, 1e4, 1e-12, b_d) / S.exp_mark(1e6, 1e4, 1e-12, b_d)
        assert r == pytest.approx(2.0, rel=1e-6)


def test_exp_mark_is_linear_in_a_for_dense_b():
    # B_d -> 1: w -> 2 = 1 + B_d whatever A_d, so the exponent -> 1
    for a_d in (0.05, 0.5, 0.95):
        r = S.exp_mark(2e6, 10.0, a_d, 1 - 1e-12) / S.exp_mark(1e6, 10.0, a_d, 1 - 1e-12)
        assert r == pytest.approx(2.0, rel=1e-6)


def test_exp_mark_grows_sublinearly_and_monotonically():
    for a_d in (0.02, 0.2, 0.6):
        for b_d in (0.05, 0.3, 0.7):
            base = S.exp_mark(1e5, 1e5, a_d, b_d)
            assert base > 0
            r = S.exp_mark(4e5, 1e5, a_d, b_d) / base
            assert 1.0 < r <= 4.0 + 1e-9          # below brute force's 4x
            assert S.exp_mark(1e5, 4e5, a_d, b_d) == pytest.approx(4 * base)   # linear in B_s
    assert S.exp_mark(0, 10, 0.2, 0.3) == 0.0 and S.exp_mark(10, 0, 0.2, 0.3) == 0.0


def test_density_of_a_list():
    # n = 70 (two words): sets of sizes 70, 1 and 3
    rows = np.zeros((3, 2), dtype=np.uint64)
    rows[0] = [np.uint64(2**64 - 1), np.uint64(2**6 - 1)]
    rows[1, 1] = np.uint64(1 << 5)
    rows[2, 0] = np.uint64(0b1011)
    assert S.density(rows, 70) == pytest.approx(74 / 210)
    assert S.density(rows[:0], 70) == 0.0


def cases():
    out = []
    for i, (n, k) in enumerate([(12, 2), (20, 2), (33, 3), (48, 2), (64, 2), (70, 4), (96, 2),
                                (100, 3), (120, 2), (128, 2)]):
        d, _ = I.first_synchronizing(n, k, I.member_seed(I.BASE_SEED ^ 7, i), O.is_synchronizing)
        out.append((n, k, d))
    return out


def test_cost_schedule_keeps_r_and_word_and_is_not_the_frontier_rule():
    """Any schedule finds the least (i, j) meeting pair at the first step
    where f + b = r, so the cost-steered search returns the plain search's r
    and word; on some of these automata it steps differently."""
    differs = 0
    for n, k, d in cases():
        sides = S.cost_sides(n, k, d)
        r, w, info = O.bidir(n, k, d)
        r2, w2, info2 = O.bidir(n, k, d, sched=sides)
        assert r2 == r and list(w2) == list(w), (n, k)
        assert info2["sides"] == sides
        differs += sides != info["sides"]
    assert differs >= 1


def test_first_step_of_the_cost_schedule_goes_forward():
    # |L_BFS| = 1 against n singletons: the forward step is the cheaper
    for n, k, d in cases()[:4]:
        _, levels = O.levels_after(n, k, d, [])
        bfs, ibfs = S.step_costs(n, k, levels)
        assert bfs < ibfs
