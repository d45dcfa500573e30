"""Invariants of the oracle's upper-bound policy (oracle/bounds.py, the
readings of Section 2.1.3 listed there): the bound is a reset word of
length R with r <= R <= Eppstein's length and R <= the first beam's R; the
beam size lies in [n, 2^20]; a first beam that cut no level was the exact
inverse search, so R = r and no second beam is run; the cost estimate on a
hand-worked example."""

import numpy as np

from oracle import bounds as Bd
from oracle import oracle as O
from paper_2207_05495_amd import inputs as I


def test_cost_estimate_hand_example():
    # levels 4, 3, 6 (first above w0 = 4 at depth 2, growth 6/3 = 2), B = 6:
    # h = 3, U = 4, 3, 6, 12 -> C = 2 * 25 = 50; width ceil(50 / 96) -> w0
    assert Bd.exact_cost([4, 3, 6, 9], 4, 6) == 50.0
    assert Bd.adaptive_width([4, 3, 6, 9], 4, 6) == 4
    # B = 20: h = 10, U = 4, 3, 6, 12, ..., 6 * 2^8 -> C = 2 * (7 + 6 * 511)
    assert Bd.exact_cost([4, 3, 6], 4, 20) == 2.0 * (7 + 6 * 511)
    assert Bd.adaptive_width([4, 3, 6], 4, 20) == -(-2 * (7 + 6 * 511) // 320)
    assert Bd.exact_cost([4, 4, 2], 4, 9) is None
    assert Bd.adaptive_width([4, 4, 2], 4, 9) == 4
    assert Bd.adaptive_width([4, 5, 10 ** 9], 4, 400) == Bd.MAX_WIDTH


def test_bound_invariants():
    seen_second = seen_exact = 0
    for i in range(24):
        n, k = 6 + 3 * i, 2 + i % 3
        d, _ = I.first_synchronizing(n, k, I.member_seed(913, i), O.is_synchronizing)
        R, w, w1, src = Bd.upper_bound(n, k, d)
        r = O.bidir(n, k, d)[0]
        ew, _ = O.eppstein(n, k, d)
        R0, _, sizes = O.beam_sizes(n, k, d, n)
        assert len(w) == R and O.verify(n, k, d, w)
        assert r <= R <= len(ew)
        if R0 is not None:
            assert R <= R0
        assert n <= w1 <= Bd.MAX_WIDTH
        if all(u <= n for u in sizes):
            assert R0 == r and R == r and w1 == n
            seen_exact += 1
        seen_second += src == 2
    assert seen_exact > 0
    assert Bd.upper_bound(1, 2, [0, 0]) == (0, [], 1, 0)


def test_second_beam_on_larger_automata():
    """n = 150 .. 200: the first beam cuts, the policy widens the beam."""
    for i, (n, k) in enumerate([(150, 2), (200, 2)]):
        d, _ = I.first_synchronizing(n, k, I.member_seed(1913, i), O.is_synchronizing)
        R, w, w1, src = Bd.upper_bound(n, k, d)
        R0 = O.beam_sizes(n, k, d, n)[0]
        assert w1 > n and O.verify(n, k, d, w) and len(w) == R
        assert R <= len(O.eppstein(n, k, d)[0]) and (R0 is None or R <= R0)
