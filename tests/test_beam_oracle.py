"""Pins of the oracle's beam search (CutOff-IBFS, an upper bound R >= r):
R is never below the exact r and its word resets the automaton; with a beam
wider than every level it is the plain search's inverse side, so R = r and
the word is the lex-least one; on Černý automata with a wide beam the unique
shortest word comes back; and on tiny automata a separate set-based search
written here, step by step from the definition, gives the same R and word."""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_05495_amd import inputs as I


def rand(n, k, i, base=I.BASE_SEED ^ 0xBEA):
    d, _ = I.first_synchronizing(n, k, I.member_seed(base, i), O.is_synchronizing)
    return d


def test_beam_bounds_the_reset_threshold_and_its_word_resets():
    for i, (n, k) in enumerate([(8, 2), (16, 2), (24, 3), (40, 2), (64, 2), (64, 3), (90, 2)]):
        d = rand(n, k, i)
        r = O.bidir(n, k, d)[0]
        for width in (1, 2, 4, 16, 64, int(n * math.log(n)) + 1):
            R, w, info = O.beam(n, k, d, width)
            assert info["widest"] <= width
            if R is None:                  # the cut led into a dead end
                continue
            assert R >= r, (n, k, width)
            assert len(w) == R and O.verify(n, k, d, w)


def test_unbounded_beam_is_the_plain_inverse_search():
    for i, (n, k) in enumerate([(5, 2), (12, 2), (20, 3), (33, 2), (48, 2), (56, 3)]):
        d = rand(n, k, i, base=77)
        r, w, _ = O.bidir(n, k, d)
        R, wb, info = O.beam(n, k, d, 1 << 40)
        assert (R, list(wb)) == (r, list(w)), (n, k)
        assert info["cut"] == 0


@pytest.mark.parametrize("n", [3, 6, 10, 14])
def test_cerny_with_a_wide_beam(n):
    # the inverse side of C_n reaches n(n-1)+1 sets in all, so no level is cut
    R, w, _ = O.beam(n, 2, I.cerny(n), n * (n - 1) + 1)
    assert R == (n - 1) ** 2 and list(w) == I.cerny_word(n)
    R1, w1, _ = O.beam(n, 2, I.cerny(n), 1)
    assert R1 is None or (R1 >= (n - 1) ** 2 and O.verify(n, 2, I.cerny(n), w1))


def small_beam(n, k, delta, width, max_steps=200):
    """The beam search on Python sets of states: level 0 the singletons;
    a step takes preimages letter by letter (letter-major keys), keeps the
    first occurrence of each nonempty set not seen before (cut sets count as
    seen), then keeps the `width` largest, ties to the earlier key; stops at
    the first level holding every state, or at an empty level."""
    d = np.asarray(delta).reshape(k, n)
    level = [(frozenset([q]), None) for q in range(n)]     # (set, key)
    seen = {s for s, _ in level}
    levels = []

    def cut(lv):
        if len(lv) <= width:
            return lv
        order = sorted(range(len(lv)), key=lambda i: (-len(lv[i][0]), i))
        keep = sorted(order[:width])
        return [lv[i] for i in keep]

    level = cut(level)
    levels.append(level)
    full = frozenset(range(n))
    for depth in range(1, max_steps + 1):
        prev = levels[-1]
        cand = []
        for a in range(k):
            for i, (S, _) in enumerate(prev):
                Y = frozenset(q for q in range(n) if d[a, q] in S)
                cand.append((Y, a * len(prev) + i))
        new = []
        for Y, g in cand:
            if Y and Y not in seen:
                seen.add(Y)
                new.append((Y, g))
        if not new:
            return None, None
        new = cut(new)
        levels.append(new)
        for j, (Y, _) in enumerate(new):
            if Y == full:
                word, jj = [], j
                for dd in range(depth, 0, -1):
                    g = levels[dd][jj][1]
                    m = len(levels[dd - 1])
                    word.append(g // m)
                    jj = g % m
                return depth, word
    return None, None


def test_beam_equals_a_set_based_search_on_tiny_automata():
    checked = 0
    for i in range(150):
        n = 3 + i % 6
        k = 2 + (i % 3 == 0)
        d = rand(n, k, i, base=4242)
        for width in (1, 2, 3, 5):
            R, w, _ = O.beam(n, k, d, width)
            Rs, ws = small_beam(n, k, d, width)
            assert (R, None if w is None else list(w)) == (Rs, ws), (n, k, i, width)
            checked += R is not None
    assert checked > 300
