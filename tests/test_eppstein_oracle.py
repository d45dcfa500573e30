"""Pins of the oracle's Eppstein heuristic (orc_pair_dist, orc_eppstein)
against what the definitions fix, computed here without the oracle:

- pair distances and their first letters against enumeration of all words
  in length order (the shortest word that merges each pair), on tiny
  automata where every word up to the largest possible pair distance,
  n(n-1)/2, can be listed;
- every round of the greedy: the chosen pair lies in the current set, has
  the least enumerated distance among its pairs (least p, then q, on ties),
  and the round's letters follow the least-first-letter shortest merging
  words; the set shrinks every round;
- the result resets the automaton, is at least r (trivial enumeration), at
  most (n^3 - n)/3 (the bound quoted in Section 1.3.2), and equals r for
  n = 2 (a single pair).
"""

import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_05495_amd import inputs as I


def word_maps(n, k, delta, max_len):
    """(word, map) for every word of length 0..max_len in length-then-lex
    order, map[q] = delta(q, word)."""
    D = np.asarray(delta, dtype=np.int64).reshape(k, n)
    level = [((), np.arange(n))]
    out = list(level)
    for _ in range(max_len):
        nxt = []
        for w, m in level:
            for a in range(k):
                nxt.append((w + (a,), D[a][m]))
        out += nxt
        level = nxt
    return out


def enumerated_dist(n, k, delta):
    """Shortest merging length of each pair, and its lex-least shortest
    merging word, from the word list."""
    maxd = n * (n - 1) // 2
    dist = -np.ones((n, n), dtype=np.int64)
    first = {}
    np.fill_diagonal(dist, 0)
    for w, m in word_maps(n, k, delta, maxd):
        for p in range(n):
            for q in range(p + 1, n):
                if dist[p, q] < 0 and m[p] == m[q]:
                    dist[p, q] = dist[q, p] = len(w)
                    first[(p, q)] = w
    return dist, first


def tiny_cases():
    out = []
    for i in range(400):
        n, k = 2 + i % 4, 1 + i % 3
        if k ** (n * (n - 1) // 2) > 5000:
            continue
        out.append((n, k, I.random_automaton(n, k, I.member_seed(515, i))))
    out.append((4, 2, I.cerny(4)))
    out.append((5, 2, I.cerny(5)))
    return out


def test_pair_dist_matches_word_enumeration():
    unmerged = 0
    for n, k, d in tiny_cases():
        dist, nxt = O.pair_dist(n, k, d)
        want, first = enumerated_dist(n, k, d)
        assert np.array_equal(dist, want), (n, k, list(d))
        for p in range(n):
            for q in range(p + 1, n):
                if want[p, q] > 0:
                    # the least first letter of a shortest merging word: the
                    # lex-least shortest word starts with it
                    assert nxt[p, q] == nxt[q, p] == first[(p, q)][0]
                else:
                    unmerged += 1
                    assert nxt[p, q] == 255
    assert unmerged > 0          # some non-synchronizing pairs were covered


def check_rounds(n, k, d, word, rounds, dist, lexw):
    """Replay the rounds with enumerated distances."""
    D = np.asarray(d, dtype=np.int64).reshape(k, n)
    S = set(range(n))
    pos = 0
    for p, q, dd in rounds:
        assert p < q and p in S and q in S
        pairs = [(dist[x, y], x, y) for x, y in itertools.combinations(sorted(S), 2)]
        assert (dd, p, q) == min(pairs)
        seg = word[pos:pos + dd]
        assert tuple(seg) == lexw[(p, q)]
        before = len(S)
        for a in seg:
            S = {int(D[a][s]) for s in S}
        assert len(S) < before
        pos += dd
    assert pos == len(word) and len(S) == 1


def lex_least_merging_words(n, k, d, dist):
    """For each pair, the letters of the greedy's segment as the
    definitions fix them: the lex-least shortest merging word."""
    return enumerated_dist(n, k, d)[1]


def test_greedy_rounds_follow_the_definition():
    done = 0
    for n, k, d in tiny_cases():
        if not O.is_synchronizing(n, k, d):
            with pytest.raises(O.OracleError) as e:
                O.eppstein(n, k, d)
            assert e.value.code == O.ENOTSYNC
            continue
        word, rounds = O.eppstein(n, k, d)
        dist, first = enumerated_dist(n, k, d)
        check_rounds(n, k, d, word, rounds, dist, first)
        r, _ = O.bruteforce(n, k, d, 40)
        assert r <= len(word) <= (n ** 3 - n) // 3
        if n == 2:
            assert len(word) == r
        done += 1
    assert done > 100


def test_greedy_on_larger_automata():
    """Resets, r <= length <= (n^3 - n)/3, rounds shrink the set, on
    automata where the exact r comes from the oracle's bidirectional
    search (pinned elsewhere), and the Černý series where r = (n-1)^2."""
    for i in range(30):
        n, k = 8 + 3 * i, 2 + i % 3
        d, _ = I.first_synchronizing(n, k, I.member_seed(77, i), O.is_synchronizing)
        word, rounds = O.eppstein(n, k, d)
        assert O.verify(n, k, d, word)
        r = O.bidir(n, k, d)[0]
        assert r <= len(word) <= (n ** 3 - n) // 3
        assert 1 <= len(rounds) <= n - 1
        assert sum(x[2] for x in rounds) == len(word)
    for n in range(2, 30):
        word, rounds = O.eppstein(n, 2, I.cerny(n))
        assert O.verify(n, 2, I.cerny(n), word)
        assert len(word) >= (n - 1) ** 2


def test_word_cap_reports_the_length():
    d = I.cerny(10)
    word, _ = O.eppstein(10, 2, d)
    import ctypes
    buf = np.zeros(5, dtype=np.uint8)
    ln = ctypes.c_int64(-1)
    rc = O.lib().orc_eppstein(10, 2, O._ptr(O._delta(d), ctypes.c_int32),
                              O._ptr(buf, ctypes.c_uint8), 5, ctypes.byref(ln), None, None)
    assert rc == O.EWORDCAP and ln.value == len(word)
    assert list(buf) == word[:5]
    assert O.eppstein(1, 3, [0, 0, 0]) == ([], [])
