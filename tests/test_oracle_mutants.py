"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle source (on the
CPU, in a temporary directory), compiles it, and runs a quick subset of the
pins of test_oracle.py against it: the hand-worked examples, the Černý closed
form, and agreement with the trivial word enumeration.  Every mutant must fail
at least one of them.
"""

import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_05495_amd import inputs as I

MUTANTS = {
    # image indexes delta as if it were state-major
    "image_wrong_index": [("setbit(X, delta[(int64_t)a * n + q])",
                           "setbit(X, delta[((int64_t)q * k + a) % ((int64_t)n * k)])")],
    # preimage tests the source state instead of its target
    "preimage_no_delta": [("if (getbit(S, delta[(int64_t)a * n + q])) setbit(Y, q);",
                           "if (getbit(S, q)) setbit(Y, delta[(int64_t)a * n + q]);")],
    # meet tests Y subset X
    "meet_swapped": [("hit = is_subset(A_row(c, a), B_row(c, b), c->W);",
                      "hit = is_subset(B_row(c, b), A_row(c, a), c->W);"),
                     ("if (is_subset(level_row(F, lf, i), level_row(B, lb, marked[t]), W)) {",
                      "if (is_subset(level_row(B, lb, marked[t]), level_row(F, lf, i), W)) {")],
    # duplicates keep the largest key instead of the least
    "dedup_keeps_last": [("return (a > b) - (a < b);", "return (a < b) - (a > b);")],
    # inverse candidates generated parent-major (decoded consistently)
    "inverse_parent_major": [
        ("orc_preimage(n, k, delta, a, level_row(s, L, i), cand + ((int64_t)a * m + i) * W);",
         "orc_preimage(n, k, delta, a, level_row(s, L, i), cand + (i * k + a) * W);"),
        ("out[pos] = (uint8_t)(g / prev);\n        j = g % prev;",
         "out[pos] = (uint8_t)(g % (g >= 0 ? (int64_t)run_k : 1));\n        j = g / run_k;")],
    # Alg. 2 split on the wrong side of the binary search
    "mark_split_wrong": [("if (getbit(A_row(c, mid), d)) hi = mid; else lo = mid + 1;",
                          "if (!getbit(A_row(c, mid), d)) hi = mid; else lo = mid + 1;")],
    # inverse half of the word read back to front
    "trace_inverse_reversed": [("out[pos] = (uint8_t)(g / prev);",
                                "out[L - 1 - pos] = (uint8_t)(g / prev);")],
    # sync check never merges through letters
    "sync_no_letters": [("if (m[(size_t)pp * n + qq]) {", "if (pp == qq) {")],
}


def build_mutant(name, edits, tmpdir):
    src = open(O.SRC).read()
    if name == "inverse_parent_major":
        src = src.replace("static void trace_inverse(const Side *s, int L, int64_t j, uint8_t *out) {",
                          "static int64_t run_k = 2;\n"
                          "static void trace_inverse(const Side *s, int L, int64_t j, uint8_t *out) {")
        src = src.replace("    run->n = n; run->k = k;", "    run->n = n; run->k = k; run_k = k;")
    for old, new in edits:
        assert old in src, (name, old)
        src = src.replace(old, new)
    path = os.path.join(tmpdir, f"{name}.c")
    so = os.path.join(tmpdir, f"lib{name}.so")
    with open(path, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w", "-o", so, path])
    return so


def pins_hold():
    """Quick subset of the pins; False as soon as one fails."""
    from tests.test_oracle import load_hand_examples
    try:
        for n, k, d, r, w in load_hand_examples():
            if r == O.ENOTSYNC:
                if O.is_synchronizing(n, k, d):
                    return False
                continue
            if O.bidir(n, k, d)[:2] != (r, w) or O.bidir(n, k, d, meet=0)[:2] != (r, w):
                return False
        for n in range(2, 12):
            got = O.bidir(n, 2, I.cerny(n))[:2]
            if got != ((n - 1) ** 2, I.cerny_word(n)):
                return False
        for i in range(200):
            n, k = 3 + i % 12, 2 + i % 3
            d = I.random_automaton(n, k, I.member_seed(31337, i))
            if not O.is_synchronizing(n, k, d):
                continue
            if O.bidir(n, k, d)[:2] != O.bruteforce(n, k, d, 30):
                return False
        for i in range(10):
            d = I.random_automaton(40, 2, I.member_seed(7, i))
            if not O.is_synchronizing(40, 2, d):
                continue
            r, w, _ = O.bidir(40, 2, d)
            if not O.verify(40, 2, d, w):
                return False
    except O.OracleError:
        return False
    return True


# planted mistakes in the self-reduction of new levels
REDUCE_MUTANTS = {
    # forward drops sets that contain another, inverse sets inside another: swapped
    "reduce_direction_swapped": [("if (dir == 0 ? is_subset(B, A, W) : is_subset(A, B, W)) drop[i] = 1;",
                                  "if (dir == 0 ? is_subset(A, B, W) : is_subset(B, A, W)) drop[i] = 1;")],
    # the forward rule on both sides
    "reduce_same_rule_both_sides": [("if (dir == 0 ? is_subset(B, A, W) : is_subset(A, B, W)) drop[i] = 1;",
                                     "if (is_subset(B, A, W)) drop[i] = 1;")],
    # rows move down but their parent keys stay
    "reduce_parents_not_moved": [("            s->par[pos] = s->par[base + i];\n", "")],
    # a set counts as its own proper subset
    "reduce_compares_with_itself": [("            if (j == i) continue;\n", "")],
    # the visited index is not rebuilt after the level shrank
    "reduce_stale_visited_index": [("    for (int64_t t = 0; t < s->nrows; t++) s->sorted[t] = t;\n",
                                    "    if (0) for (int64_t t = 0; t < s->nrows; t++) s->sorted[t] = t;\n")],
}


# planted mistakes in the reductions through Alg. 2
ALG2_MUTANTS = {
    # the proper-superset leaf compares a set with itself: every set is dropped
    "alg2_not_proper": [("                if (c->proper && c->A[a] == c->B[b]) continue;\n", "")],
    # the mask of the last word also clears the last state
    "alg2_mask_drops_last_state": [("(((u64)1 << (n - lo)) - 1);", "(((u64)1 << (n - lo - 1)) - 1);")],
    # the inverse side marked without complementing
    "alg2_inverse_not_complemented": [("    if (dir == 1) {\n        /* complements",
                                       "    if (0) {\n        /* complements")],
    # history marks run on the history itself instead of the new level
    "alg2_history_wrong_list": [("if (!rc && nh) rc = alg2_mark(hist, nh, lev, m, n, W, 0, drop, tests);",
                                 "if (!rc && nh) rc = alg2_mark(lev, m, hist, nh < m ? nh : m, n, W, 0, drop, tests);")],
}


def alg2_pins_hold():
    from tests.test_oracle import same_search, reduction_cases
    try:
        for n, k, d in reduction_cases(24, base=777):
            for reduce in (True, "history"):
                a = O.bidir(n, k, d, reduce=reduce, keep_levels=True)
                b = O.bidir(n, k, d, reduce=reduce, keep_levels=True, alg2=True)
                if not same_search(a, b):
                    return False
        for n in (63, 65):
            d, _ = I.first_synchronizing(n, 2, I.member_seed(4321, 0), O.is_synchronizing)
            a = O.bidir(n, 2, d, reduce=True, keep_levels=True)
            b = O.bidir(n, 2, d, reduce=True, keep_levels=True, alg2=True)
            if not same_search(a, b):
                return False
    except O.OracleError:
        return False
    return True


# planted mistakes in the reduction by history
HISTORY_MUTANTS = {
    # forward drops sets inside an earlier set, inverse sets containing one: swapped
    "history_direction_swapped": [("if (dir == 0 ? is_subset(H, A, W) : is_subset(A, H, W)) drop[i] = 1;",
                                   "if (dir == 0 ? is_subset(A, H, W) : is_subset(H, A, W)) drop[i] = 1;")],
    # the level being reduced counts as history, so each set meets itself
    "history_includes_own_level": [("history && h < base && !drop[i]",
                                    "history && h < base + m && !drop[i]")],
    # the level just before the new one is left out of the history
    "history_skips_previous_level": [("history && h < base && !drop[i]",
                                      "history && h < s->off[L - 1] && !drop[i]")],
    # history reduction never switched on
    "history_never_applied": [("side ? &run->B : &run->F, side, reduce & 2, reduce & 4,",
                               "side ? &run->B : &run->F, side, 0, reduce & 4,")],
}


def reduction_pins_hold(reduce=True):
    """The pins of the self-reduced (or history-reduced) search; False as
    soon as one fails."""
    from tests.test_oracle import reduced_levels_hold, reduction_cases
    try:
        for n, k, d in reduction_cases(24):
            r0 = O.bidir(n, k, d)[0]
            r1, w1, _ = O.bidir(n, k, d, reduce=reduce)
            if r1 != r0 or len(w1) != r1 or not O.verify(n, k, d, w1):
                return False
        for n, k, d in reduction_cases(16, base=4242):
            if not reduced_levels_hold(n, k, d, reduce=reduce):
                return False
    except O.OracleError:
        return False
    return True


# planted mistakes in the Eppstein heuristic
EPPSTEIN_MUTANTS = {
    # the diagonal starts at 1: every distance one too long
    "pair_dist_off_by_one": [("dist[(size_t)p * n + q] = p == q ? 0 : -1;",
                              "dist[(size_t)p * n + q] = p == q ? 1 : -1;")],
    # the last letter reaching distance d - 1 instead of the least
    "pair_dist_last_letter": [("                        any = 1;\n                        break;\n",
                               "                        any = 1;\n")],
    # equal distances go to the last pair
    "greedy_ties_last": [("if (bp < 0 || d < bd) { bp = p; bq = q; bd = d; }",
                          "if (bp < 0 || d <= bd) { bp = p; bq = q; bd = d; }")],
    # the pair with the longest merging word
    "greedy_longest_pair": [("if (bp < 0 || d < bd) { bp = p; bq = q; bd = d; }",
                             "if (bp < 0 || d > bd) { bp = p; bq = q; bd = d; }")],
    # only the first letter of each round's word
    "greedy_one_letter_rounds": [("for (int t = 0; t < bd; t++) {", "for (int t = 0; t < 1; t++) {")],
    # the pair is not followed through the round's letters
    "greedy_pair_not_followed": [("            p = delta[(int64_t)a * n + p];\n"
                                  "            q = delta[(int64_t)a * n + q];\n", "")],
}


def eppstein_pins_hold():
    from tests.test_eppstein_oracle import check_rounds, enumerated_dist, tiny_cases
    try:
        for n, k, d in tiny_cases()[::3]:
            dist, nxt = O.pair_dist(n, k, d)
            want, first = enumerated_dist(n, k, d)
            if not np.array_equal(dist, want):
                return False
            for (p, q), w in first.items():
                if w and nxt[p, q] != w[0]:
                    return False
            if not O.is_synchronizing(n, k, d):
                continue
            word, rounds = O.eppstein(n, k, d)
            try:
                check_rounds(n, k, d, word, rounds, want, first)
            except AssertionError:
                return False
    except O.OracleError:
        return False
    return True


@pytest.mark.parametrize("name", sorted(EPPSTEIN_MUTANTS))
def test_eppstein_mutant_is_caught(name, tmp_path):
    so = build_mutant(name, EPPSTEIN_MUTANTS[name], str(tmp_path))
    saved = O._lib
    try:
        O._lib = O.bind(so)
        assert not eppstein_pins_hold(), f"planted mistake {name} went unnoticed"
    finally:
        O._lib = saved


def test_unmutated_oracle_passes():
    assert pins_hold()
    assert reduction_pins_hold()
    assert reduction_pins_hold("history")
    assert alg2_pins_hold()
    assert eppstein_pins_hold()


@pytest.mark.parametrize("name", sorted(REDUCE_MUTANTS))
def test_reduction_mutant_is_caught(name, tmp_path):
    so = build_mutant(name, REDUCE_MUTANTS[name], str(tmp_path))
    saved = O._lib
    try:
        O._lib = O.bind(so)
        assert not reduction_pins_hold(), f"planted mistake {name} went unnoticed"
    finally:
        O._lib = saved


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    so = build_mutant(name, MUTANTS[name], str(tmp_path))
    saved = O._lib
    try:
        O._lib = O.bind(so)
        assert not pins_hold(), f"planted mistake {name} went unnoticed"
    finally:
        O._lib = saved


@pytest.mark.parametrize("name", sorted(HISTORY_MUTANTS))
def test_history_mutant_is_caught(name, tmp_path):
    so = build_mutant(name, HISTORY_MUTANTS[name], str(tmp_path))
    saved = O._lib
    try:
        O._lib = O.bind(so)
        assert not reduction_pins_hold("history"), f"planted mistake {name} went unnoticed"
    finally:
        O._lib = saved


@pytest.mark.parametrize("name", sorted(ALG2_MUTANTS))
def test_alg2_mutant_is_caught(name, tmp_path):
    so = build_mutant(name, ALG2_MUTANTS[name], str(tmp_path))
    saved = O._lib
    try:
        O._lib = O.bind(so)
        assert not alg2_pins_hold(), f"planted mistake {name} went unnoticed"
    finally:
        O._lib = saved
