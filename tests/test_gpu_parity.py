"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Results (r and the lex-least reset word) are integers and words: the bar is
bit-exact equality.  Per-level tests compare the device lists (sets, order,
parent keys) with the oracle's level by level.
"""

import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_05495_amd import inputs as I
from paper_2207_05495_amd import srw

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    srw.use_torch(0)
    for key, v in DEFAULTS:
        srw.set_option(key, v)
    yield
    for key, v in DEFAULTS:
        srw.set_option(key, v)


DEFAULTS = (("schedule", 0), ("meet_tiles", 0), ("keep_levels", 0), ("budget", 0), ("meet", 0),
            ("max_slots", 4096), ("meet_rows", 512), ("meet_groups", 16), ("meet_order", 1),
            ("meet_grid", 0), ("small_cand", 2048), ("ysort", 0), ("deadline_ms", 0),
            ("verbose", 0), ("persist", 1), ("bucket", 16384), ("meet_xcd", 0), ("meet_bgrid", 4096))


def say(*a):
    print(*a, flush=True)


def rand_sync(n, k, i, base=I.BASE_SEED):
    d, _ = I.first_synchronizing(n, k, I.member_seed(base, i), O.is_synchronizing)
    return d


def _stored():
    """(r, word) the oracle stored under tests/golden, keyed by the bytes of
    the transition table (rebuilt from each entry's seed and attempt)."""
    out = {}
    for name in sorted(os.listdir(GOLDEN)):
        if not name.endswith(".json"):
            continue
        with open(os.path.join(GOLDEN, name)) as f:
            rec = json.load(f)
        for c in rec.get("cases", []):
            if "r" not in c or "attempt" not in c:
                continue
            d = I.random_automaton(c["n"], c["k"], c["seed"], c["attempt"])
            w = c["word"]
            out[(c["n"], c["k"], d.tobytes())] = (c["r"], [int(x) for x in w] if isinstance(w, str) else list(w))
    return out


_MEMO = {}


def oracle_rw(n, k, d):
    """(r, word) of the oracle: a value it stored, or computed now (once per
    session)."""
    if not _MEMO:
        _MEMO.update(_stored())
    key = (n, k, np.asarray(d, dtype=np.int32).tobytes())
    if key not in _MEMO:
        _MEMO[key] = tuple(O.bidir(n, k, d)[:2])
    return _MEMO[key]


# --------------------------------------------------------------- golden

def hand_cases():
    from tests.test_oracle import load_hand_examples
    return load_hand_examples()


@pytest.mark.parametrize("case", hand_cases())
def test_hand_examples(case):
    n, k, d, r, w = case
    say("hand", n, k, d)
    if r == O.ENOTSYNC:
        with pytest.raises(srw.SrwError) as e:
            srw.solve(n, k, d)
        assert e.value.code == srw.ENOTSYNC
    else:
        assert srw.solve(n, k, d) == (r, w)


@pytest.mark.parametrize("n", list(range(2, 41)))
def test_cerny(n):
    say("cerny", n)
    assert srw.solve(n, 2, I.cerny(n)) == ((n - 1) ** 2, I.cerny_word(n))


@pytest.mark.parametrize("n", list(range(2, 21)))
def test_sink_series(n):
    """Rystsov's sink series: n - 1 letters, r = n(n - 1)/2, word in closed
    form; the oracle agrees on these sizes."""
    say("sink series", n)
    d = I.sink_series(n)
    want = (n * (n - 1) // 2, I.sink_word(n))
    assert srw.solve(n, n - 1, d) == want
    if n <= 16:
        assert O.bidir(n, n - 1, d)[:2] == want


def test_sink_series_paper_member():
    """The member with 26 states and 25 letters: r = 325 (Section 3.1.1),
    with the closed-form lex-least word."""
    import time
    say("sink series 26")
    t = time.perf_counter()
    got = srw.solve(26, 25, I.sink_series(26))
    say(f"sink series 26: {time.perf_counter() - t:.2f} s")
    assert got == (325, I.sink_word(26))


# ------------------------------------------------------ random vs oracle

def test_random_n64_k2_100_seeds():
    """n=64, k=2, one 64-bit word per subset: 100 seeds."""
    for i in range(100):
        d = rand_sync(64, 2, i)
        say("n=64 seed", i)
        assert srw.solve(64, 2, d) == O.bidir(64, 2, d)[:2]


@pytest.mark.parametrize("n,k", [(63, 2), (65, 2), (127, 2), (128, 2), (129, 3), (191, 2),
                                 (192, 2), (193, 2), (100, 4), (40, 7)])
def test_ragged_widths(n, k):
    for i in range(3):
        d = rand_sync(n, k, i, base=77)
        say("ragged", n, k, i)
        assert srw.solve(n, k, d) == oracle_rw(n, k, d)


def max_size_automaton(n, seed):
    """Letter 0 halves every state (q -> q // 2), letter 1 is a random
    permutation: r <= ceil(log2 n), so the oracle is quick at n = 512."""
    rng = np.random.default_rng(seed)
    half = (np.arange(n) // 2).astype(np.int32)
    perm = rng.permutation(n).astype(np.int32)
    return np.concatenate([half, perm])


@pytest.mark.parametrize("n", [449, 511, 512])
def test_max_width(n):
    for s in range(3):
        d = max_size_automaton(n, s)
        say("max width", n, s)
        assert srw.solve(n, 2, d) == oracle_rw(n, 2, d)


# ------------------------------------------------------ per-level parity

@pytest.mark.parametrize("n,k,i", [(20, 2, 0), (64, 2, 1), (100, 3, 2), (130, 2, 3),
                                   (200, 2, 4), (70, 4, 5), (33, 3, 6)])
def test_levels_match_oracle(n, k, i):
    d = rand_sync(n, k, i, base=555)
    say("levels", n, k, i)
    srw.set_option("keep_levels", 1)
    try:
        got = srw.solve(n, k, d)
        gl = [srw.last_levels(side, (n + 63) // 64) for side in (0, 1)]
    finally:
        srw.set_option("keep_levels", 0)
    r, w, info = O.bidir(n, k, d, keep_levels=True)
    assert got == (r, w)
    for side in (0, 1):
        ol = info["levels"][side]
        assert len(gl[side]) == len(ol)
        for L, ((grows, gpar), (orows, opar)) in enumerate(zip(gl[side], ol)):
            assert np.array_equal(grows, orows), (side, L)
            if L > 0:
                assert np.array_equal(gpar.astype(np.int64), opar), (side, L)


# ------------------------------------------------------ invariances

@pytest.mark.parametrize("sched", [(1, 1), (1, 7), (1, 99), (2, 0)])
def test_schedule_invariance(sched):
    mode, seed = sched
    cases = [(rand_sync(90, 2, j, base=31), 90, 2) for j in range(3)]
    cases.append((I.cerny(20), 20, 2))
    want = [srw.solve(n, k, d) for d, n, k in cases]
    srw.set_option("schedule", mode)
    srw.set_option("sched_seed", seed)
    try:
        for (d, n, k), w in zip(cases, want):
            say("schedule", mode, seed, n)
            assert srw.solve(n, k, d) == w
    finally:
        srw.set_option("schedule", 0)


def cost_cases():
    from tests.test_schedule_oracle import cases
    return cases()


def test_cost_model_schedule_sides_and_results():
    """Schedule 3 (Section 2.1.2's step costs): with every step chosen by
    the host, the side of each step equals the oracle's cost-model choice
    (oracle/schedule.py, written separately), and r and word equal the
    oracle's."""
    from oracle import schedule as S
    srw.set_option("schedule", 3)
    srw.set_option("persist", 0)
    srw.set_option("keep_levels", 1)
    try:
        for n, k, d in cost_cases():
            say("cost schedule", n, k)
            assert srw.solve(n, k, d) == oracle_rw(n, k, d)
            assert srw.last_sides() == S.cost_sides(n, k, d), (n, k)
    finally:
        srw.set_option("schedule", 0)
        srw.set_option("persist", 1)
        srw.set_option("keep_levels", 0)


def test_recorded_sides_follow_the_frontier_rule():
    """Schedule 0 with the one-launch small steps on: the sides the runner
    and the host took, in order, are the oracle's (smaller list first, ties
    forward)."""
    srw.set_option("keep_levels", 1)
    try:
        for n, k, d in cost_cases() + [(24, 2, I.cerny(24))]:
            say("frontier sides", n, k)
            srw.solve(n, k, d)
            assert srw.last_sides() == O.bidir(n, k, d)[2]["sides"], (n, k)
    finally:
        srw.set_option("keep_levels", 0)


def test_cost_model_schedule_per_width_in_a_batch():
    """Schedule 3 for some set widths only, the one-launch small steps on:
    a batch of mixed widths keeps the oracle's r and word, and so does the
    n = 256 automaton stored by the oracle."""
    cs = [(n, k, d) for n, k, d in cost_cases()]
    cs += [(n, 2, rand_sync(n, 2, i, base=55)) for i, n in enumerate((130, 190, 200))]
    want = [oracle_rw(n, k, d) for n, k, d in cs]
    for w in (1, 3, 4):
        srw.set_option(f"schedule@{w}", 3)
    srw.set_option("schedule@2", 2)
    try:
        res = srw.solve_batch(cs)
        assert [(st, (r, wd)) for st, r, wd in res] == [(srw.OK, w) for w in want]
        c = golden("rand256.json")[0]
        d = I.random_automaton(c["n"], c["k"], c["seed"], c["attempt"])
        r, w = srw.solve(c["n"], c["k"], d)
        assert r == c["r"] and "".join(map(str, w)) == c["word"]
    finally:
        for w in (1, 2, 3, 4):
            srw.set_option(f"schedule@{w}", -1)


@pytest.mark.parametrize("tiles", [1, 2, 3, 8, 32])
def test_meet_tile_shape_invariance(tiles):
    d = rand_sync(150, 2, 4, base=8)
    want = O.bidir(150, 2, d)[:2]
    srw.set_option("meet_tiles", tiles)
    try:
        say("meet tiles", tiles)
        assert srw.solve(150, 2, d) == want
    finally:
        srw.set_option("meet_tiles", 0)


@pytest.mark.parametrize("mode", [1, 2])
def test_meet_modes_agree(mode):
    """Mode 1 tests every X against LDS tiles; mode 2 bucket-sorts every
    forward level and tests 64-set chunks (including tiny levels and chunks
    with no common state).  Both must reproduce the oracle."""
    cases = [(64, 2), (150, 2), (200, 3), (129, 2), (40, 4), (255, 2), (90, 3)]
    srw.set_option("meet", mode)
    try:
        for j, (n, k) in enumerate(cases):
            d = rand_sync(n, k, j, base=61)
            say("meet mode", mode, n, k)
            assert srw.solve(n, k, d) == oracle_rw(n, k, d)
        for n in (5, 17, 33):
            assert srw.solve(n, 2, I.cerny(n)) == ((n - 1) ** 2, I.cerny_word(n))
    finally:
        srw.set_option("meet", 0)


def many_common_states(n, seed):
    """Letter 0 fixes every state >= 16 and scrambles 0..15; letter 1 is a
    random map.  Forward sets reached through 0s share dozens of states, so
    64-set chunks have far more than 8 common states."""
    rng = np.random.default_rng(seed)
    a = np.arange(n, dtype=np.int32)
    a[:16] = rng.integers(0, 16, 16)
    b = rng.integers(0, n, n).astype(np.int32)
    return np.concatenate([a, b])


@pytest.mark.parametrize("n", [70, 130, 200])
def test_chunked_meet_with_large_common_sets(n):
    srw.set_option("meet", 2)
    try:
        for s in range(4):
            d = many_common_states(n, s)
            if not O.is_synchronizing(n, 2, d):
                continue
            say("many common states", n, s)
            assert srw.solve(n, 2, d) == oracle_rw(n, 2, d)
    finally:
        srw.set_option("meet", 0)


def test_meet_mode_levels_and_batch():
    """Forced chunked meet with schedule changes and a batch of mixed sizes."""
    cases = mixed_cases(30, 2024)
    want = [oracle_rw(n, k, d) for n, k, d in cases]
    srw.set_option("meet", 2)
    srw.set_option("schedule", 1)
    srw.set_option("sched_seed", 5)
    try:
        say("meet mode 2 batch")
        res = srw.solve_batch(cases)
        assert [(r, w) for _, r, w in res] == want
    finally:
        srw.set_option("meet", 0)
        srw.set_option("schedule", 0)


def test_relabel_invariance():
    n, k = 120, 2
    d = rand_sync(n, k, 9, base=17)
    want = srw.solve(n, k, d)
    for s in range(3):
        perm = np.random.default_rng(s).permutation(n)
        say("relabel", s)
        assert srw.solve(n, k, I.relabel(d, n, k, perm)) == want


# ------------------------------------------------------ batch and serving

def mixed_cases(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        if i % 10 == 9:
            n = int(rng.integers(8, 25))
            out.append((n, 2, I.cerny(n)))
        else:
            n = int(rng.integers(24, 110))
            k = int(rng.integers(2, 4))
            out.append((n, k, rand_sync(n, k, i, base=seed)))
    return out


def test_fuzz_batch_against_the_oracle():
    """400 seeded random automata, n = 1 .. 120 (1 .. 80 for k >= 4), k = 1 ..
    6, uniform delta without the redraw (so 66 are not synchronizing), in
    one batch: every r and word equals the oracle's, every
    non-synchronizing member is SRW_ENOTSYNC, and so is the oracle's."""
    rng = np.random.default_rng(2024)
    cases = []
    for i in range(400):
        k = int(rng.integers(1, 7))
        n = int(rng.integers(1, 81 if k >= 4 else 121))
        cases.append((n, k, I.random_automaton(n, k, I.member_seed(99991, i))))
    want = [O.bidir(n, k, d)[:2] if O.is_synchronizing(n, k, d) else None for n, k, d in cases]
    assert sum(w is None for w in want) > 20
    say("fuzz batch", len(cases))
    got = srw.solve_batch(cases)
    for (n, k, _), g, w in zip(cases, got, want):
        if w is None:
            assert g[0] == srw.ENOTSYNC, (n, k)
        else:
            assert g == (srw.OK, w[0], w[1]), (n, k)
    # the same automata through Eppstein's heuristic and the chained bound
    from oracle import bounds as Bd
    say("fuzz eppstein and bound")
    ge = srw.eppstein_batch(cases)
    gb = srw.bound_batch(cases)
    for (n, k, d), e, b, w in zip(cases, ge, gb, want):
        if w is None:
            assert e[0] == srw.ENOTSYNC and b[0] == srw.ENOTSYNC, (n, k)
            continue
        ew = O.eppstein(n, k, d)[0]
        assert e == (srw.OK, len(ew), ew), (n, k)
        R, bw, w1, _ = Bd.upper_bound(n, k, d)
        assert b == (srw.OK, R, w1, bw) and R >= w[0], (n, k)


def test_batch_matches_oracle_and_single():
    cases = mixed_cases(60, 1234)
    cases.append((1, 2, [0, 0]))
    cases.append((3, 2, [1, 2, 0, 0, 2, 1]))   # not synchronizing
    say("batch", len(cases))
    res = srw.solve_batch(cases)
    for (n, k, d), (st, r, w) in zip(cases, res):
        if n == 3:
            assert st == srw.ENOTSYNC
            continue
        assert st == srw.OK
        assert (r, w) == oracle_rw(n, k, d)
    # the same automaton alone gives the same answer
    for (n, k, d), (st, r, w) in list(zip(cases, res))[:10]:
        assert srw.solve(n, k, d) == (r, w)


def test_batch_slot_limit_same_results():
    cases = mixed_cases(40, 99)
    want = srw.solve_batch(cases)
    srw.set_option("max_slots", 7)
    try:
        say("batch max_slots 7")
        assert srw.solve_batch(cases) == want
    finally:
        srw.set_option("max_slots", 4096)


def test_server_results_same_alone_and_in_mix():
    cases = mixed_cases(50, 4321)
    alone = [srw.solve(n, k, d) for n, k, d in cases]
    say("server", len(cases))
    got = {}
    with srw.Server(max_slots=16) as s:
        for t, (n, k, d) in enumerate(cases):
            s.submit(n, k, d, t)
            if t % 5 == 0:
                for x in s.poll(0):
                    got[x["tag"]] = x
        for _ in range(600):                 # at most 120 s
            if len(got) == len(cases):
                break
            for x in s.poll(200000):
                got[x["tag"]] = x
        assert len(got) == len(cases) and s.pending() == 0
    for t, (n, k, d) in enumerate(cases):
        x = got[t]
        assert x["status"] == srw.OK
        assert (x["r"], x["word"]) == alone[t]
        assert x["latency_ms"] >= x["queue_ms"] >= 0


def test_server_serving_mix_against_stored_oracle_values():
    """Requests of the serving workload's mix (random n in [64, 400], k in
    2..4, 10% Černý C_8..C_40), submitted in arrival order while earlier
    ones run: every served result equals the oracle's -- the stored oracle
    value for the random requests the oracle finished within its time limit
    (tests/golden/serve5.json), the closed form for the Černý ones.  The
    requests the oracle did not finish are left out (parity unpinned)."""
    path = os.path.join(GOLDEN, "serve5.json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle values for the serving mix")
    with open(path) as f:
        stored = {c["seed"]: c for c in json.load(f)["cases"] if "r" in c}
    reqs = I.serve_mix(120, 400, 4, srw.check_sync)
    pick = []
    for i, m in enumerate(reqs):
        if m["label"] == "cerny":
            pick.append((i, m, (m["n"] - 1) ** 2, I.cerny_word(m["n"])))
        elif m["seed"] in stored:
            c = stored[m["seed"]]
            assert (c["n"], c["k"], c["attempt"]) == (m["n"], m["k"], m["attempt"])
            w = c["word"]
            pick.append((i, m, c["r"], [int(x) for x in w] if isinstance(w, str) else w))
    say("serving mix", len(pick), "of", len(reqs), "requests pinned")
    assert len(pick) >= 40
    got = {}
    with srw.Server() as s:
        for j, (i, m, _, _) in enumerate(pick):
            s.submit(m["n"], m["k"], m["delta"], i)
            if j % 4 == 3:                         # arrivals while earlier requests run
                for x in s.poll(20000):
                    got[x["tag"]] = x
        for _ in range(600):                       # at most 120 s
            if len(got) == len(pick):
                break
            for x in s.poll(200000):
                got[x["tag"]] = x
        assert len(got) == len(pick) and s.pending() == 0
    for i, m, r, w in pick:
        x = got[i]
        assert x["status"] == srw.OK, (i, m["n"], m["k"], x["status"])
        assert (x["r"], x["word"]) == (r, w), (i, m["n"], m["k"])


def test_server_lane_budget_trim_enomem_then_later_requests():
    """A server whose lanes have small budgets (512 MiB in all): requests
    that do not fit their lane end with ENOMEM, blocks freed by finished
    requests go back to the allocator when a later request needs room (the
    lane's stream is drained first), and the lane goes on serving: every
    request that completes equals the oracle, and a small request submitted
    after all the others is served."""
    spec = [(150, 2), (200, 3), (120, 2), (96, 3), (160, 2), (64, 2), (130, 3)]
    cases = [(n, k, rand_sync(n, k, i, base=313)) for i, (n, k) in enumerate(spec)]
    got = {}
    with srw.Server(hbm_budget=512 << 20, max_slots=2) as s:
        for t, (n, k, d) in enumerate(cases):
            say("small-budget server", t, n, k)
            s.submit(n, k, d, t)
            for x in s.poll(0):
                got[x["tag"]] = x
        for _ in range(600):
            if len(got) == len(cases):
                break
            for x in s.poll(200000):
                got[x["tag"]] = x
        assert len(got) == len(cases)
        n, k, d = 48, 2, rand_sync(48, 2, 99, base=313)
        s.submit(n, k, d, 99)
        for _ in range(600):
            xs = s.poll(200000)
            if xs:
                got[99] = xs[0]
                break
    cases.append((n, k, d))
    tags = list(range(len(spec))) + [99]
    statuses = [got[t]["status"] for t in tags]
    say("statuses", statuses)
    assert set(statuses) <= {srw.OK, srw.ENOMEM}
    assert srw.ENOMEM in statuses                  # the budget did bind
    assert statuses[-1] == srw.OK                  # and the lane still serves
    for t, (n, k, d) in zip(tags, cases):
        x = got[t]
        if x["status"] == srw.OK:
            assert (x["r"], x["word"]) == oracle_rw(n, k, d), (n, k)


# ------------------------------------------------------ limits and errors

def test_budget_exhaustion_then_recovery():
    d = rand_sync(200, 3, 1, base=5)
    want = oracle_rw(200, 3, d)
    srw.set_option("budget", 96 << 20)
    try:
        say("tiny budget")
        with pytest.raises(srw.SrwError) as e:
            srw.solve(200, 3, d)
        assert e.value.code == srw.ENOMEM
    finally:
        srw.set_option("budget", 0)
    assert srw.solve(200, 3, d) == want


def test_deadline_then_recovery():
    """A solve still running after its deadline ends with ETIMEOUT, and the
    context keeps working."""
    d = I.cerny(40)
    srw.set_option("deadline_ms", 1)
    try:
        say("deadline")
        with pytest.raises(srw.SrwError) as e:
            srw.solve(40, 2, d)
        assert e.value.code == srw.ETIMEOUT
    finally:
        srw.set_option("deadline_ms", 0)
    assert srw.solve(40, 2, d) == (39 ** 2, I.cerny_word(40))


@pytest.mark.parametrize("rows,groups,order,grid", [(0, 1, 0, 0), (8, 3, 1, 0), (100000, 64, 0, 7),
                                                   (512, 8, 1, 65536)])
def test_meet_tuning_options_keep_results(rows, groups, order, grid):
    cs = [(150, 2, 4), (200, 3, 1), (90, 4, 2)]
    srw.set_option("meet_rows", rows)
    srw.set_option("meet_groups", groups)
    srw.set_option("meet_order", order)
    srw.set_option("meet_grid", grid)
    try:
        for n, k, i in cs:
            d = rand_sync(n, k, i, base=71)
            say("meet tuning", rows, groups, order, grid, n, k)
            assert srw.solve(n, k, d) == oracle_rw(n, k, d)
    finally:
        srw.set_option("meet_rows", 512)
        srw.set_option("meet_groups", 16)
        srw.set_option("meet_order", 1)
        srw.set_option("meet_grid", 0)


def test_word_cap():
    with pytest.raises(srw.SrwError) as e:
        srw.solve(10, 2, I.cerny(10), word_cap=5)
    assert e.value.code == srw.EWORDCAP


def test_r_only():
    assert srw.solve(12, 2, I.cerny(12), want_word=False)[0] == 121


# ------------------------------------------------------ full-size config 2

def golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    with open(path) as f:
        return json.load(f)["cases"]


def test_random_n256_against_stored_oracle_values():
    """n=256, k=2, four 64-bit words per subset: r and word of every seed
    equal the oracle's stored values (tests/golden/make_golden.py)."""
    for c in golden("rand256.json"):
        n, k = c["n"], c["k"]
        d = I.random_automaton(n, k, c["seed"], c["attempt"])
        say("n256 seed", c["seed"])
        r, w = srw.solve(n, k, d)
        assert r == c["r"]
        assert "".join(map(str, w)) == c["word"]


@pytest.mark.parametrize("bucket,xcd", [(16384, 0), (0, 0), (16384, 64)])
def test_random_n450_against_stored_oracle_value(bucket, xcd):
    """The n = 450, k = 2 automaton of the benchmark: 8-word sets, levels of
    millions of sets, hash tables grown far past 10^7 slots, the chunked meet
    at full size with its inverse levels in buckets (default) and in level
    order (0), and with per-XCD work queues.  r and word equal the oracle's
    stored values (tests/golden/n450.json; about 40 minutes of oracle
    time)."""
    path = os.path.join(GOLDEN, "n450.json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle value for n = 450")
    with open(path) as f:
        c = json.load(f)["cases"][0]
    d = I.random_automaton(c["n"], c["k"], c["seed"], c["attempt"])
    assert I.first_synchronizing(450, 2, c["seed"], srw.check_sync)[1] == c["attempt"]
    srw.set_option("bucket", bucket)
    srw.set_option("meet_xcd", xcd)
    try:
        say("n450 bucket", bucket, "xcd", xcd)
        assert srw.solve(450, 2, d) == (c["r"], [int(x) for x in c["word"]])
    finally:
        srw.set_option("bucket", 16384)
        srw.set_option("meet_xcd", 0)


def test_random_n256_lds_tile_meet_equals_stored():
    cs = golden("rand256.json")[:2]
    srw.set_option("meet", 1)
    try:
        for c in cs:
            d = I.random_automaton(c["n"], c["k"], c["seed"], c["attempt"])
            say("n256 lds-tile meet seed", c["seed"])
            r, w = srw.solve(c["n"], c["k"], d)
            assert r == c["r"] and "".join(map(str, w)) == c["word"]
    finally:
        srw.set_option("meet", 0)


def test_random_n256_batched_equals_stored():
    cs = golden("rand256.json")
    probs = [(c["n"], c["k"], I.random_automaton(c["n"], c["k"], c["seed"], c["attempt"]))
             for c in cs]
    say("n256 batched")
    res = srw.solve_batch(probs)
    for c, (st, r, w) in zip(cs, res):
        assert st == srw.OK and r == c["r"] and "".join(map(str, w)) == c["word"]


def test_profile_counters_per_width():
    """With profiling on, the per-width meet counters add up to the totals
    and the meet reports the set operations it performed."""
    probs = [(150, 2, rand_sync(150, 2, 0, base=73)), (60, 3, rand_sync(60, 3, 1, base=73))]
    srw.reset_stats()
    srw.set_option("profile", 1)
    srw.set_option("small_cand", 0)        # every meet as its own launch
    try:
        say("profile counters")
        res = srw.solve_batch(probs)
    finally:
        srw.set_option("profile", 0)
        srw.set_option("small_cand", 2048)
    assert all(st == srw.OK for st, _, _ in res)
    st = srw.get_stats()
    mw = st["meet_w"]
    assert set(mw) == {1, 3}                       # n=60 -> W=1, n=150 -> W=3
    assert sum(m["pair_words"] for m in mw.values()) == st["pair_words"]
    for m in mw.values():
        assert m["launches"] > 0 and m["ms"] > 0 and m["ops"] > 0


@pytest.mark.parametrize("small", [0, 1 << 20])
def test_one_block_steps_keep_results(small):
    """Whole steps in one block (small segments) and the per-phase kernels
    give the same r and word; 1 << 20 sends every step with an LDS-tile meet
    of at most 64 blocks through the one-block path."""
    cs = [(n, 2, I.cerny(n)) for n in (2, 3, 7, 16, 25)]
    cs += [(n, k, rand_sync(n, k, i, base=79)) for i, (n, k) in
           enumerate([(40, 2), (64, 3), (100, 2), (150, 2), (200, 3)])]
    srw.set_option("small_cand", small)
    try:
        for n, k, d in cs:
            say("one-block steps", small, n, k)
            assert srw.solve(n, k, d) == oracle_rw(n, k, d)
        res = srw.solve_batch(cs)
        for (n, k, d), (st, r, w) in zip(cs, res):
            assert st == srw.OK and (r, w) == oracle_rw(n, k, d)
    finally:
        srw.set_option("small_cand", 2048)


@pytest.mark.parametrize("persist,small", [(0, 2048), (1, 2048), (1, 64), (1, 1 << 20)])
def test_persistent_small_steps_keep_results(persist, small):
    """The small steps of every automaton run in one launch, a block per
    automaton stepping it until it meets or until a step is too large, after
    which the host goes on from the state the block left.  On and off, with
    the limit moved so that the hand-over comes early (64), at the default
    (2048) or as late as the block's buffers allow (1 << 20): the same r and
    word as the oracle, singly and batched, and the same levels."""
    cs = [(n, 2, I.cerny(n)) for n in (2, 3, 9, 24, 33)]
    cs += [(n, k, rand_sync(n, k, i, base=97)) for i, (n, k) in
           enumerate([(20, 2), (64, 2), (65, 3), (128, 2), (190, 3), (257, 2)])]
    want = [oracle_rw(n, k, d) for n, k, d in cs]
    srw.set_option("persist", persist)
    srw.set_option("small_cand", small)
    try:
        for (n, k, d), w in zip(cs, want):
            say("persist", persist, small, n, k)
            assert srw.solve(n, k, d) == w
        res = srw.solve_batch(cs)
        assert [(st, (r, wd)) for st, r, wd in res] == [(srw.OK, w) for w in want]
        n, k, d = cs[7]                    # random n = 128: levels after the hand-over too
        srw.set_option("keep_levels", 1)
        srw.solve(n, k, d)
        _, _, info = O.bidir(n, k, d, keep_levels=True)
        for side in (0, 1):
            got = srw.last_levels(side, (n + 63) // 64)
            exp = info["levels"][side]
            assert len(got) == len(exp)
            for L, ((gr, gp), (er, ep)) in enumerate(zip(got, exp)):
                assert np.array_equal(gr, er), (side, L)
                if L > 0:
                    assert np.array_equal(gp.astype(np.int64), ep), (side, L)
    finally:
        srw.set_option("keep_levels", 0)
        srw.set_option("persist", 1)
        srw.set_option("small_cand", 2048)


@pytest.mark.parametrize("bucket,meet,xcd,bgrid", [(0, 0, 0, 4096), (1, 2, 0, 4096), (64, 0, 0, 4096),
                                                    (1, 0, 0, 4096), (1, 2, 1, 4096), (1, 2, 64, 4096),
                                                    (64, 0, 7, 4096), (1, 2, 0, 1), (1, 2, 8, 7)])
def test_bucketed_meet_keeps_results(bucket, meet, xcd, bgrid):
    """Inverse levels in buckets by their membership of the forward level's
    most frequent states, met by chunks that scan only the buckets holding
    their common split states: off (0), for every level against every
    forward level sorted into chunks (1 with meet mode 2, so tiny and
    one-bucket levels too), from 64 sets on, and for every level the default
    schedule sorts; work items from one queue or dealt to per-XCD queues in
    runs of 1, 7 or 64; a launch of 4096, 7 or a single block taking the
    items.  r and word equal the oracle's, singly and batched."""
    cs = [(n, 2, I.cerny(n)) for n in (9, 20)]
    cs += [(n, k, rand_sync(n, k, j, base=61)) for j, (n, k) in
           enumerate([(64, 2), (150, 2), (200, 3), (129, 2), (40, 4), (255, 2), (90, 3)])]
    cs += [(200, 2, d) for d in (many_common_states(200, s) for s in range(4))
           if O.is_synchronizing(200, 2, d)][:2]
    want = [oracle_rw(n, k, d) for n, k, d in cs]
    srw.set_option("bucket", bucket)
    srw.set_option("meet", meet)
    srw.set_option("meet_xcd", xcd)
    srw.set_option("meet_bgrid", bgrid)
    try:
        for (n, k, d), w in zip(cs, want):
            say("bucketed meet", bucket, meet, xcd, bgrid, n, k)
            assert srw.solve(n, k, d) == w, (n, k)
        res = srw.solve_batch(cs)
        assert [(st, (r, wd)) for st, r, wd in res] == [(srw.OK, w) for w in want]
    finally:
        srw.set_option("bucket", 16384)
        srw.set_option("meet", 0)
        srw.set_option("meet_xcd", 0)
        srw.set_option("meet_bgrid", 4096)


@pytest.mark.parametrize("ysort", [0, 1])
def test_cardinality_order_keeps_results(ysort):
    """Inverse levels in order of decreasing cardinality (every level with
    ysort 1) and in level order give the least index pair alike, in both meet
    modes and batched; n=256 against the stored oracle values."""
    cs = [(n, k, rand_sync(n, k, i, base=83)) for i, (n, k) in
          enumerate([(70, 2), (130, 2), (100, 3), (160, 2)])]
    want = [oracle_rw(n, k, d) for n, k, d in cs]
    g = golden("rand256.json")[:3]
    cs += [(c["n"], c["k"], I.random_automaton(c["n"], c["k"], c["seed"], c["attempt"])) for c in g]
    want += [(c["r"], [int(ch) for ch in c["word"]]) for c in g]
    srw.set_option("ysort", ysort)
    try:
        for meet in (0, 1, 2):
            srw.set_option("meet", meet)
            for (n, k, d), ww in zip(cs, want):
                say("cardinality order", ysort, "meet", meet, n, k)
                r, w = srw.solve(n, k, d)
                assert (r, list(w)) == (ww[0], list(ww[1]))
        srw.set_option("meet", 0)
        res = srw.solve_batch(cs)
        for (st, r, w), ww in zip(res, want):
            assert st == srw.OK and (r, list(w)) == (ww[0], list(ww[1]))
    finally:
        srw.set_option("meet", 0)
        srw.set_option("ysort", 0)


def test_edge_shapes():
    """One letter (a path into a fixed point: r = n - 1), 255 letters,
    an empty batch and a batch that repeats one automaton."""
    for n in (2, 5, 64, 65, 200):
        d = np.array([max(q - 1, 0) for q in range(n)], np.int32)   # q -> q-1, 0 fixed
        say("one letter path", n)
        assert srw.solve(n, 1, d) == (n - 1, [0] * (n - 1))
    rng = np.random.default_rng(5)
    for n in (3, 6, 9):                    # 255-way branching: small n keeps the oracle quick
        d = rng.integers(0, n, size=255 * n).astype(np.int32)
        if not srw.check_sync(n, 255, d):
            continue
        say("255 letters", n)
        assert srw.solve(n, 255, d) == O.bidir(n, 255, d)[:2]
    assert srw.solve_batch([]) == []
    d = rand_sync(90, 2, 0, base=89)
    res = srw.solve_batch([(90, 2, d)] * 5)
    want = O.bidir(90, 2, d)[:2]
    assert all(st == srw.OK and (r, w) == want for st, r, w in res)


def test_mixed_batch_members_against_stored_oracle_values():
    """The members with n <= 160 among the first 300 of the seeded
    4096-member batch (n uniform in [32, 320], k in {2, 3}), solved together
    in one batch: r and word equal the oracle's stored values."""
    cs = golden("mix4096.json")
    probs = [(c["n"], c["k"], I.random_automaton(c["n"], c["k"], c["seed"], c["attempt"]))
             for c in cs]
    say("mix4096 members", len(probs))
    res = srw.solve_batch(probs)
    for c, (st, r, w) in zip(cs, res):
        assert st == srw.OK and r == c["r"], (c["n"], c["k"], c["seed"])
        assert "".join(map(str, w)) == c["word"], (c["n"], c["k"], c["seed"])


@pytest.mark.parametrize("k", [2, 3])
def test_mixed_batch_larger_members_against_stored_oracle_values(k):
    """The members with n > 160 among the first 300 of the seeded 4096-member
    batch that the oracle finished within its time budget (tests/golden/
    mix4096big.json records the budget of the others), solved together in
    one batch per alphabet size: r and word equal the oracle's stored
    values.  The others are parity unpinned."""
    path = os.path.join(GOLDEN, "mix4096big.json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle values for the larger members")
    cs = [c for c in golden("mix4096big.json") if "r" in c and c["k"] == k]
    probs = [(c["n"], c["k"], I.random_automaton(c["n"], c["k"], c["seed"], c["attempt"]))
             for c in cs]
    say("mix4096 larger members, k =", k, len(probs))
    res = srw.solve_batch(probs)
    for c, (st, r, w) in zip(cs, res):
        assert st == srw.OK and r == c["r"], (c["n"], c["k"], c["seed"])
        assert "".join(map(str, w)) == c["word"], (c["n"], c["k"], c["seed"])


def test_server_deadline_then_recovery():
    """A server with a 1 ms per-request deadline ends two Černý C_40 solves
    (1,521 steps each) with ETIMEOUT and returns both; a server without a
    deadline then solves them exactly."""
    d = I.cerny(40)
    say("server deadline")
    got = {}
    with srw.Server(max_slots=4, deadline_ms=1) as s:
        s.submit(40, 2, d, 0)
        s.submit(40, 2, d, 1)
        for _ in range(300):                 # at most 60 s
            for x in s.poll(200000):
                got[x["tag"]] = x
            if len(got) == 2:
                break
        assert len(got) == 2 and s.pending() == 0
    assert [got[t]["status"] for t in (0, 1)] == [srw.ETIMEOUT] * 2
    got = {}
    with srw.Server(max_slots=4) as s:
        s.submit(40, 2, d, 7)
        for _ in range(300):
            for x in s.poll(200000):
                got[x["tag"]] = x
            if got:
                break
    assert got[7]["status"] == srw.OK
    assert (got[7]["r"], got[7]["word"]) == (39 ** 2, I.cerny_word(40))


# ------------------------------------------------------ beam search (upper bound)

def beam_cases():
    cs = []
    for i, (n, k) in enumerate([(8, 2), (20, 2), (33, 3), (64, 2), (65, 3), (100, 2), (130, 2),
                                (200, 3), (300, 2), (450, 2)]):
        d, _ = I.first_synchronizing(n, k, I.member_seed(I.BASE_SEED ^ 0xBEA, i), O.is_synchronizing)
        cs.append((n, k, d))
    return cs


def test_beam_matches_the_oracle():
    """srw_beam_batch against the oracle's beam search (orc_beam): the same
    R and word, or both ending at an empty level, over widths from 1 to
    n log n, set widths 1..8, in one batch."""
    import math
    probs, want = [], []
    for n, k, d in beam_cases():
        for width in sorted({1, 4, 16, 64, int(n * math.log(n)) + 1}):
            R, w, _ = O.beam(n, k, d, width)
            probs.append((n, k, d, width))
            want.append((srw.OK, R, list(w)) if R is not None else (srw.ENOBOUND, -1, None))
    say("beam batch", len(probs))
    got = srw.beam_batch(probs)
    for p, g, w in zip(probs, got, want):
        assert g == w, (p[0], p[1], p[3])


def test_unbounded_beam_is_exact():
    """A width above every level size makes the beam search the plain
    inverse search: R = r and the word srw_solve returns (and the oracle)."""
    for n, k, d in beam_cases()[:6] + [(n, 2, I.cerny(n)) for n in (5, 17, 40)]:
        say("beam exact", n, k)
        want = oracle_rw(n, k, d)
        assert srw.beam(n, k, d, 1 << 40) == want, (n, k)


def test_beam_edges():
    st = srw.beam_batch([(1, 2, np.zeros(2, np.int32), 3), (4, 2, np.array([0, 1, 2, 3, 0, 1, 2, 3], np.int32), 8),
                         (3, 1, np.array([1, 2, 0], np.int32), 2), (9, 2, I.cerny(9), 0)])
    assert st[0] == (srw.OK, 0, [])
    assert st[1][0] == srw.ENOTSYNC and st[2][0] == srw.ENOTSYNC
    assert st[3][0] == srw.EINVAL
    assert srw.beam_batch([]) == []


# ------------------------------------------------------ Eppstein's heuristic

def eppstein_cases():
    cs = []
    for i, (n, k) in enumerate([(2, 1), (2, 3), (3, 2), (5, 2), (8, 4), (16, 2), (33, 3), (64, 2),
                                (65, 5), (100, 2), (200, 3), (300, 2), (450, 2), (512, 2), (512, 40),
                                (40, 255)]):
        d, _ = I.first_synchronizing(n, k, I.member_seed(I.BASE_SEED ^ 0xE99, i), O.is_synchronizing)
        cs.append((n, k, d))
    # Černý automata: pair distances up to n(n-1)/2, rounds longer than the
    # kernel's letter chunk from n = 72 on
    cs += [(n, 2, I.cerny(n)) for n in (2, 3, 7, 20, 80)]
    return cs


def test_eppstein_matches_the_oracle():
    """srw_eppstein_batch against the oracle's Eppstein heuristic
    (orc_eppstein): the same word, letter for letter, over n = 2 .. 512,
    k = 1 .. 255 (transition tables in LDS and in global memory), and Černý
    automata with rounds of up to 3,160 letters; in one batch and singly."""
    cs = eppstein_cases()
    want = [O.eppstein(n, k, d)[0] for n, k, d in cs]
    say("eppstein batch", len(cs))
    got = srw.eppstein_batch(cs)
    for (n, k, _), g, w in zip(cs, got, want):
        assert g == (srw.OK, len(w), w), (n, k)
    for (n, k, d), w in list(zip(cs, want))[-4:]:
        say("eppstein single", n, k)
        assert srw.eppstein(n, k, d) == w


def test_eppstein_edges():
    """n = 1, non-synchronizing automata, bad input, a word longer than its
    buffer (SRW_EWORDCAP with the length), an empty batch."""
    st = srw.eppstein_batch([(1, 2, np.zeros(2, np.int32)), (4, 2, np.array([0, 1, 2, 3, 0, 1, 2, 3], np.int32)),
                             (3, 1, np.array([1, 2, 0], np.int32)), (3, 1, np.array([1, 2, 7], np.int32))])
    assert st[0] == (srw.OK, 0, [])
    assert st[1][0] == srw.ENOTSYNC and st[2][0] == srw.ENOTSYNC
    assert st[3][0] == srw.EINVAL
    assert srw.eppstein_batch([]) == []
    w = O.eppstein(20, 2, I.cerny(20))[0]
    st = srw.eppstein_batch([(20, 2, I.cerny(20))], word_cap=100)
    assert st[0][0] == srw.EWORDCAP and st[0][1] == len(w) > 100


def test_eppstein_and_bound_deadlines():
    """Option deadline_ms ends a long Eppstein search (Černý C_512: about
    1.3e5 levels of the search over pairs) with SRW_ETIMEOUT, on the device,
    without touching the other automata of the batch; srw_bound passes the
    status on and runs no beam for it.  Without the deadline the same batch
    is solved (every word checked on the host)."""
    big = (512, 2, I.cerny(512))
    d, _ = I.first_synchronizing(40, 2, I.member_seed(I.BASE_SEED ^ 0xDEAD, 0), O.is_synchronizing)
    small = (40, 2, d)
    want = O.eppstein(40, 2, d)[0]
    try:
        srw.set_option("deadline_ms", 2)
        say("eppstein deadline")
        got = srw.eppstein_batch([big, small])
        assert got[0][0] == srw.ETIMEOUT
        assert got[1][0] in (srw.OK, srw.ETIMEOUT)
        if got[1][0] == srw.OK:
            assert got[1][2] == want
        say("bound deadline")
        assert srw.bound_batch([big])[0][0] == srw.ETIMEOUT
    finally:
        srw.set_option("deadline_ms", 0)
    say("eppstein no deadline")
    got = srw.eppstein_batch([big, small], word_cap=1 << 26)
    assert got[0][0] == srw.OK and got[0][1] >= 511 ** 2
    assert got[1] == (srw.OK, len(want), want)


def test_bound_matches_the_oracle():
    """srw_bound_batch (Eppstein, the beam of width n, the beam of the
    adaptive width) against the oracle's composition of the same three
    (oracle/bounds.py): the same R, width and word; the n = 450 automaton
    of the default workload reaches its exact r = 50 with width 18,106."""
    from oracle import bounds as Bd
    cs = []
    for i, (n, k) in enumerate([(20, 2), (64, 2), (100, 3), (150, 2), (200, 2), (256, 2), (300, 2),
                                (120, 4)]):
        d, _ = I.first_synchronizing(n, k, I.member_seed(I.BASE_SEED ^ 0xB0, i), O.is_synchronizing)
        cs.append((n, k, d))
    d450, _ = I.first_synchronizing(450, 2, I.member_seed(I.BASE_SEED, 0), O.is_synchronizing)
    cs += [(450, 2, d450), (9, 2, I.cerny(9)), (1, 2, np.zeros(2, np.int32))]
    want = []
    for n, k, d in cs:
        R, w, w1, _ = Bd.upper_bound(n, k, d)
        want.append((srw.OK, R, w1, w))
    say("bound batch", len(cs))
    got = srw.bound_batch(cs)
    for (n, k, _), g, w in zip(cs, got, want):
        assert g == w, (n, k)
    assert got[8][1:3] == (50, 18106)
    # non-synchronizing automata: found by Eppstein's search over pairs
    bad = [(4, 2, np.array([1, 2, 3, 0, 0, 2, 1, 3], np.int32)), (3, 2, np.array([1, 2, 0, 0, 2, 1], np.int32)),
           (6, 2, np.array([1, 0, 3, 2, 5, 4, 2, 3, 4, 5, 0, 1], np.int32)),
           (4, 2, np.array([0, 0, 2, 2, 2, 3, 0, 1], np.int32))]     # merges, then a stuck pair
    assert [g[0] for g in srw.bound_batch(bad)] == [srw.ENOTSYNC] * 4
    assert [g[0] for g in srw.eppstein_batch(bad)] == [srw.ENOTSYNC] * 4
    assert not any(O.is_synchronizing(n, k, d) for n, k, d in bad)


# ------------------------------------------------------ self-reduction on the device

def reduce_cases():
    cs = []
    for i, (n, k) in enumerate([(12, 2), (20, 2), (33, 3), (48, 2), (64, 2), (90, 3), (128, 2), (160, 2)]):
        d, _ = I.first_synchronizing(n, k, I.member_seed(I.BASE_SEED ^ 0x5ED, i), O.is_synchronizing)
        cs.append((n, k, d))
    cs += [(n, 2, I.cerny(n)) for n in (6, 13)]
    return cs


@pytest.mark.parametrize("mode", [1, 2])
def test_self_reduction_matches_the_oracle(mode):
    """Option reduce: every new level self-reduced on the device (Alg. 1),
    with mode 2 also reduced by the side's earlier levels; dropped sets kept
    visited.  r and word equal the oracle's search with the same reduction
    (oracle.bidir(reduce=True or "history", keep_dropped=True)), r equals
    the unreduced r, and every level (sets, order, parent keys) equals the
    oracle's; singly and in one batch."""
    cs = reduce_cases()
    want = []
    for n, k, d in cs:
        r, w, info = O.bidir(n, k, d, reduce=True if mode == 1 else "history", keep_dropped=True,
                             keep_levels=True)
        want.append((r, list(w), info["levels"]))
        assert r == oracle_rw(n, k, d)[0]
    srw.set_option("reduce", mode)
    srw.set_option("keep_levels", 1)
    try:
        for (n, k, d), (r, w, levels) in zip(cs, want):
            say("reduce", n, k)
            assert srw.solve(n, k, d) == (r, w), (n, k)
            for side in (0, 1):
                got = srw.last_levels(side, (n + 63) // 64)
                assert len(got) == len(levels[side]), (n, k, side)
                for L, ((gr, gp), (er, ep)) in enumerate(zip(got, levels[side])):
                    assert np.array_equal(gr, er), (n, k, side, L)
                    if L > 0:
                        assert np.array_equal(gp.astype(np.int64), ep), (n, k, side, L)
        srw.set_option("keep_levels", 0)
        res = srw.solve_batch(cs)
        assert [(st, (r, wd)) for st, r, wd in res] == [(srw.OK, (r, w)) for r, w, _ in want]
        assert srw.get_stats()["reduced"] > 0
    finally:
        srw.set_option("reduce", 0)
        srw.set_option("keep_levels", 0)
