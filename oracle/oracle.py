"""ctypes wrapper of the C oracle (srw_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module; the library itself
never does.  See srw_oracle.c for what each function computes and the passage
of the paper it follows.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "srw_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, EINVAL, ENOTSYNC, ELIMIT, ENOMEM, EWORDCAP = 0, -1, -2, -3, -4, -5

MEET_BRUTE = 0      # all pairs in (i, j) order: the definition
MEET_MARK = 1       # Alg. 2 MarkSupersets, then the least marked pair


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, single-threaded)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = bind(LIB)
    return _lib


def bind(path):
    """Load a compiled oracle (the real one, or a planted-mistake copy that
    the mutation tests build) and declare its signatures."""
    if True:
        L = ctypes.CDLL(path)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.orc_is_synchronizing.argtypes = [ctypes.c_int, ctypes.c_int, i32p]
        L.orc_verify.argtypes = [ctypes.c_int, ctypes.c_int, i32p, u8p, ctypes.c_int64]
        L.orc_image.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int, u64p, u64p]
        L.orc_image.restype = None
        L.orc_preimage.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int, u64p, u64p]
        L.orc_preimage.restype = None
        L.orc_bruteforce.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int,
                                     i32p, u8p, ctypes.c_int64]
        L.orc_exhaustive.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, u8p,
                                     ctypes.c_int64]
        L.orc_forward.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int64,
                                  i32p, u8p, ctypes.c_int64]
        L.orc_bidir.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int,
                                u8p, ctypes.c_int, ctypes.c_int,
                                i32p, u8p, ctypes.c_int64, u8p, i64p,
                                ctypes.POINTER(ctypes.c_void_p)]
        L.orc_bidir_reduced.argtypes = L.orc_bidir.argtypes
        L.orc_bidir_history.argtypes = L.orc_bidir.argtypes
        L.orc_bidir_reduce.argtypes = L.orc_bidir.argtypes + [ctypes.c_int]
        L.orc_beam.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int64, ctypes.c_int,
                               i32p, u8p, ctypes.c_int64, i64p]
        L.orc_beam_sizes.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int64, ctypes.c_int,
                                     i32p, u8p, ctypes.c_int64, i64p, ctypes.c_int, i32p]
        L.orc_pair_dist.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, u8p]
        L.orc_eppstein.argtypes = [ctypes.c_int, ctypes.c_int, i32p, u8p, ctypes.c_int64,
                                   i64p, i32p, i32p]
        L.orc_levels.argtypes = [ctypes.c_void_p, ctypes.c_int, i32p, i64p, i64p,
                                 u64p, i64p]
        L.orc_free.argtypes = [ctypes.c_void_p]
        L.orc_free.restype = None
    return L


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _delta(delta):
    return np.ascontiguousarray(np.asarray(delta, dtype=np.int32))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def is_synchronizing(n, k, delta) -> bool:
    d = _delta(delta)
    rc = lib().orc_is_synchronizing(n, k, _ptr(d, ctypes.c_int32))
    if rc < 0:
        raise OracleError(rc, "is_synchronizing")
    return bool(rc)


def verify(n, k, delta, word) -> bool:
    d = _delta(delta)
    w = np.ascontiguousarray(np.asarray(word, dtype=np.uint8))
    rc = lib().orc_verify(n, k, _ptr(d, ctypes.c_int32), _ptr(w, ctypes.c_uint8), len(w))
    if rc < 0:
        raise OracleError(rc, "verify")
    return bool(rc)


def _words(n):
    return (n + 63) // 64


def image(n, k, delta, a, S):
    d = _delta(delta)
    s = np.ascontiguousarray(np.asarray(S, dtype=np.uint64))
    out = np.zeros(_words(n), dtype=np.uint64)
    lib().orc_image(n, k, _ptr(d, ctypes.c_int32), a, _ptr(s, ctypes.c_uint64),
                    _ptr(out, ctypes.c_uint64))
    return out


def preimage(n, k, delta, a, S):
    d = _delta(delta)
    s = np.ascontiguousarray(np.asarray(S, dtype=np.uint64))
    out = np.zeros(_words(n), dtype=np.uint64)
    lib().orc_preimage(n, k, _ptr(d, ctypes.c_int32), a, _ptr(s, ctypes.c_uint64),
                       _ptr(out, ctypes.c_uint64))
    return out


def _result(rc, what, r, word):
    if rc != OK:
        raise OracleError(rc, what)
    return int(r.value), [int(x) for x in word[: r.value]]


def bruteforce(n, k, delta, max_len=24):
    d = _delta(delta)
    r = ctypes.c_int32(-1)
    word = np.zeros(max(max_len, 1), dtype=np.uint8)
    rc = lib().orc_bruteforce(n, k, _ptr(d, ctypes.c_int32), max_len, ctypes.byref(r),
                              _ptr(word, ctypes.c_uint8), len(word))
    return _result(rc, "bruteforce", r, word)


def exhaustive(n, k, delta):
    d = _delta(delta)
    r = ctypes.c_int32(-1)
    word = np.zeros(1 << 16, dtype=np.uint8)
    rc = lib().orc_exhaustive(n, k, _ptr(d, ctypes.c_int32), ctypes.byref(r),
                              _ptr(word, ctypes.c_uint8), len(word))
    return _result(rc, "exhaustive", r, word)


def forward(n, k, delta, max_sets=5_000_000):
    d = _delta(delta)
    r = ctypes.c_int32(-1)
    word = np.zeros(1 << 16, dtype=np.uint8)
    rc = lib().orc_forward(n, k, _ptr(d, ctypes.c_int32), max_sets, ctypes.byref(r),
                           _ptr(word, ctypes.c_uint8), len(word))
    return _result(rc, "forward", r, word)


STAT_NAMES = ("steps", "f", "b", "visited_f", "visited_b", "candidates",
              "pair_tests", "pairs", "reduce_tests")


def bidir(n, k, delta, meet=MEET_MARK, sched=None, max_steps=1 << 20,
          keep_levels=False, reduce=False, alg2=False, keep_dropped=False):
    """Plain bidirectional BFS.  Returns (r, word, info) where info holds the
    sides chosen per step, run statistics and (optionally) all levels.  With
    reduce, every new level is self-reduced before the meet test; with
    reduce="history", also reduced by the sets of the side's earlier levels.
    With alg2, the reductions find their drops with Alg. 2 (the same drops);
    with keep_dropped, dropped sets stay in the visited index."""
    d = _delta(delta)
    r = ctypes.c_int32(-1)
    cap = 1 << 20
    word = np.zeros(cap, dtype=np.uint8)
    sides = np.zeros(min(max_steps, cap) + 1, dtype=np.uint8)
    stats = np.zeros(len(STAT_NAMES), dtype=np.int64)
    if sched is not None:
        s = np.ascontiguousarray(np.asarray(sched, dtype=np.uint8))
        sp, sl = _ptr(s, ctypes.c_uint8), len(s)
    else:
        sp, sl = None, 0
    h = ctypes.c_void_p(None)
    args = (n, k, _ptr(d, ctypes.c_int32), meet, sp, sl, min(max_steps, cap), ctypes.byref(r),
            _ptr(word, ctypes.c_uint8), cap, _ptr(sides, ctypes.c_uint8),
            _ptr(stats, ctypes.c_int64), ctypes.byref(h) if keep_levels else None)
    if alg2 or keep_dropped:
        if not reduce:
            raise ValueError("alg2 and keep_dropped change how reductions are done: "
                             "reduce must be set")
        flags = 1 | (2 if reduce == "history" else 0) | (4 if alg2 else 0) | (8 if keep_dropped else 0)
        rc = lib().orc_bidir_reduce(*args, flags)
    elif reduce == "history":
        rc = lib().orc_bidir_history(*args)
    elif reduce:
        rc = lib().orc_bidir_reduced(*args)
    else:
        rc = lib().orc_bidir(*args)
    rr, ww = _result(rc, "bidir", r, word)
    info = dict(zip(STAT_NAMES, (int(x) for x in stats)))
    info["sides"] = [int(x) for x in sides[: info["steps"]]]
    if keep_levels:
        try:
            info["levels"] = [_levels(h, side, _words(n)) for side in (0, 1)]
        finally:
            lib().orc_free(h)
    return rr, ww, info


def bidir_steps(n, k, delta, max_steps, meet=MEET_MARK):
    """The plain bidirectional search stopped after at most `max_steps`
    expansion steps (or at the meet, whichever comes first).  Returns
    (done, info): done is True when the searches met; info holds the run
    statistics of the steps taken (the benchmark's bounded CPU sample)."""
    d = _delta(delta)
    r = ctypes.c_int32(-1)
    stats = np.zeros(len(STAT_NAMES), dtype=np.int64)
    rc = lib().orc_bidir(n, k, _ptr(d, ctypes.c_int32), meet, None, 0, max_steps,
                         ctypes.byref(r), None, 0, None, _ptr(stats, ctypes.c_int64), None)
    if rc not in (OK, ELIMIT):
        raise OracleError(rc, "bidir_steps")
    return rc == OK, dict(zip(STAT_NAMES, (int(x) for x in stats)))


BEAM_STATS = ("steps", "kept", "cut", "widest")


def beam(n, k, delta, width, max_steps=1 << 20):
    """Beam search upper bound (orc_beam): returns (R, word, info), or
    (None, None, info) when the cut led into a dead end."""
    d = _delta(delta)
    R = ctypes.c_int32(-1)
    cap = 1 << 20
    word = np.zeros(cap, dtype=np.uint8)
    stats = np.zeros(len(BEAM_STATS), dtype=np.int64)
    rc = lib().orc_beam(n, k, _ptr(d, ctypes.c_int32), int(width), int(max_steps), ctypes.byref(R),
                        _ptr(word, ctypes.c_uint8), cap, _ptr(stats, ctypes.c_int64))
    info = dict(zip(BEAM_STATS, (int(x) for x in stats)))
    if rc == ELIMIT:
        return None, None, info
    rr, ww = _result(rc, "beam", R, word)
    return rr, ww, info


def pair_dist(n, k, delta):
    """Shortest merging word length of every pair (orc_pair_dist): returns
    (dist, next), two n x n arrays; dist -1 where no word merges the pair,
    next the least letter starting a shortest merging word (255 where
    dist <= 0)."""
    d = _delta(delta)
    dist = np.zeros((n, n), dtype=np.int32)
    nxt = np.zeros((n, n), dtype=np.uint8)
    rc = lib().orc_pair_dist(n, k, _ptr(d, ctypes.c_int32), _ptr(dist, ctypes.c_int32),
                             _ptr(nxt, ctypes.c_uint8))
    if rc != OK:
        raise OracleError(rc, "pair_dist")
    return dist, nxt


def eppstein(n, k, delta, cap=1 << 22):
    """Eppstein's greedy heuristic (orc_eppstein): returns (word, rounds),
    rounds a list of (p, q, dist) per round."""
    d = _delta(delta)
    word = np.zeros(max(cap, 1), dtype=np.uint8)
    ln = ctypes.c_int64(-1)
    rounds = np.zeros(3 * max(n, 1), dtype=np.int32)
    nr = ctypes.c_int32(0)
    rc = lib().orc_eppstein(n, k, _ptr(d, ctypes.c_int32), _ptr(word, ctypes.c_uint8), len(word),
                            ctypes.byref(ln), _ptr(rounds, ctypes.c_int32), ctypes.byref(nr))
    if rc != OK:
        raise OracleError(rc, "eppstein")
    rr = [tuple(int(x) for x in rounds[3 * i:3 * i + 3]) for i in range(nr.value)]
    return [int(x) for x in word[:ln.value]], rr


def beam_sizes(n, k, delta, width, max_steps=1 << 20):
    """orc_beam_sizes: (R, word, sizes), sizes[L] the new sets of depth L
    before the cut (sizes[0] = n); R and word None at a dead end."""
    d = _delta(delta)
    R = ctypes.c_int32(-1)
    cap = 1 << 20
    word = np.zeros(cap, dtype=np.uint8)
    sizes = np.zeros(1 << 16, dtype=np.int64)
    ns = ctypes.c_int32(0)
    rc = lib().orc_beam_sizes(n, k, _ptr(d, ctypes.c_int32), int(width), int(max_steps), ctypes.byref(R),
                              _ptr(word, ctypes.c_uint8), cap, _ptr(sizes, ctypes.c_int64), len(sizes),
                              ctypes.byref(ns))
    sz = [int(x) for x in sizes[:ns.value]]
    if rc == ELIMIT:
        return None, None, sz
    rr, ww = _result(rc, "beam_sizes", R, word)
    return rr, ww, sz


def levels_after(n, k, delta, sched):
    """The lists of the plain bidirectional search after the steps `sched`
    (0 forward, 1 inverse), or fewer if the searches meet first.  Returns
    (met, levels): met is True when the meet test succeeded after the steps
    taken; levels[side] is a list of (rows, parent keys) per level."""
    d = _delta(delta)
    r = ctypes.c_int32(-1)
    s = np.ascontiguousarray(np.asarray(list(sched) + [0], dtype=np.uint8))
    stats = np.zeros(len(STAT_NAMES), dtype=np.int64)
    h = ctypes.c_void_p(None)
    rc = lib().orc_bidir(n, k, _ptr(d, ctypes.c_int32), MEET_MARK, _ptr(s, ctypes.c_uint8),
                         len(sched), len(sched), ctypes.byref(r), None, 0, None,
                         _ptr(stats, ctypes.c_int64), ctypes.byref(h))
    if rc not in (OK, ELIMIT):
        raise OracleError(rc, "levels_after")
    try:
        levels = [_levels(h, side, _words(n)) for side in (0, 1)]
    finally:
        lib().orc_free(h)
    return rc == OK, levels


def _levels(h, side, W):
    L = lib()
    nlev = ctypes.c_int32(0)
    nrows = ctypes.c_int64(0)
    rc = L.orc_levels(h, side, ctypes.byref(nlev), ctypes.byref(nrows), None, None, None)
    if rc:
        raise OracleError(rc, "levels")
    off = np.zeros(nlev.value + 1, dtype=np.int64)
    rows = np.zeros(max(nrows.value, 1) * W, dtype=np.uint64)
    par = np.zeros(max(nrows.value, 1), dtype=np.int64)
    rc = L.orc_levels(h, side, ctypes.byref(nlev), ctypes.byref(nrows),
                      _ptr(off, ctypes.c_int64), _ptr(rows, ctypes.c_uint64),
                      _ptr(par, ctypes.c_int64))
    if rc:
        raise OracleError(rc, "levels")
    rows = rows[: nrows.value * W].reshape(nrows.value, W)
    out = []
    for L_ in range(nlev.value):
        a, b = off[L_], off[L_ + 1]
        out.append((rows[a:b].copy(), par[a:b].copy()))
    return out
