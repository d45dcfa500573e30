"""Python binding of libsrw (ctypes over the C ABI in include/srw.h).

Argument marshalling only: every step of the search runs in the library's
HIP kernels.  PyTorch, when asked (``use_torch``), only supplies device memory
(its caching allocator) and the stream.  There is no CPU fallback: if
libsrw.so is missing or no GPU is usable, calls raise.
"""

from __future__ import annotations

import atexit
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsrw.so")

OK = 0
EINVAL, ENOTSYNC, EUNSUPPORTED, ENOMEM, EWORDCAP, EDEVICE, ETIMEOUT, EINTERNAL, ENOBOUND = (
    -1, -2, -3, -4, -5, -6, -7, -8, -9)
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOTSYNC", -3: "EUNSUPPORTED", -4: "ENOMEM",
                -5: "EWORDCAP", -6: "EDEVICE", -7: "ETIMEOUT", -8: "EINTERNAL", -9: "ENOBOUND"}

# every symbol include/srw.h declares
EXPORTS = ("srw_solve", "srw_solve_batch", "srw_solve_noalloc", "srw_beam", "srw_beam_batch",
           "srw_eppstein", "srw_eppstein_batch", "srw_bound", "srw_bound_batch",
           "srw_check_sync", "srw_verify",
           "srw_server_create", "srw_server_submit", "srw_server_poll",
           "srw_server_pending", "srw_server_destroy", "srw_set_allocator",
           "srw_set_stream", "srw_set_option", "srw_get_stats", "srw_reset_stats",
           "srw_last_levels", "srw_last_sides", "srw_last_error")

KERNEL_CLASSES = ("expand", "insert", "compact", "prep", "meet", "trace", "setup", "step")


class SrwError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS_NAMES.get(code, code)} ({code}): {last_error()}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("global_steps", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("unique", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("cand_words", ctypes.c_int64), ("pair_words", ctypes.c_int64),
                ("launches", ctypes.c_int64 * 8), ("ms", ctypes.c_double * 8),
                ("bytes_expand", ctypes.c_int64), ("bytes_insert", ctypes.c_int64),
                ("bytes_compact", ctypes.c_int64), ("peak_device_bytes", ctypes.c_int64),
                ("meet_launches_w", ctypes.c_int64 * 8), ("meet_ms_w", ctypes.c_double * 8),
                ("pair_words_w", ctypes.c_int64 * 8), ("meet_ops_w", ctypes.c_int64 * 8),
                ("host_ms", ctypes.c_double * 4), ("meet_work", ctypes.c_int64 * 8),
                ("meet_b_launches_w", ctypes.c_int64 * 8), ("meet_b_ms_w", ctypes.c_double * 8),
                ("meet_b_ops_w", ctypes.c_int64 * 8), ("reduced", ctypes.c_int64)]

    def as_dict(self):
        arrays = ("launches", "ms", "meet_launches_w", "meet_ms_w", "pair_words_w", "meet_ops_w", "host_ms",
                  "meet_work", "meet_b_launches_w", "meet_b_ms_w", "meet_b_ops_w")
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in arrays}
        d["launches"] = dict(zip(KERNEL_CLASSES, list(self.launches)))
        d["ms"] = dict(zip(KERNEL_CLASSES, list(self.ms)))
        d["host_ms"] = dict(zip(("prepare", "launch", "wait", "results"), list(self.host_ms)))
        d["meet_work"] = dict(zip(("items", "groups", "groups_with_candidates", "candidates",
                                   "signature_passes", "column_tiles", "tiles", "bucketed_launches"),
                                  list(self.meet_work)))
        d["meet_w"] = {w + 1: {"launches": self.meet_launches_w[w], "ms": self.meet_ms_w[w],
                               "pair_words": self.pair_words_w[w], "ops": self.meet_ops_w[w],
                               "b_launches": self.meet_b_launches_w[w], "b_ms": self.meet_b_ms_w[w],
                               "b_ops": self.meet_b_ops_w[w]}
                       for w in range(8) if self.meet_launches_w[w]}
        return d


class Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("deadline_ms", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("r", ctypes.c_int32),
                ("word", ctypes.POINTER(ctypes.c_uint8)), ("latency_ms", ctypes.c_double),
                ("queue_ms", ctypes.c_double), ("est_bytes", ctypes.c_int64),
                ("dev_bytes", ctypes.c_int64)]


_lib = None
_keep = []

i32p = ctypes.POINTER(ctypes.c_int32)
i64p = ctypes.POINTER(ctypes.c_int64)
u8p = ctypes.POINTER(ctypes.c_uint8)
u32p = ctypes.POINTER(ctypes.c_uint32)
u64p = ctypes.POINTER(ctypes.c_uint64)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def load(path: str = LIB_PATH):
    """Load libsrw.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it first (python -c "
                          "'import __graft_entry__ as g; g.build()')")
    # PyTorch-ROCm ships its own HIP runtime.  Importing torch first (this
    # does not initialise the GPU) lets libsrw bind to that runtime instead of
    # loading a second one from /opt/rocm: with two HSA runtimes in a process
    # the one initialised second finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    L.srw_solve.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, u8p, ctypes.c_int64]
    L.srw_solve_noalloc.argtypes = L.srw_solve.argtypes
    L.srw_solve_batch.argtypes = [ctypes.c_int32, i32p, i32p, i64p, i32p, i32p, i32p,
                                  i64p, u8p, i64p]
    L.srw_beam.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, ctypes.c_int64, i32p, u8p,
                           ctypes.c_int64]
    L.srw_bound.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, i64p, u8p, ctypes.c_int64]
    L.srw_bound_batch.argtypes = [ctypes.c_int32, i32p, i32p, i64p, i32p, i32p, i64p, i32p,
                                  i64p, u8p, i64p]
    L.srw_eppstein.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i64p, u8p, ctypes.c_int64]
    L.srw_eppstein_batch.argtypes = [ctypes.c_int32, i32p, i32p, i64p, i32p, i64p, i32p,
                                     i64p, u8p, i64p]
    L.srw_beam_batch.argtypes = [ctypes.c_int32, i32p, i32p, i64p, i32p, i64p, i32p, i32p,
                                 i64p, u8p, i64p]
    L.srw_check_sync.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p]
    L.srw_verify.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, u8p, ctypes.c_int64]
    L.srw_server_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Config)]
    L.srw_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, i32p,
                                    ctypes.c_uint64]
    L.srw_server_poll.argtypes = [ctypes.c_void_p, ctypes.POINTER(Result), ctypes.c_int32,
                                  ctypes.c_int32]
    L.srw_server_pending.argtypes = [ctypes.c_void_p]
    L.srw_server_pending.restype = ctypes.c_int64
    L.srw_server_destroy.argtypes = [ctypes.c_void_p]
    L.srw_server_destroy.restype = None
    L.srw_set_allocator.argtypes = [ALLOC_FN, FREE_FN, ctypes.c_void_p]
    L.srw_set_stream.argtypes = [ctypes.c_void_p]
    L.srw_set_option.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    L.srw_get_stats.argtypes = [ctypes.POINTER(Stats)]
    L.srw_reset_stats.argtypes = []
    L.srw_last_levels.argtypes = [ctypes.c_int32, i32p, i64p, i64p, u64p, u32p]
    L.srw_last_sides.argtypes = [i32p, u8p, ctypes.c_int64]
    L.srw_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def last_error() -> str:
    if _lib is None:
        return ""
    s = _lib.srw_last_error()
    return s.decode() if s else ""


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _delta(delta):
    return np.ascontiguousarray(np.asarray(delta, dtype=np.int32))


def use_torch(device: int = 0):
    """Take device memory from PyTorch's caching allocator and launch on
    PyTorch's current stream."""
    import torch

    L = load()

    def _alloc(size, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(size), device)
        except Exception:
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a, f = ALLOC_FN(_alloc), FREE_FN(_free)
    # every pair ever registered stays referenced: setting a new allocator
    # frees the default context's memory through the previous pair, and a
    # server created earlier keeps using the pair it was created with
    _keep.extend([a, f])
    rc = L.srw_set_allocator(a, f, None)
    if rc:
        raise SrwError(rc, "set_allocator")
    rc = L.srw_set_stream(ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream))
    if rc:
        raise SrwError(rc, "set_stream")


@atexit.register
def _shutdown():
    # drop the default context while the allocator callbacks still work
    if _lib is not None and _keep:
        _lib.srw_set_allocator(ALLOC_FN(), FREE_FN(), None)


def set_option(key: str, value: int):
    rc = load().srw_set_option(key.encode(), int(value))
    if rc:
        raise SrwError(rc, f"set_option({key})")


TUNING_TABLE = os.path.join(HERE, "tuning.json")


def apply_tuning(path: str = TUNING_TABLE) -> dict:
    """Set the per-width options of the autotuner's table (autotune.py):
    option "<key>@<W>" for every tuned key and width.  Returns the values
    set, {W: {key: value}} ({} when there is no table)."""
    if not os.path.exists(path):
        return {}
    import json
    with open(path) as f:
        rec = json.load(f)
    out = {}
    for w, ent in sorted(rec.get("widths", {}).items()):
        vals = {key: int(v) for key, v in ent["values"].items()}
        for key, v in vals.items():
            set_option(f"{key}@{int(w)}", v)
        out[int(w)] = vals
    return out


def clear_tuning(path: str = TUNING_TABLE):
    """Remove the per-width values apply_tuning set."""
    if not os.path.exists(path):
        return
    import json
    with open(path) as f:
        rec = json.load(f)
    for w, ent in rec.get("widths", {}).items():
        for key in ent["values"]:
            set_option(f"{key}@{int(w)}", -1)


def check_sync(n, k, delta) -> bool:
    d = _delta(delta)
    rc = load().srw_check_sync(n, k, _ptr(d, ctypes.c_int32))
    if rc < 0:
        raise SrwError(rc, "check_sync")
    return bool(rc)


def verify(n, k, delta, word) -> bool:
    d = _delta(delta)
    w = np.ascontiguousarray(np.asarray(word, dtype=np.uint8))
    rc = load().srw_verify(n, k, _ptr(d, ctypes.c_int32), _ptr(w, ctypes.c_uint8), len(w))
    if rc < 0:
        raise SrwError(rc, "verify")
    return bool(rc)


def solve(n, k, delta, want_word=True, word_cap=1 << 20):
    """(r, word) of one automaton; raises SrwError on any failure."""
    d = _delta(delta)
    r = ctypes.c_int32(-1)
    word = np.zeros(word_cap if want_word else 1, dtype=np.uint8)
    rc = load().srw_solve(n, k, _ptr(d, ctypes.c_int32), ctypes.byref(r),
                          _ptr(word, ctypes.c_uint8) if want_word else None,
                          word_cap if want_word else 0)
    if rc:
        raise SrwError(rc, "solve")
    return int(r.value), ([int(x) for x in word[: r.value]] if want_word else None)


def solve_noalloc(n, k, delta, want_word=True, word_cap=1 << 20):
    """srw_solve_noalloc: (r, word) with every device buffer carved from the
    library's fixed scratch array (no allocation); raises SrwError."""
    d = _delta(delta)
    r = ctypes.c_int32(-1)
    word = np.zeros(word_cap if want_word else 1, dtype=np.uint8)
    rc = load().srw_solve_noalloc(n, k, _ptr(d, ctypes.c_int32), ctypes.byref(r),
                                  _ptr(word, ctypes.c_uint8) if want_word else None,
                                  word_cap if want_word else 0)
    if rc:
        raise SrwError(rc, "solve_noalloc")
    return int(r.value), ([int(x) for x in word[: r.value]] if want_word else None)


def solve_batch(problems, want_words=True):
    """problems: list of (n, k, delta).  Returns a list of (status, r, word)."""
    cnt = len(problems)
    ns = np.array([p[0] for p in problems], dtype=np.int32)
    ks = np.array([p[1] for p in problems], dtype=np.int32)
    sizes = np.array([p[0] * p[1] for p in problems], dtype=np.int64)
    doff = np.zeros(cnt, dtype=np.int64)
    if cnt:
        doff[1:] = np.cumsum(sizes)[:-1]
    delta = np.ascontiguousarray(np.concatenate([_delta(p[2]) for p in problems])
                                 if cnt else np.zeros(1, np.int32))
    r = np.full(cnt, -1, dtype=np.int32)
    st = np.zeros(cnt, dtype=np.int32)
    caps = np.array([max(1, (p[0] - 1) ** 2 + 8) for p in problems], dtype=np.int64)
    woff = np.zeros(cnt, dtype=np.int64)
    if cnt:
        woff[1:] = np.cumsum(caps)[:-1]
    words = np.zeros(max(1, int(caps.sum())), dtype=np.uint8)
    rc = load().srw_solve_batch(cnt, _ptr(ns, ctypes.c_int32), _ptr(ks, ctypes.c_int32),
                                _ptr(doff, ctypes.c_int64), _ptr(delta, ctypes.c_int32),
                                _ptr(r, ctypes.c_int32), _ptr(st, ctypes.c_int32),
                                _ptr(woff, ctypes.c_int64) if want_words else None,
                                _ptr(words, ctypes.c_uint8) if want_words else None,
                                _ptr(caps, ctypes.c_int64) if want_words else None)
    if rc:
        raise SrwError(rc, "solve_batch")
    out = []
    for i in range(cnt):
        w = None
        if want_words and st[i] == OK:
            w = [int(x) for x in words[woff[i]: woff[i] + r[i]]]
        out.append((int(st[i]), int(r[i]), w))
    return out


def beam_batch(problems, want_words=True):
    """problems: list of (n, k, delta, width).  Beam-search upper bounds
    (srw_beam_batch): a list of (status, R, word)."""
    cnt = len(problems)
    ns = np.array([p[0] for p in problems], dtype=np.int32)
    ks = np.array([p[1] for p in problems], dtype=np.int32)
    ws = np.array([p[3] for p in problems], dtype=np.int64)
    sizes = np.array([p[0] * p[1] for p in problems], dtype=np.int64)
    doff = np.zeros(cnt, dtype=np.int64)
    if cnt:
        doff[1:] = np.cumsum(sizes)[:-1]
    delta = np.ascontiguousarray(np.concatenate([_delta(p[2]) for p in problems])
                                 if cnt else np.zeros(1, np.int32))
    R = np.full(cnt, -1, dtype=np.int32)
    st = np.zeros(cnt, dtype=np.int32)
    caps = np.array([1 << 16 for _ in problems], dtype=np.int64)
    woff = np.arange(cnt, dtype=np.int64) * (1 << 16)
    words = np.zeros(max(1, cnt << 16), dtype=np.uint8) if want_words else np.zeros(1, np.uint8)
    rc = load().srw_beam_batch(cnt, _ptr(ns, ctypes.c_int32), _ptr(ks, ctypes.c_int32),
                               _ptr(doff, ctypes.c_int64), _ptr(delta, ctypes.c_int32),
                               _ptr(ws, ctypes.c_int64), _ptr(R, ctypes.c_int32),
                               _ptr(st, ctypes.c_int32),
                               _ptr(woff, ctypes.c_int64) if want_words else None,
                               _ptr(words, ctypes.c_uint8) if want_words else None,
                               _ptr(caps, ctypes.c_int64) if want_words else None)
    if rc:
        raise SrwError(rc, "beam_batch")
    out = []
    for i in range(cnt):
        w = None
        if want_words and st[i] == OK:
            w = [int(x) for x in words[woff[i]: woff[i] + R[i]]]
        out.append((int(st[i]), int(R[i]), w))
    return out


def beam(n, k, delta, width):
    """Beam-search upper bound of one automaton: (R, word); raises on any
    status but SRW_OK."""
    st, R, w = beam_batch([(n, k, delta, width)])[0]
    if st != OK:
        raise SrwError(st, "beam")
    return R, w


def eppstein_batch(problems, want_words=True, word_cap=1 << 22):
    """problems: list of (n, k, delta).  Eppstein upper bounds
    (srw_eppstein_batch): a list of (status, length, word)."""
    cnt = len(problems)
    ns = np.array([p[0] for p in problems], dtype=np.int32)
    ks = np.array([p[1] for p in problems], dtype=np.int32)
    sizes = np.array([p[0] * p[1] for p in problems], dtype=np.int64)
    doff = np.zeros(cnt, dtype=np.int64)
    if cnt:
        doff[1:] = np.cumsum(sizes)[:-1]
    delta = np.ascontiguousarray(np.concatenate([_delta(p[2]) for p in problems])
                                 if cnt else np.zeros(1, np.int32))
    ln = np.full(cnt, -1, dtype=np.int64)
    st = np.zeros(cnt, dtype=np.int32)
    caps = np.full(cnt, word_cap, dtype=np.int64)
    woff = np.arange(cnt, dtype=np.int64) * word_cap
    words = np.zeros(max(1, cnt * word_cap), dtype=np.uint8) if want_words else np.zeros(1, np.uint8)
    rc = load().srw_eppstein_batch(cnt, _ptr(ns, ctypes.c_int32), _ptr(ks, ctypes.c_int32),
                                   _ptr(doff, ctypes.c_int64), _ptr(delta, ctypes.c_int32),
                                   _ptr(ln, ctypes.c_int64), _ptr(st, ctypes.c_int32),
                                   _ptr(woff, ctypes.c_int64) if want_words else None,
                                   _ptr(words, ctypes.c_uint8) if want_words else None,
                                   _ptr(caps, ctypes.c_int64) if want_words else None)
    if rc:
        raise SrwError(rc, "eppstein_batch")
    out = []
    for i in range(cnt):
        w = None
        if want_words and st[i] == OK:
            w = [int(x) for x in words[woff[i]: woff[i] + ln[i]]]
        out.append((int(st[i]), int(ln[i]), w))
    return out


def eppstein(n, k, delta):
    """Eppstein upper bound of one automaton: the word; raises on any status
    but SRW_OK."""
    st, ln, w = eppstein_batch([(n, k, delta)], word_cap=max(1 << 16, n ** 3 // 3 + 1))[0]
    if st != OK:
        raise SrwError(st, "eppstein")
    return w


def bound_batch(problems, want_words=True, word_cap=1 << 16):
    """problems: list of (n, k, delta).  Upper bounds of Section 2.1.3
    (srw_bound_batch): a list of (status, R, width, word)."""
    cnt = len(problems)
    ns = np.array([p[0] for p in problems], dtype=np.int32)
    ks = np.array([p[1] for p in problems], dtype=np.int32)
    sizes = np.array([p[0] * p[1] for p in problems], dtype=np.int64)
    doff = np.zeros(cnt, dtype=np.int64)
    if cnt:
        doff[1:] = np.cumsum(sizes)[:-1]
    delta = np.ascontiguousarray(np.concatenate([_delta(p[2]) for p in problems])
                                 if cnt else np.zeros(1, np.int32))
    R = np.full(cnt, -1, dtype=np.int32)
    wd = np.zeros(cnt, dtype=np.int64)
    st = np.zeros(cnt, dtype=np.int32)
    caps = np.full(cnt, word_cap, dtype=np.int64)
    woff = np.arange(cnt, dtype=np.int64) * word_cap
    words = np.zeros(max(1, cnt * word_cap), dtype=np.uint8) if want_words else np.zeros(1, np.uint8)
    rc = load().srw_bound_batch(cnt, _ptr(ns, ctypes.c_int32), _ptr(ks, ctypes.c_int32),
                                _ptr(doff, ctypes.c_int64), _ptr(delta, ctypes.c_int32),
                                _ptr(R, ctypes.c_int32), _ptr(wd, ctypes.c_int64),
                                _ptr(st, ctypes.c_int32),
                                _ptr(woff, ctypes.c_int64) if want_words else None,
                                _ptr(words, ctypes.c_uint8) if want_words else None,
                                _ptr(caps, ctypes.c_int64) if want_words else None)
    if rc:
        raise SrwError(rc, "bound_batch")
    out = []
    for i in range(cnt):
        w = None
        if want_words and st[i] == OK:
            w = [int(x) for x in words[woff[i]: woff[i] + R[i]]]
        out.append((int(st[i]), int(R[i]), int(wd[i]), w))
    return out


def get_stats() -> dict:
    s = Stats()
    rc = load().srw_get_stats(ctypes.byref(s))
    if rc:
        raise SrwError(rc, "get_stats")
    return s.as_dict()


def reset_stats():
    load().srw_reset_stats()


def last_levels(side: int, W: int):
    """Lists of the last srw_solve run with keep_levels=1: a list of
    (rows[m, W] uint64, parent keys[m] uint32) per level."""
    L = load()
    nlev = ctypes.c_int32(0)
    nrows = ctypes.c_int64(0)
    rc = L.srw_last_levels(side, ctypes.byref(nlev), ctypes.byref(nrows), None, None, None)
    if rc:
        raise SrwError(rc, "last_levels")
    off = np.zeros(nlev.value + 1, dtype=np.int64)
    rows = np.zeros(max(1, nrows.value * W), dtype=np.uint64)
    par = np.zeros(max(1, nrows.value), dtype=np.uint32)
    rc = L.srw_last_levels(side, ctypes.byref(nlev), ctypes.byref(nrows),
                           _ptr(off, ctypes.c_int64), _ptr(rows, ctypes.c_uint64),
                           _ptr(par, ctypes.c_uint32))
    if rc:
        raise SrwError(rc, "last_levels")
    rows = rows[: nrows.value * W].reshape(nrows.value, W)
    return [(rows[off[i]:off[i + 1]].copy(), par[off[i]:off[i + 1]].copy())
            for i in range(nlev.value)]


def last_sides():
    """Sides of the steps of the last srw_solve run with keep_levels=1 (0
    forward, 1 inverse), in order."""
    L = load()
    steps = ctypes.c_int32(0)
    rc = L.srw_last_sides(ctypes.byref(steps), None, 0)
    if rc:
        raise SrwError(rc, "last_sides")
    out = np.zeros(max(1, steps.value), dtype=np.uint8)
    rc = L.srw_last_sides(ctypes.byref(steps), _ptr(out, ctypes.c_uint8), len(out))
    if rc:
        raise SrwError(rc, "last_sides")
    return [int(x) for x in out[: steps.value]]


class Server:
    """Continuous-batching server (srw_server_*)."""

    def __init__(self, device=0, max_slots=0, hbm_budget=0, deadline_ms=0):
        self._h = ctypes.c_void_p(None)
        cfg = Config(device, max_slots, hbm_budget, deadline_ms)
        rc = load().srw_server_create(ctypes.byref(self._h), ctypes.byref(cfg))
        if rc:
            raise SrwError(rc, "server_create")
        self._buf = (Result * 256)()

    def submit(self, n, k, delta, tag):
        d = _delta(delta)
        rc = _lib.srw_server_submit(self._h, n, k, _ptr(d, ctypes.c_int32), tag)
        if rc:
            raise SrwError(rc, "server_submit")

    def poll(self, timeout_us=1000, max_results=256):
        """List of dicts for the requests completed since the last poll."""
        m = min(max_results, len(self._buf))
        rc = _lib.srw_server_poll(self._h, self._buf, m, timeout_us)
        if rc == ETIMEOUT:
            return []
        if rc < 0:
            raise SrwError(rc, "server_poll")
        out = []
        for i in range(rc):
            x = self._buf[i]
            w = [x.word[t] for t in range(x.r)] if (x.status == OK and x.r > 0) else []
            out.append({"tag": int(x.tag), "status": int(x.status), "r": int(x.r), "word": w,
                        "latency_ms": float(x.latency_ms), "queue_ms": float(x.queue_ms),
                        "est_bytes": int(x.est_bytes), "dev_bytes": int(x.dev_bytes)})
        return out

    def pending(self) -> int:
        return int(_lib.srw_server_pending(self._h))

    def close(self):
        if self._h:
            _lib.srw_server_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
