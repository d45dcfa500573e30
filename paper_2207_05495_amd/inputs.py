"""Seeded synthetic inputs: random automata and Černý automata.

This module only draws transition tables.  It holds none of the search
arithmetic (no images, no preimages, no synchronizability test), so both the
GPU harness and the CPU oracle tests can share it.

Random automata follow the experimental setup of the paper (Section 3): every
transition delta(q, a) is drawn uniformly from Q, and draws that turn out not
to be synchronizing are excluded.  The paper does not name a generator, so the
recipe is fixed here:

* SplitMix64 (Steele, Lea, Flood 2014) is counter based: output i of the
  stream seeded with ``s`` is ``mix(s + (i + 1) * GAMMA)`` with the published
  finaliser ``mix``.  That makes it vectorisable in numpy.
* A uniform draw on [0, n) is ``((x >> 32) * n) >> 32`` (32-bit
  multiply-high; bias below n / 2**32).
* Attempt ``t`` of an automaton fills delta letter-major (a outer, q inner)
  from outputs ``t*k*n .. (t+1)*k*n - 1``.  A caller that finds attempt ``t``
  not synchronizing asks for attempt ``t + 1`` (the continuing stream).
* Member ``i`` of a batch seeded with ``base`` uses seed ``mix(base ^ i)``.

Layout of every table returned: ``delta[a * n + q] = delta(q, a)``, int32,
shape (k * n,), the layout the C ABI takes.

The Černý automaton C_n is not defined in the paper (it only cites it as the
series meeting the (n-1)^2 bound, Section 1.1 and Section 3.1.1).  Convention
used here: letter 0 maps state 0 to state 1 and fixes every other state;
letter 1 is the cyclic shift q -> q + 1 mod n.
"""

from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
BASE_SEED = 2207055495

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: int) -> int:
    """SplitMix64 finaliser on a Python int (mod 2**64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix64_stream(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream of ``seed``."""
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + idx * np.uint64(GAMMA)
    return _mix64_np(z)


def member_seed(base: int, index: int) -> int:
    """Seed of member ``index`` of a batch seeded with ``base``."""
    return mix64((base ^ index) & MASK64)


def random_automaton(n: int, k: int, seed: int, attempt: int = 0) -> np.ndarray:
    """Attempt ``attempt`` of the uniform random automaton with this seed."""
    if n < 1 or k < 1:
        raise ValueError("n and k must be positive")
    x = splitmix64_stream(seed, attempt * k * n, k * n)
    d = ((x >> np.uint64(32)) * np.uint64(n)) >> np.uint64(32)
    return d.astype(np.int32)


def first_synchronizing(n: int, k: int, seed: int, is_sync, max_attempts: int = 64):
    """First attempt that the predicate ``is_sync(n, k, delta)`` accepts.

    The predicate is supplied by the caller (the library's own check on the
    product side, the oracle's check in oracle tests), so this module never
    decides synchronizability itself.  Returns ``(delta, attempt)``.
    """
    for t in range(max_attempts):
        d = random_automaton(n, k, seed, t)
        if is_sync(n, k, d):
            return d, t
    raise RuntimeError(f"no synchronizing draw in {max_attempts} attempts "
                       f"(n={n}, k={k}, seed={seed})")


def cerny(n: int) -> np.ndarray:
    """Černý automaton C_n (two letters) in the convention stated above."""
    if n < 1:
        raise ValueError("n must be positive")
    q = np.arange(n, dtype=np.int32)
    merge = q.copy()
    if n > 1:
        merge[0] = 1
    rotate = ((q + 1) % n).astype(np.int32)
    return np.concatenate([merge, rotate]).astype(np.int32)


def cerny_word(n: int) -> list[int]:
    """The word (0 1^(n-1))^(n-2) 0, of length (n-1)^2, for C_n (n >= 2)."""
    if n < 2:
        return []
    return ([0] + [1] * (n - 1)) * (n - 2) + [0]


def sink_series(n: int) -> np.ndarray:
    """Rystsov's series with a sink (Section 3.1.1): n states,
    state 0 the sink, n - 1 letters.  Letter 0 sends state 1 to the sink and
    fixes every other state; letter i (1 <= i <= n - 2) swaps states i and
    i + 1 and fixes the rest.  Its reset threshold is n(n - 1)/2, the largest
    an automaton with a sink can have."""
    if n < 2:
        raise ValueError("n must be at least 2")
    k = n - 1
    d = np.tile(np.arange(n, dtype=np.int32), (k, 1))
    d[0, 1] = 0
    for i in range(1, n - 1):
        d[i, i], d[i, i + 1] = i + 1, i
    return d.reshape(-1)


def sink_word(n: int) -> list[int]:
    """The blocks (j, j-1, ..., 1, 0) for j = 0, ..., n - 2, of total length
    n(n - 1)/2, for the sink series of n states (n >= 2)."""
    return [a for j in range(n - 1) for a in range(j, -1, -1)]


def relabel(delta: np.ndarray, n: int, k: int, perm: np.ndarray) -> np.ndarray:
    """The same automaton with state q renamed perm[q]."""
    d = np.asarray(delta, dtype=np.int64).reshape(k, n)
    out = np.empty_like(d)
    for a in range(k):
        out[a, perm] = perm[d[a]]
    return out.reshape(-1).astype(np.int32)


def permute_letters(delta: np.ndarray, n: int, k: int, sigma) -> np.ndarray:
    """The same automaton with letter a renamed sigma[a]."""
    d = np.asarray(delta, dtype=np.int32).reshape(k, n)
    out = np.empty_like(d)
    for a in range(k):
        out[sigma[a]] = d[a]
    return out.reshape(-1)


# ---- workload recipes (sizes of the paper's experiments, Section 3) --------

def config_single(n: int, k: int, count: int, is_sync, base: int = BASE_SEED):
    """``count`` synchronizing random automata with fixed n, k."""
    out = []
    for i in range(count):
        s = member_seed(base, i)
        d, t = first_synchronizing(n, k, s, is_sync)
        out.append({"n": n, "k": k, "seed": s, "attempt": t, "delta": d})
    return out


def mixed_batch(count: int, n_lo: int, n_hi: int, ks, is_sync,
                 base: int = BASE_SEED):
    """Random automata with n uniform in [n_lo, n_hi] and k uniform in ks.

    The size draw for member i uses outputs 0 and 1 of its own stream's
    sibling seed ``mix(seed ^ 0x5A5A...)`` so it never overlaps the table.
    """
    out = []
    ks = list(ks)
    for i in range(count):
        s = member_seed(base, i)
        sz = splitmix64_stream(mix64(s ^ 0x5A5A5A5A5A5A5A5A), 0, 2)
        n = n_lo + int(((int(sz[0]) >> 32) * (n_hi - n_lo + 1)) >> 32)
        k = ks[int(((int(sz[1]) >> 32) * len(ks)) >> 32)]
        d, t = first_synchronizing(n, k, s, is_sync)
        out.append({"n": n, "k": k, "seed": s, "attempt": t, "delta": d})
    return out


def serve_mix(count: int, nmax: int, kmax: int, is_sync, base: int = BASE_SEED ^ 5):
    """Requests of the serving workload, in arrival order: 90% random
    automata (n uniform in [64, nmax], k uniform in 2..kmax), 10% Černý C_n
    with n uniform in [8, 40].  Returns dicts with n, k, delta, label and,
    for random members, seed and attempt (the class draws come from numpy's
    PCG64 seeded with the low 32 bits of ``base``; request i's table is
    member i of the batch seeded with ``base``)."""
    rng = np.random.default_rng(base & 0xFFFFFFFF)
    out = []
    for i in range(count):
        if rng.random() < 0.1:
            n = int(rng.integers(8, 41))
            out.append({"n": n, "k": 2, "delta": cerny(n), "label": "cerny"})
        else:
            n = int(rng.integers(64, nmax + 1))
            k = int(rng.integers(2, kmax + 1))
            s = member_seed(base, i)
            d, t = first_synchronizing(n, k, s, is_sync)
            out.append({"n": n, "k": k, "delta": d, "seed": s, "attempt": t,
                        "label": f"k{k}" + ("big" if n > 300 else "")})
    return out
