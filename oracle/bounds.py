"""The upper bound of Section 2.1.3: Eppstein's heuristic first, then the
beam search with a small beam, then the beam search with a beam size chosen
from a rough estimate of the exact algorithm's cost.

TEST INFRASTRUCTURE ONLY.  Only the test suite may import this module; the
library never does.

The paper states the policy in words only; readings where it is silent:
  - the small beam is w0 = n;
  - B = the least bound found so far (Eppstein's length, the first beam's R);
  - the exact cost is estimated from the first beam's levels before their
    cut: those up to the first level larger than w0 are the exact inverse
    search's; beyond it a level grows by g = U_c / U_(c-1), the ratio of that
    first large level to the one before.  The exact search takes both sides
    to about depth h = ceil(B / 2), so its cost is C = 2 * sum over d <= h of
    U(d) sets;
  - a beam of width w costs about w * B sets; its share of the exact cost is
    1/16, so w1 = ceil(C / (16 B)), clamped to [w0, 2^20];
  - no level of the first beam larger than w0: it was the exact inverse
    search, so R = r already and no second beam is run (w1 = w0);
  - R is the least of the three bounds; its word is that of the first
    source reaching it, in the order Eppstein, first beam, second beam.

Parity unpinned beyond the invariants of tests/test_bounds_oracle.py: the
paper gives no beam size it chose.
"""

from __future__ import annotations

import math

from oracle import oracle as O

FRACTION = 16
MAX_WIDTH = 1 << 20


def exact_cost(sizes, w0, B):
    """C of the policy above from the first beam's level sizes, or None
    when no level was larger than w0."""
    c = next((L for L, u in enumerate(sizes) if u > w0), None)
    if c is None:
        return None
    g = sizes[c] / sizes[c - 1]
    h = (B + 1) // 2
    total, u = 0.0, 0.0
    for d in range(h + 1):
        u = float(sizes[d]) if d <= c else u * g
        total += u
        if total > 1e30:
            break
    return 2.0 * total


def adaptive_width(sizes, w0, B):
    C = exact_cost(sizes, w0, B)
    if C is None:
        return w0
    w = math.ceil(C / (FRACTION * B))
    return int(min(max(w, w0), MAX_WIDTH))


def upper_bound(n, k, delta):
    """(R, word, w1, source) with source 0 Eppstein, 1 the first beam, 2 the
    second beam."""
    if n == 1:
        return 0, [], n, 0
    ew, _ = O.eppstein(n, k, delta)
    w0 = n
    R0, w0word, sizes = O.beam_sizes(n, k, delta, w0)
    cands = [(len(ew), 0, ew)]
    if R0 is not None:
        cands.append((R0, 1, w0word))
    B = min(c[0] for c in cands)
    w1 = adaptive_width(sizes, w0, B)
    if w1 > w0:
        R1, w1word, _ = O.beam_sizes(n, k, delta, w1)
        if R1 is not None:
            cands.append((R1, 2, w1word))
    R, src, word = min(cands, key=lambda c: (c[0], c[1]))
    return R, list(word), w1, src
