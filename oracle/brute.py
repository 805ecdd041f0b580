"""Definitions of arc consistency evaluated by exhaustive enumeration (tiny
instances only). TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

* ``brute_dac``   Section 3: a set D' of values is arc consistent iff every
  (x,a) in D' has, on every constraint c_xy of x, a support (y,b) in D'; the
  closure D_ac is the union of all arc-consistent subsets of D. Evaluated by
  testing every subset of D (|D| <= 22).
* ``solutions``   every complete assignment drawn from D that satisfies every
  constraint (enumeration with the constraints among already-assigned
  variables checked as they are fixed, which never drops a solution).
"""
from __future__ import annotations

import numpy as np


def _neighbour_constraints(n, edges):
    """For each variable x: list of (y, edge index, x-is-second-endpoint)."""
    nb = [[] for _ in range(n)]
    for e, (x, y) in enumerate(np.asarray(edges).tolist()):
        nb[x].append((y, e, False))
        nb[y].append((x, e, True))
    return nb


def _allowed(rel_u8, e, flip, a, b):
    return bool(rel_u8[e, b, a]) if flip else bool(rel_u8[e, a, b])


def brute_dac(n: int, d: int, edges, rel_u8, dom_u8) -> np.ndarray:
    """Union of all arc-consistent subsets of D, as 0/1 bytes [n, d]."""
    dom_u8 = np.asarray(dom_u8, dtype=np.uint8)
    rel_u8 = np.asarray(rel_u8, dtype=np.uint8)
    values = [(x, a) for x in range(n) for a in range(d) if dom_u8[x, a]]
    N = len(values)
    if N > 22:
        raise ValueError("brute_dac: |D| too large for exhaustive enumeration")
    index = {v: i for i, v in enumerate(values)}
    nb = _neighbour_constraints(n, edges)
    subsets = np.arange(1 << N, dtype=np.uint32)
    ok = np.ones(1 << N, dtype=bool)
    for i, (x, a) in enumerate(values):
        member = ((subsets >> np.uint32(i)) & np.uint32(1)).astype(bool)
        for (y, e, flip) in nb[x]:
            supp = 0
            for b in range(d):
                if dom_u8[y, b] and _allowed(rel_u8, e, flip, a, b):
                    supp |= 1 << index[(y, b)]
            has_support = (subsets & np.uint32(supp)) != 0
            ok &= (~member) | has_support
    union = np.bitwise_or.reduce(subsets[ok]) if ok.any() else np.uint32(0)
    out = np.zeros((n, d), dtype=np.uint8)
    for i, (x, a) in enumerate(values):
        if (int(union) >> i) & 1:
            out[x, a] = 1
    return out


def solutions(n: int, d: int, edges, rel_u8, dom_u8, limit: int = 2_000_000) -> np.ndarray:
    """All solutions within D as an int array [S, n]."""
    dom_u8 = np.asarray(dom_u8, dtype=np.uint8)
    rel_u8 = np.asarray(rel_u8, dtype=np.uint8)
    size = 1
    for x in range(n):
        size *= max(1, int(dom_u8[x].sum()))
    if size > limit:
        raise ValueError("solutions: search space too large")
    edges = np.asarray(edges)
    partial = np.zeros((1, 0), dtype=np.int64)
    for x in range(n):
        vals = np.nonzero(dom_u8[x])[0]
        if len(vals) == 0:
            return np.zeros((0, n), dtype=np.int64)
        rep = np.repeat(partial, len(vals), axis=0)
        col = np.tile(vals, partial.shape[0]).reshape(-1, 1)
        cand = np.concatenate([rep, col], axis=1)
        keep = np.ones(cand.shape[0], dtype=bool)
        for e, (u, v) in enumerate(edges.tolist()):
            if max(u, v) != x:
                continue
            keep &= rel_u8[e, cand[:, u], cand[:, v]].astype(bool)
        partial = cand[keep]
        if partial.shape[0] == 0:
            return np.zeros((0, n), dtype=np.int64)
    return partial
