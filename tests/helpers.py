"""Test-side helpers: golden-fixture loading and small instance builders.

Instances here are described the way the paper writes them: variables, domains,
and for each constraint the set of allowed value pairs (Section 2)."""
from __future__ import annotations

import glob
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_cases():
    out = []
    for path in sorted(glob.glob(os.path.join(GOLDEN, "*.json"))):
        with open(path) as f:
            case = json.load(f)
        case["name"] = os.path.basename(path)[:-5]
        out.append(case)
    return out


def instance_from_pairs(n, d, constraints):
    """constraints: list of (x, y, allowed_pairs) -> edges [m,2], rel_u8 [m,d,d]."""
    m = len(constraints)
    edges = np.zeros((m, 2), dtype=np.int32)
    rel = np.zeros((m, d, d), dtype=np.uint8)
    for e, (x, y, allowed) in enumerate(constraints):
        edges[e] = (x, y)
        for a, b in allowed:
            rel[e, a, b] = 1
    return edges, rel


def golden_instance(case):
    n, d = case["n"], case["d"]
    edges, rel = instance_from_pairs(n, d, [(c["x"], c["y"], c["allowed"]) for c in case["constraints"]])
    return n, d, edges, rel, value_lists_to_u8(case["domains"], d)


def value_lists_to_u8(lists, d):
    out = np.zeros((len(lists), d), dtype=np.uint8)
    for x, vals in enumerate(lists):
        for a in vals:
            out[x, a] = 1
    return out


def masks_to_u8(masks, d):
    masks = np.asarray(masks, dtype=np.uint64)
    out = np.zeros(masks.shape + (d,), dtype=np.uint8)
    for a in range(d):
        out[..., a] = ((masks >> np.uint64(a)) & np.uint64(1)).astype(np.uint8)
    return out


def u8_to_masks(u8):
    u8 = np.asarray(u8)
    d = u8.shape[-1]
    out = np.zeros(u8.shape[:-1], dtype=np.uint64)
    for a in range(d):
        out |= u8[..., a].astype(np.uint64) << np.uint64(a)
    return out


def chain(L, d, relation):
    """x0 - x1 - ... - xL with the same relation on every link."""
    allowed = [(a, b) for a in range(d) for b in range(d) if relation(a, b)]
    return instance_from_pairs(L + 1, d, [(i, i + 1, allowed) for i in range(L)])


def clique_neq(n, d):
    allowed = [(a, b) for a in range(d) for b in range(d) if a != b]
    cons = [(x, y, allowed) for x in range(n) for y in range(x + 1, n)]
    return instance_from_pairs(n, d, cons)


def oracle_expect(n, d, edges, rel_u8, dom_masks, mode=0, changed=None, max_steps=0):
    """What the oracle says for one state: (dom masks [n], iters, status, checks, converged).

    Run-to-fixpoint: domains and status from AC-3 (the closure D_ac), the step
    count from the Eq. (1) recurrence; the two must agree on the domains.
    Stop-on-wipe-out: everything from the recurrence."""
    import oracle

    dom_u8 = masks_to_u8(dom_masks, d)
    r = oracle.rac_sync(n, d, edges, rel_u8, dom_u8, changed0=changed, mode=mode,
                        max_steps=max_steps)
    if mode == 0 and changed is None and r["converged"]:
        dac, status, _, _ = oracle.ac3(n, d, edges, rel_u8, dom_u8)
        assert np.array_equal(dac, r["dom"]), "oracle disagrees with itself"
        assert status == r["status"]
    return u8_to_masks(r["dom"]), r["iters"], r["status"], r["checks"], r["converged"]


def queens(n):
    """The n-queens problem (the generator's builder): (edges, relations)."""
    from paper_2407_11388_amd import gen
    return gen.queens(n)


def cycle_colouring(n, k):
    """Proper k-colourings of the cycle on n >= 3 vertices."""
    neq = [(a, b) for a in range(k) for b in range(k) if a != b]
    return instance_from_pairs(n, k, [(i, (i + 1) % n, neq) for i in range(n)])
