"""MAC search (maintaining arc consistency) on the CPU — TEST INFRASTRUCTURE
ONLY, like the rest of ``oracle``.

Algorithm 2 of the paper: a depth-first search that, after every
assignment, enforces arc consistency and backtracks on a wipe-out. The
paper leaves the branching heuristic open; the reading used here (and by
the GPU search) is: branch on the variable with the smallest domain of size
> 1 (lowest index on ties), one child per value in ascending order.

Every node's domains are the closure D_ac of its initial domains, computed by
the oracle's AC-3 (``oracle.ac3``) run from scratch; the closure is unique, so
any arc-consistency algorithm gives the same tree. Per node the search also
records the steps of the Eq. (1) recurrence (``oracle.rac_sync``, stopping at
the first wipe-out, started from the assigned variable as @changed for a
child: Proposition 2) and AC-3's revisions, the two counts Table 1 compares.
A node is a failure when its closure has an empty domain, a solution when
every domain is a singleton (an arc-consistent state of singletons satisfies
every constraint), and open otherwise.

Pins (``tests/test_search_oracle.py``): the solution set equals ``brute.solutions``
on tiny instances; closed forms for unconstrained variables (d^n solutions,
1 + d + ... + d^n nodes), proper colourings of a cycle ((k-1)^n +
(-1)^n (k-1)) and the n-queens counts.
"""
from __future__ import annotations

import numpy as np

from . import STOP_ON_WIPEOUT, ac3, rac_sync


def mac_search(n: int, d: int, edges, rel_u8, dom_u8, max_nodes: int = 10_000_000,
               stop_after: int = 0):
    """MAC search. Returns dict(solutions, nodes, failures, steps, revisions,
    complete, best, assignments): ``best`` is the lexicographically smallest
    solution as an int array [n] (value of variable 0 first), ``assignments``
    all solutions as an int array [S, n]; ``steps`` and ``revisions`` are
    summed over the enforced nodes. ``stop_after`` > 0 ends the search (not
    complete) once that many nodes were enforced; more than ``max_nodes``
    raises."""
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    rel_u8 = np.ascontiguousarray(rel_u8, dtype=np.uint8)
    dom_u8 = np.asarray(dom_u8, dtype=np.uint8)

    counts = dict(steps=0, revisions=0)

    def closure(dom, changed=None):
        out, status, revisions, _ = ac3(n, d, edges, rel_u8, dom)
        r = rac_sync(n, d, edges, rel_u8, dom, changed0=changed, mode=STOP_ON_WIPEOUT)
        if (r["status"] != 0) != (status != 0):
            raise AssertionError("mac_search: AC-3 and the recurrence disagree on a wipe-out")
        counts["steps"] += r["iters"]
        counts["revisions"] += revisions
        return out, status != 0

    nodes, failures = 1, 0
    found = []
    root, wiped = closure(dom_u8)
    stack = []
    if wiped:
        failures = 1
    elif (root.sum(axis=1) == 1).all():
        found.append(root.argmax(axis=1))
    else:
        stack.append(root)
    complete = True
    while stack:
        if nodes > max_nodes:
            raise RuntimeError("mac_search: node limit exceeded")
        if stop_after and nodes >= stop_after:
            complete = False
            break
        node = stack.pop()
        sizes = node.sum(axis=1)
        cand = np.where(sizes > 1, sizes, d + 1)
        x = int(np.argmin(cand))        # smallest size > 1, lowest index first
        for a in np.nonzero(node[x])[0]:
            child = node.copy()
            child[x] = 0
            child[x, a] = 1
            res, wiped = closure(child, [x])
            nodes += 1
            if wiped:
                failures += 1
            elif (res.sum(axis=1) == 1).all():
                found.append(res.argmax(axis=1))
            else:
                stack.append(res)
    assignments = np.array(found, dtype=np.int64).reshape(-1, n)
    best = None
    if len(found):
        order = np.lexsort(assignments.T[::-1])
        best = assignments[order[0]]
    return dict(solutions=len(found), nodes=nodes, failures=failures, steps=counts["steps"],
                revisions=counts["revisions"], complete=complete, best=best,
                assignments=assignments)
