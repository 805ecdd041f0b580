"""Pins of the oracle's MAC search (Algorithm 2 with the smallest-domain
branching reading): brute-force solution sets, closed-form counts."""
import numpy as np
import pytest

from oracle import brute
from oracle.search import mac_search
from paper_2407_11388_amd import gen

from helpers import cycle_colouring, queens


@pytest.mark.parametrize("seed", range(0, 40))
def test_solutions_equal_brute_force(seed):
    n = 2 + seed % 5
    d = 1 + (seed // 5) % 4
    inst, dom_masks = gen.random_tiny(7000 + seed, n, d, [0.5, 0.8, 1.0][seed % 3],
                                      [0.2, 0.4, 0.6][(seed // 3) % 3], 1.0)
    rel = inst.rel_u8()
    dom = np.array([[(int(m) >> a) & 1 for a in range(d)] for m in dom_masks], np.uint8)
    r = mac_search(n, d, inst.edges, rel, dom)
    sols = brute.solutions(n, d, inst.edges, rel, dom)
    assert r["solutions"] == len(sols)
    assert {tuple(s) for s in r["assignments"].tolist()} == {tuple(s) for s in sols.tolist()}
    if len(sols):
        assert tuple(r["best"].tolist()) == min(tuple(s) for s in sols.tolist())
    # leaves (failures and solutions) are among the enforced nodes
    assert r["failures"] + r["solutions"] <= r["nodes"]


@pytest.mark.parametrize("n,d", [(1, 4), (2, 3), (3, 3), (4, 2)])
def test_unconstrained_tree(n, d):
    # no constraint prunes anything: every assignment is a solution, and the
    # tree branches on x0, x1, ... in turn (all sizes equal, lowest index)
    r = mac_search(n, d, np.zeros((0, 2), np.int32), np.zeros((0, d, d), np.uint8),
                   np.ones((n, d), np.uint8))
    assert r["solutions"] == d ** n
    assert r["failures"] == 0
    assert r["nodes"] == sum(d ** i for i in range(n + 1))
    # nothing to propagate: every enforcement takes exactly one step
    assert r["steps"] == r["nodes"]
    assert r["best"].tolist() == [0] * n


@pytest.mark.parametrize("n,k", [(3, 3), (4, 3), (5, 3), (6, 2), (7, 2), (5, 4), (6, 3)])
def test_cycle_colourings(n, k):
    edges, rel = cycle_colouring(n, k)
    r = mac_search(n, k, edges, rel, np.ones((n, k), np.uint8))
    assert r["solutions"] == (k - 1) ** n + (-1) ** n * (k - 1)


@pytest.mark.parametrize("n,count", [(4, 2), (5, 10), (6, 4), (7, 40), (8, 92)])
def test_queens(n, count):
    edges, rel = queens(n)
    r = mac_search(n, n, edges, rel, np.ones((n, n), np.uint8))
    assert r["solutions"] == count
    # every solution is a valid placement
    for s in r["assignments"].tolist():
        for i in range(n):
            for j in range(i + 1, n):
                assert s[i] != s[j] and abs(s[i] - s[j]) != j - i
