"""Pins of the CPU oracle against what the paper and the mathematics fix.

* Brute force (the definition of Section 3: D_ac is the union of all
  arc-consistent subsets of D) on tiny random instances, including asymmetric
  relations, pre-removed and empty initial domains.
* Hand-worked golden cases (tests/golden/*.json), including every step of the
  Eq. (1) recurrence.
* Closed forms: no constraints, universal and empty relations, equality and
  strict-order chains (the step count is the chain length + 1), the !=-clique.
* Invariants: result arc consistent, idempotent, monotone, contains every
  solution; Proposition 1 (steps shrink D and never go below D_ac, the count is
  bounded by |D|+1); Proposition 2 (the @changed restriction changes no step);
  restart from any intermediate step.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2407_11388_amd import gen

from helpers import (chain, clique_neq, golden_cases, golden_instance, masks_to_u8,
                     value_lists_to_u8)

CASES = golden_cases()


def tiny_instances():
    """(n, d, edges, rel_u8, dom_u8) with |D| <= 16, deterministic."""
    out = []
    for seed in range(120):
        n = 2 + seed % 4                 # 2..5 variables
        d = 2 + (seed // 4) % 3          # 2..4 values
        p1 = [0.5, 0.8, 1.0][seed % 3]
        p2 = [0.3, 0.5, 0.7][(seed // 3) % 3]
        keep = [1.0, 0.8, 0.6][(seed // 9) % 3]
        inst, dom = gen.random_tiny(1000 + seed, n, d, p1, p2, keep)
        dom_u8 = masks_to_u8(dom, d)
        if dom_u8.sum() > 16:
            # drop values deterministically until |D| <= 16
            flat = np.argwhere(dom_u8)
            for (x, a) in flat[16:]:
                dom_u8[x, a] = 0
        out.append((n, d, inst.edges, inst.rel_u8(), dom_u8))
    return out


TINY = tiny_instances()


# --------------------------------------------------------------------------
# golden, hand-worked cases
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_ac3(case):
    n, d, edges, rel, dom = golden_instance(case)
    got, status, _, _ = oracle.ac3(n, d, edges, rel, dom)
    assert np.array_equal(got, value_lists_to_u8(case["expect_dac"], d))
    assert status == case["expect_status"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_ac3_counters(case):
    # revisions (arcs popped and revised: Table 1's #Revision) and relation
    # look-ups, counted by hand for the FIFO order stated in each fixture
    n, d, edges, rel, dom = golden_instance(case)
    _, _, revisions, lookups = oracle.ac3(n, d, edges, rel, dom)
    assert revisions == case["expect_ac3_revisions"]
    assert lookups == case["expect_ac3_lookups"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_is_ac_rejects_each_removed_value(case):
    # Section 3: D_ac is the largest arc-consistent subset of D, so D_ac plus
    # any value of D it lacks is not arc consistent; D_ac itself is.
    n, d, edges, rel, dom = golden_instance(case)
    dac = value_lists_to_u8(case["expect_dac"], d)
    assert oracle.is_ac(n, d, edges, rel, dac)
    removed = np.argwhere(dom & (1 - dac))
    for x, a in removed:
        plus = dac.copy()
        plus[x, a] = 1
        assert not oracle.is_ac(n, d, edges, rel, plus), (x, a)
    assert oracle.is_ac(n, d, edges, rel, dom) == (len(removed) == 0)


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
@pytest.mark.parametrize("incremental", [True, False])
def test_golden_recurrence_steps(case, incremental):
    n, d, edges, rel, dom = golden_instance(case)
    r = oracle.rac_sync(n, d, edges, rel, dom, incremental=incremental, trace=True)
    assert r["iters"] == case["expect_iters"]
    assert r["status"] == case["expect_status"]
    assert np.array_equal(r["dom"], value_lists_to_u8(case["expect_dac"], d))
    expect_trace = np.stack([value_lists_to_u8(s, d) for s in case["expect_trace"]])
    assert np.array_equal(r["trace"], expect_trace)
    if "expect_iters_stop_on_wipeout" in case:
        r1 = oracle.rac_sync(n, d, edges, rel, dom, mode=oracle.STOP_ON_WIPEOUT)
        assert r1["iters"] == case["expect_iters_stop_on_wipeout"] and r1["status"] == 1


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_brute_force_agrees(case):
    n, d, edges, rel, dom = golden_instance(case)
    assert np.array_equal(brute.brute_dac(n, d, edges, rel, dom),
                          value_lists_to_u8(case["expect_dac"], d))
    if "expect_solutions" in case:
        assert len(brute.solutions(n, d, edges, rel, dom)) == case["expect_solutions"]


# --------------------------------------------------------------------------
# brute force on tiny instances (the definition of D_ac)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("idx", range(len(TINY)))
def test_ac3_and_recurrence_equal_brute_force(idx):
    n, d, edges, rel, dom = TINY[idx]
    expect = brute.brute_dac(n, d, edges, rel, dom)
    got, status, _, _ = oracle.ac3(n, d, edges, rel, dom)
    assert np.array_equal(got, expect)
    assert status == int((expect.sum(axis=1) == 0).any())
    for inc in (True, False):
        r = oracle.rac_sync(n, d, edges, rel, dom, incremental=inc)
        assert np.array_equal(r["dom"], expect)
        assert r["converged"]
    # every solution survives (Section 3: solutions are arc consistent sets)
    sols = brute.solutions(n, d, edges, rel, dom)
    for s in sols:
        assert all(expect[x, s[x]] for x in range(n))


@pytest.mark.parametrize("idx", range(0, len(TINY), 3))
def test_is_ac_equals_definition_by_brute_force(idx):
    # A set S is arc consistent iff it equals its own closure (the union of
    # all arc-consistent subsets of S contains S exactly when S is one of
    # them). Checked on D, on D_ac, on D_ac plus each value it lacks and on
    # D_ac minus each value it holds.
    n, d, edges, rel, dom = TINY[idx]
    dac = brute.brute_dac(n, d, edges, rel, dom)
    sets = [dom, dac]
    for x, a in np.argwhere(dom):
        s = dac.copy()
        s[x, a] = 1 - s[x, a]
        sets.append(s)
    for s in sets:
        expect = np.array_equal(brute.brute_dac(n, d, edges, rel, s), s)
        assert oracle.is_ac(n, d, edges, rel, s) == expect


def test_oracle_rejects_duplicate_constraints():
    # Section 2: at most one constraint per pair of variables; (x,y) and then
    # (y,x) is the same pair.
    d = 3
    rel = np.ones((2, d, d), np.uint8)
    dom = np.ones((3, d), np.uint8)
    for edges in (np.array([[0, 1], [0, 1]], np.int32), np.array([[0, 1], [1, 0]], np.int32),
                  np.array([[2, 2], [0, 1]], np.int32)):
        with pytest.raises(ValueError):
            oracle.ac3(3, d, edges, rel, dom)
        with pytest.raises(ValueError):
            oracle.rac_sync(3, d, edges, rel, dom)
        with pytest.raises(ValueError):
            oracle.is_ac(3, d, edges, rel, dom)


def test_ac3_counters_closed_form_universal_relations():
    # Nothing is removed when every pair is allowed: each arc is popped once
    # (2m revisions) and each value of x finds its support at the first value
    # of dom(y) tried (|dom(x)| look-ups per arc x->y).
    inst = gen.model_b(21, 25, 5, 0.6, 0.0)
    dom = masks_to_u8(gen.preremove(22, 25, 5, 30), 5)
    dom[dom.sum(axis=1) == 0, 2] = 1
    _, status, revisions, lookups = oracle.ac3(25, 5, inst.edges, inst.rel_u8(), dom)
    size = dom.sum(axis=1)
    assert status == 0 and revisions == 2 * inst.m
    assert lookups == int(sum(size[x] + size[y] for x, y in inst.edges))


def test_brute_force_catches_transposed_relation():
    # The asymmetric golden case distinguishes R from its transpose: reading
    # the arc y->x with the untransposed relation gives a different closure.
    case = [c for c in CASES if c["name"] == "asymmetric_pair"][0]
    n, d, edges, rel, dom = golden_instance(case)
    wrong = brute.brute_dac(n, d, edges, rel.transpose(0, 2, 1).copy(), dom)
    assert not np.array_equal(wrong, value_lists_to_u8(case["expect_dac"], d))


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

def test_no_constraints():
    n, d = 6, 5
    edges = np.zeros((0, 2), np.int32)
    rel = np.zeros((0, d, d), np.uint8)
    dom = masks_to_u8(np.array([31, 1, 0, 7, 16, 5], np.uint64), d)
    r = oracle.rac_sync(n, d, edges, rel, dom)
    assert np.array_equal(r["dom"], dom) and r["iters"] == 1
    got, status, revisions, _ = oracle.ac3(n, d, edges, rel, dom)
    assert np.array_equal(got, dom) and revisions == 0 and status == 1


def test_universal_relations():
    inst = gen.model_b(8, 30, 6, 0.7, 0.0)
    dom = masks_to_u8(gen.preremove(9, 30, 6, 40), 6)
    dom[dom.sum(axis=1) == 0, 0] = 1
    r = oracle.rac_sync(30, 6, inst.edges, inst.rel_u8(), dom)
    assert np.array_equal(r["dom"], dom) and r["iters"] == 1 and r["status"] == 0


def test_empty_relations():
    inst = gen.model_b(8, 30, 6, 0.3, 1.0)
    dom = np.ones((30, 6), np.uint8)
    isolated = np.ones(30, bool)
    isolated[inst.edges.ravel()] = False
    r = oracle.rac_sync(30, 6, inst.edges, inst.rel_u8(), dom)
    assert r["iters"] == 2 and r["status"] == 1
    assert (r["dom"][~isolated] == 0).all() and (r["dom"][isolated] == 1).all()
    r1 = oracle.rac_sync(30, 6, inst.edges, inst.rel_u8(), dom, mode=oracle.STOP_ON_WIPEOUT)
    assert r1["iters"] == 1 and r1["status"] == 1
    got, _, _, _ = oracle.ac3(30, 6, inst.edges, inst.rel_u8(), dom)
    assert np.array_equal(got, r["dom"])


@pytest.mark.parametrize("L,d,v", [(1, 2, 0), (3, 3, 1), (7, 5, 4), (12, 4, 2)])
def test_equality_chain(L, d, v):
    edges, rel = chain(L, d, lambda a, b: a == b)
    dom = np.ones((L + 1, d), np.uint8)
    dom[0] = 0
    dom[0, v] = 1
    r = oracle.rac_sync(L + 1, d, edges, rel, dom, trace=True)
    expect = np.zeros_like(dom)
    expect[:, v] = 1
    assert np.array_equal(r["dom"], expect) and r["iters"] == L + 1
    # step k fixes exactly x_k
    for k in range(1, L + 1):
        assert r["trace"][k - 1][: k + 1].sum() == k + 1
    got, _, _, _ = oracle.ac3(L + 1, d, edges, rel, dom)
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("L,d", [(1, 2), (2, 3), (4, 9), (6, 7), (10, 12)])
def test_strict_chain(L, d):
    edges, rel = chain(L, d, lambda a, b: a < b)
    dom = np.ones((L + 1, d), np.uint8)
    r = oracle.rac_sync(L + 1, d, edges, rel, dom)
    expect = np.zeros_like(dom)
    for i in range(L + 1):
        expect[i, i: d - L + i] = 1
    assert np.array_equal(r["dom"], expect)
    assert r["iters"] == L + 1 and r["status"] == 0


@pytest.mark.parametrize("L,d", [(2, 2), (5, 5), (8, 3)])
def test_strict_chain_too_long_wipes_out(L, d):
    edges, rel = chain(L, d, lambda a, b: a < b)
    dom = np.ones((L + 1, d), np.uint8)
    r = oracle.rac_sync(L + 1, d, edges, rel, dom)
    assert r["status"] == 1 and r["dom"].sum() == 0
    got, status, _, _ = oracle.ac3(L + 1, d, edges, rel, dom)
    assert status == 1 and got.sum() == 0


@pytest.mark.parametrize("n", [3, 4, 6])
def test_neq_clique_is_arc_consistent_but_unsatisfiable(n):
    d = n - 1
    edges, rel = clique_neq(n, d)
    dom = np.ones((n, d), np.uint8)
    r = oracle.rac_sync(n, d, edges, rel, dom)
    assert np.array_equal(r["dom"], dom) and r["iters"] == 1 and r["status"] == 0
    assert len(brute.solutions(n, d, edges, rel, dom)) == 0


# --------------------------------------------------------------------------
# invariants on larger random instances
# --------------------------------------------------------------------------

MEDIUM = [(s, 8 + s % 23, 3 + s % 6, [0.2, 0.5, 1.0][s % 3], [0.4, 0.55, 0.7][s % 3])
          for s in range(24)]


def _medium(s, n, d, p1, p2):
    inst = gen.model_b(500 + s, n, d, p1, p2)
    dom = masks_to_u8(gen.preremove(600 + s, n, d, (n * d) // 5), d)
    return inst.edges, inst.rel_u8(), dom


@pytest.mark.parametrize("s,n,d,p1,p2", MEDIUM)
def test_invariants(s, n, d, p1, p2):
    edges, rel, dom = _medium(s, n, d, p1, p2)
    dac, status, _, _ = oracle.ac3(n, d, edges, rel, dom)
    assert (dac <= dom).all()
    assert oracle.is_ac(n, d, edges, rel, dac)
    # idempotent, and a second enforcement takes one step
    again, _, _, _ = oracle.ac3(n, d, edges, rel, dac)
    assert np.array_equal(again, dac)
    assert oracle.rac_sync(n, d, edges, rel, dac)["iters"] == 1
    # the recurrence reaches the same closure; Proposition 1's bound holds
    r = oracle.rac_sync(n, d, edges, rel, dom, trace=True)
    assert np.array_equal(r["dom"], dac) and r["status"] == status
    assert r["iters"] <= int(dom.sum()) + 1
    # steps only remove, never below D_ac (Proposition 1 (1))
    prev = dom
    for step in r["trace"]:
        assert (step <= prev).all() and (step >= dac).all()
        prev = step
    # Proposition 2: restricting each step to the changed variables changes nothing
    r_full = oracle.rac_sync(n, d, edges, rel, dom, incremental=False, trace=True)
    assert np.array_equal(r_full["trace"], r["trace"]) and r_full["iters"] == r["iters"]
    # restart from any intermediate step
    for k in range(1, r["iters"]):
        rk = oracle.rac_sync(n, d, edges, rel, r["trace"][k - 1])
        assert rk["iters"] == r["iters"] - k and np.array_equal(rk["dom"], dac)
    # monotone: a smaller D gives a smaller closure
    sub = dom.copy()
    sub[:, 0] = 0
    dsub, _, _, _ = oracle.ac3(n, d, edges, rel, sub)
    assert (dsub <= dac).all()
    # stop-on-wipe-out stops at the first step that empties a domain
    r1 = oracle.rac_sync(n, d, edges, rel, dom, mode=oracle.STOP_ON_WIPEOUT)
    if status == 0:
        assert r1["iters"] == r["iters"] and np.array_equal(r1["dom"], dac)
    else:
        first = next(k for k, st in enumerate(r["trace"], 1) if (st.sum(axis=1) == 0).any())
        assert r1["iters"] == first and r1["status"] == 1
        assert np.array_equal(r1["dom"], r["trace"][first - 1])


def test_incremental_start_from_changed_variables():
    # Algorithm 2 calls tensorAC(Vars, [idx]) after assigning idx in an arc-
    # consistent state; starting from @changed = [idx] equals a full start.
    inst = gen.model_b(77, 40, 6, 0.3, 0.45)
    n, d = 40, 6
    rel = inst.rel_u8()
    base, status, _, _ = oracle.ac3(n, d, inst.edges, rel, np.ones((n, d), np.uint8))
    assert status == 0
    for x in range(0, n, 7):
        vals = np.nonzero(base[x])[0]
        st = base.copy()
        st[x] = 0
        st[x, vals[-1]] = 1
        full = oracle.rac_sync(n, d, inst.edges, rel, st, trace=True)
        inc = oracle.rac_sync(n, d, inst.edges, rel, st, changed0=[x], trace=True)
        assert np.array_equal(full["dom"], inc["dom"])
        assert full["iters"] == inc["iters"]
        assert np.array_equal(full["trace"], inc["trace"])


def test_support_check_count():
    # With every variable changed and nothing removed, one step checks every
    # arc once: 2m arcs of d*d cells.
    inst = gen.model_b(1, 50, 10, 0.5, 0.0)
    r = oracle.rac_sync(50, 10, inst.edges, inst.rel_u8(), np.ones((50, 10), np.uint8))
    assert r["iters"] == 1 and r["checks"] == 2 * inst.m * 100
    # Equality chain: step 1 checks all 2L arcs; step k>=2 checks only the arcs
    # into x_{k-1} (the one variable that changed), i.e. deg(x_{k-1}) arcs.
    L, d = 6, 3
    edges, rel = chain(L, d, lambda a, b: a == b)
    dom = np.ones((L + 1, d), np.uint8)
    dom[0] = [0, 1, 0]
    r = oracle.rac_sync(L + 1, d, edges, rel, dom)
    deg = [1] + [2] * (L - 1) + [1]
    expect = 2 * L + sum(deg[k - 1] for k in range(2, L + 2))
    assert r["iters"] == L + 1 and r["checks"] == expect * d * d


def test_max_steps_cap_reports_not_converged():
    L, d = 8, 10
    edges, rel = chain(L, d, lambda a, b: a < b)
    dom = np.ones((L + 1, d), np.uint8)
    r = oracle.rac_sync(L + 1, d, edges, rel, dom, max_steps=3, trace=True)
    assert not r["converged"] and r["iters"] == 3
    full = oracle.rac_sync(L + 1, d, edges, rel, dom, trace=True)
    assert np.array_equal(r["dom"], full["trace"][2])
