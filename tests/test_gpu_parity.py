"""GPU parity: every result of the HIP paths equals the CPU oracle bit for bit
(domains, step count, wipe-out status and support-check count), on the tiny,
golden and medium instances, for the bit-row, int8-row and fused (one
workgroup per state, every step in one launch) paths, both stop modes, forced
item splitting, graph and direct launches, incremental starts, the step cap,
batched states and groups of networks."""
import sys

import numpy as np
import pytest

import oracle
from paper_2407_11388_amd import gen

from helpers import (golden_cases, golden_instance, masks_to_u8, oracle_expect, u8_to_masks)

pytestmark = pytest.mark.gpu

rac = pytest.importorskip("paper_2407_11388_amd.rac")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_vs_oracle(name, n, d, edges, rel_u8, dom_masks, path, mode=0, item_bytes=0,
                  use_graph=True, changed=None):
    say(f"[gpu] {name} n={n} d={d} m={len(edges)} path={path} mode={mode} "
        f"item_bytes={item_bytes} graph={use_graph}")
    net = rac.Net.from_u8(n, d, edges, rel_u8, path=path, mode=mode, item_bytes=item_bytes,
                          use_graph=use_graph)
    got, iters, status = net.enforce(dom_masks, changed=changed)
    st = net.stats()
    exp, e_iters, e_status, e_checks, _ = oracle_expect(n, d, edges, rel_u8, dom_masks, mode,
                                                        changed)
    assert np.array_equal(got, exp), f"{name}: domains differ"
    assert iters == e_iters, f"{name}: iters {iters} != {e_iters}"
    assert status == e_status
    assert st.support_checks == e_checks, f"{name}: checks {st.support_checks} != {e_checks}"
    net.close()


PATHS = [rac.PATH_BITS, rac.PATH_INT8, rac.PATH_FUSED]
CASES = golden_cases()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden(case, mode, path):
    n, d, edges, rel, dom = golden_instance(case)
    gpu_vs_oracle(case["name"], n, d, edges, rel, u8_to_masks(dom), path, mode)


def _tiny(seed):
    n = 2 + seed % 6
    d = 1 + (seed // 6) % 6
    p1 = [0.4, 0.7, 1.0][seed % 3]
    p2 = [0.2, 0.45, 0.7][(seed // 3) % 3]
    keep = [1.0, 0.75][(seed // 9) % 2]
    inst, dom = gen.random_tiny(5000 + seed, n, d, p1, p2, keep)
    return inst, dom


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", range(0, 72, 3))
def test_tiny_random(seed, path):
    inst, dom = _tiny(seed)
    for mode in (0, 1):
        gpu_vs_oracle(f"tiny{seed}", inst.n, inst.d, inst.edges, inst.rel_u8(), dom, path, mode)


MEDIUM_D = [1, 3, 4, 5, 10, 17, 20, 31, 32, 33, 40, 63, 64]


@pytest.mark.parametrize("d", MEDIUM_D)
@pytest.mark.parametrize("item_bytes", [0, 256])
def test_medium_bits(d, item_bytes):
    n = 60
    p2 = 0.5 if d <= 4 else (0.62 if d <= 12 else 0.8)
    inst = gen.model_b(900 + d, n, d, 0.35, p2)
    dom = gen.preremove(901 + d, n, d, (n * d) // 6)
    for mode in (0, 1):
        gpu_vs_oracle(f"medium-d{d}", n, d, inst.edges, inst.rel_u8(), dom, rac.PATH_BITS, mode,
                      item_bytes=item_bytes, use_graph=(d % 2 == 0))


@pytest.mark.parametrize("d", MEDIUM_D)
def test_medium_fused(d):
    n = 60
    p2 = 0.5 if d <= 4 else (0.62 if d <= 12 else 0.8)
    inst = gen.model_b(900 + d, n, d, 0.35, p2)
    dom = gen.preremove(901 + d, n, d, (n * d) // 6)
    for mode in (0, 1):
        gpu_vs_oracle(f"medium-fused-d{d}", n, d, inst.edges, inst.rel_u8(), dom, rac.PATH_FUSED,
                      mode)


@pytest.mark.parametrize("d", [d for d in MEDIUM_D if d <= 32])
def test_medium_int8(d):
    n = 50
    p2 = 0.5 if d <= 4 else (0.62 if d <= 12 else 0.8)
    inst = gen.model_b(700 + d, n, d, 0.4, p2)
    dom = gen.preremove(701 + d, n, d, (n * d) // 5)
    for mode in (0, 1):
        for ib in (0, 512):
            gpu_vs_oracle(f"medium-int8-d{d}", n, d, inst.edges, inst.rel_u8(), dom,
                          rac.PATH_INT8, mode, item_bytes=ib)


@pytest.mark.parametrize("path", [rac.PATH_BITS, rac.PATH_FUSED])
def test_incremental_start(path):
    n, d = 80, 8
    inst = gen.model_b(31, n, d, 0.2, 0.45)
    rel = inst.rel_u8()
    base, status, _, _ = oracle.ac3(n, d, inst.edges, rel, np.ones((n, d), np.uint8))
    assert status == 0
    for x in range(0, n, 11):
        st = base.copy()
        vals = np.nonzero(st[x])[0]
        st[x] = 0
        st[x, vals[0]] = 1
        gpu_vs_oracle(f"incremental-x{x}", n, d, inst.edges, rel, u8_to_masks(st),
                      path, 0, changed=[x])


@pytest.mark.parametrize("path", [rac.PATH_BITS, rac.PATH_FUSED])
def test_step_cap_reports_not_converged(path):
    L, d = 9, 12
    allowed = [(a, b) for a in range(d) for b in range(d) if a < b]
    edges = np.array([[i, i + 1] for i in range(L)], np.int32)
    rel = np.zeros((L, d, d), np.uint8)
    for a, b in allowed:
        rel[:, a, b] = 1
    dom = np.full(L + 1, (1 << d) - 1, np.uint64)
    say(f"[gpu] step cap path={path}")
    net = rac.Net.from_u8(L + 1, d, edges, rel, max_sweeps=4, path=path)
    with pytest.raises(rac.RacError) as ei:
        net.enforce(dom)
    assert ei.value.code == rac.RAC_ENOTCONVERGED
    net.close()
    # resume: the full run equals a capped run then a second run
    net = rac.Net.from_u8(L + 1, d, edges, rel, path=path)
    full, it_full, _ = net.enforce(dom)
    exp = oracle.rac_sync(L + 1, d, edges, rel, masks_to_u8(dom, d), trace=True)
    mid = u8_to_masks(exp["trace"][3])
    rest, it_rest, _ = net.enforce(mid)
    assert np.array_equal(full, rest) and it_full == 4 + it_rest == L + 1
    net.close()


@pytest.mark.parametrize("path,use_graph", [(rac.PATH_BITS, True), (rac.PATH_BITS, False),
                                            (rac.PATH_FUSED, True)])
def test_batch_states_bits(use_graph, path):
    n, d, B = 40, 6, 37
    inst = gen.model_b(12, n, d, 0.5, 0.4)
    doms, _ = gen.partial_assign_states(13, n, d, B, 8)
    rel = inst.rel_u8()
    say(f"[gpu] batch path={path} B={B} graph={use_graph}")
    net = rac.Net.from_u8(n, d, inst.edges, rel, path=path, use_graph=use_graph)
    for rep in range(2):
        got, iters, status = net.enforce_batch(doms)
        total_checks = 0
        for s in range(B):
            exp, e_it, e_st, e_ch, _ = oracle_expect(n, d, inst.edges, rel, doms[s])
            assert np.array_equal(got[s], exp), f"state {s}"
            assert iters[s] == e_it and status[s] == e_st
            total_checks += e_ch
        assert net.stats().support_checks == total_checks
    net.close()


@pytest.mark.parametrize("path,use_graph", [(rac.PATH_AUTO, True), (rac.PATH_AUTO, False),
                                            (rac.PATH_FUSED, True)])
def test_group_of_networks(use_graph, path):
    rng = np.random.default_rng(5)
    nets, doms, insts = [], [], []
    for i in range(23):
        n = int(rng.integers(2, 70))
        d = int(rng.integers(1, 65))
        inst = gen.model_b(100 + i, n, d, float(rng.uniform(0.1, 1.0)), float(rng.uniform(0.1, 0.8)))
        insts.append(inst)
        nets.append(rac.Net.from_instance(inst))
        doms.append(gen.preremove(200 + i, n, d, (n * d) // 7))
    say(f"[gpu] group k={len(nets)} path={path} graph={use_graph}")
    grp = rac.Group(nets, use_graph=use_graph, path=path)
    for rep in range(2):
        outs, iters, status = grp.enforce(doms)
        if path == rac.PATH_AUTO:
            # the first call measured the work-item size of the later steps
            st = grp.stats()
            assert st.tune_source == 3 and st.item_bytes >= 16 << 10
        for i, inst in enumerate(insts):
            exp, e_it, e_st, _, _ = oracle_expect(inst.n, inst.d, inst.edges, inst.rel_u8(), doms[i])
            assert np.array_equal(outs[i], exp), f"instance {i}"
            assert iters[i] == e_it and status[i] == e_st
    outs2, it2, st2 = rac.enforce_multi(nets, doms)
    for i in range(len(nets)):
        assert np.array_equal(outs2[i], outs[i]) and it2[i] == iters[i]
    grp.close()
    for n_ in nets:
        n_.close()


@pytest.mark.parametrize("ratio", ["0", "1"])
def test_scan_and_changed_variable_steps(ratio, monkeypatch):
    # Steps k >= 2 of the bit-row path either scan every group for arcs into
    # changed variables, or walk the changed variables' own arcs (reverse-arc
    # table). RAC_PUSH_RATIO 0 forces the scan, 1 the changed-variable walk;
    # both must give the oracle's results, uint32 and uint64 rows alike.
    monkeypatch.setenv("RAC_PUSH_RATIO", ratio)
    for seed in range(1, 72, 5):
        inst, dom = _tiny(seed)
        for mode in (0, 1):
            gpu_vs_oracle(f"tiny{seed}-r{ratio}", inst.n, inst.d, inst.edges, inst.rel_u8(), dom,
                          rac.PATH_BITS, mode)
    for d in (3, 32, 33, 64):
        test_medium_bits(d, 0)
    test_incremental_start(rac.PATH_BITS)
    test_batch_states_bits(True, rac.PATH_BITS)
    test_group_of_networks(True, rac.PATH_AUTO)


@pytest.mark.parametrize("path", [rac.PATH_BITS, rac.PATH_FUSED])
def test_empty_domains_and_isolated_variables(path):
    n, d = 7, 5
    edges = np.array([[0, 1], [1, 2], [4, 5]], np.int32)
    rel = np.ones((3, d, d), np.uint8)
    dom = np.array([31, 31, 31, 0, 31, 0, 31], np.uint64)   # x3 isolated & empty, x5 empty
    for mode in (0, 1):
        gpu_vs_oracle("empty-isolated", n, d, edges, rel, dom, path, mode)
    # no constraints at all
    gpu_vs_oracle("no-edges", n, d, np.zeros((0, 2), np.int32), np.zeros((0, d, d), np.uint8),
                  dom, path, 0)


def test_dense_create_matches():
    inst = gen.model_b(3, 12, 5, 0.5, 0.5)
    n, d = 12, 5
    u8 = inst.rel_u8()
    R = np.zeros((n, d, n, d), np.uint8)
    for e, (x, y) in enumerate(inst.edges):
        R[x, :, y, :] = u8[e]
        R[y, :, x, :] = u8[e].T
    dom = gen.full_domains(n, d)
    say("[gpu] dense create")
    a = rac.Net.from_dense(n, d, R, inst.edges).enforce(dom)
    b = rac.Net.from_bits(n, d, inst.edges, inst.rel).enforce(dom)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


MFMA_CASES = [(40, 32, 37, 0.6, 0.3), (45, 10, 130, 0.8, 0.5), (13, 4, 300, 1.0, 0.55),
              (70, 17, 129, 0.4, 0.7), (9, 1, 64, 0.9, 0.0), (100, 32, 257, 0.8, 0.25),
              # more than 64 blocks of 8 neighbours: the step kernel's
              # lane tables of unit descriptors come in chunks of 64 blocks
              (2200, 6, 33, 0.006, 0.35), (2100, 32, 20, 0.004, 0.35)]


@pytest.mark.parametrize("handoff", ["0", "32", "100000"])
@pytest.mark.parametrize("n,d,B,p1,p2", MFMA_CASES)
def test_batch_states_mfma(n, d, B, p1, p2, handoff, monkeypatch):
    # handoff: states left when the rest moves to the bit-row path
    # (0: never; 100000: right after the first matrix-core steps)
    monkeypatch.setenv("RAC_MFMA_HANDOFF", handoff)
    inst = gen.model_b(40 + n + d, n, d, p1, p2)
    doms, _ = gen.partial_assign_states(41 + B, n, d, B, min(n, 12))
    rel = inst.rel_u8()
    for mode in (0, 1):
        say(f"[gpu] batch mfma n={n} d={d} B={B} mode={mode} handoff={handoff}")
        net = rac.Net.from_u8(n, d, inst.edges, rel, path=rac.PATH_MFMA, mode=mode)
        for rep in range(2):
            got, iters, status = net.enforce_batch(doms)
            st = net.stats()
            assert st.path == rac.PATH_MFMA
            total_checks = 0
            for s in range(B):
                exp, e_it, e_st, e_ch, _ = oracle_expect(n, d, inst.edges, rel, doms[s], mode)
                assert np.array_equal(got[s], exp), f"state {s} (mode {mode})"
                assert iters[s] == e_it, f"state {s}: iters {iters[s]} != {e_it}"
                assert status[s] == e_st
                total_checks += e_ch
            assert st.support_checks == total_checks
        net.close()


@pytest.mark.parametrize("n,d,B,p1,p2", [(45, 10, 130, 0.8, 0.5), (100, 32, 257, 0.8, 0.25),
                                         (70, 17, 129, 0.4, 0.7)])
def test_batch_states_mfma_handoff_state_by_state(n, d, B, p1, p2, monkeypatch):
    # The hand-off's bit-row steps normally read each group's rows once for
    # up to 16 states (revise_shared_kernel); RAC_SHARED_ROWS=0 revises the
    # handed-over states one by one. Both equal the oracle, with every state
    # handed over after the first matrix-core steps and with the default
    # threshold.
    monkeypatch.setenv("RAC_SHARED_ROWS", "0")
    for handoff in ("100000", "32"):
        test_batch_states_mfma(n, d, B, p1, p2, handoff, monkeypatch)


@pytest.mark.parametrize("segments", ["2", "3", "4"])
@pytest.mark.parametrize("n,d,B,p1,p2", [(45, 10, 130, 0.8, 0.5), (2200, 6, 33, 0.006, 0.35),
                                         (100, 32, 257, 0.8, 0.25)])
def test_batch_states_mfma_split_steps(n, d, B, p1, p2, segments, monkeypatch):
    # every step's neighbour blocks split over 2-4 workgroups per tile (the
    # segments cross the 64-block chunks of the lane tables for n = 2200)
    monkeypatch.setenv("RAC_MFMA_SEGMENTS", segments)
    monkeypatch.setenv("RAC_MFMA_HANDOFF", "0")
    inst = gen.model_b(40 + n + d, n, d, p1, p2)
    doms, _ = gen.partial_assign_states(41 + B, n, d, B, min(n, 12))
    rel = inst.rel_u8()
    say(f"[gpu] batch mfma split={segments} n={n} d={d} B={B}")
    net = rac.Net.from_u8(n, d, inst.edges, rel, path=rac.PATH_MFMA)
    got, iters, status = net.enforce_batch(doms)
    for s in range(B):
        exp, e_it, e_st, _, _ = oracle_expect(n, d, inst.edges, rel, doms[s])
        assert np.array_equal(got[s], exp), f"state {s}"
        assert iters[s] == e_it and status[s] == e_st, f"state {s}"
    net.close()


def test_random_shapes_bits_int8_fused(monkeypatch):
    # Seeded random shapes on the bit, int8 and fused paths (n 10..399, d up
    # to 64 on bit rows and 32 otherwise, one state or a batch, both modes,
    # the sparse-step ratio varied); every state against the oracle.
    rng = np.random.default_rng(2025)
    for c in range(30):
        path = int(rng.choice([rac.PATH_BITS, rac.PATH_INT8, rac.PATH_FUSED]))
        n = int(rng.integers(10, 400))
        d = int(rng.integers(1, 65 if path == rac.PATH_BITS else 33))
        B = int(rng.integers(1, 80))
        p1, p2 = float(rng.uniform(0.02, 1.0)), float(rng.uniform(0.05, 0.7))
        mode = int(rng.integers(0, 2))
        push = str(rng.choice(["16", "0", "4", "64"]))
        monkeypatch.setenv("RAC_PUSH_RATIO", push)
        inst = gen.model_b(3000 + c, n, d, p1, p2)
        doms, _ = gen.partial_assign_states(4000 + c, n, d, B, min(n, int(rng.integers(0, 20))))
        rel = inst.rel_u8()
        say(f"[gpu] random {c}: path={path} n={n} d={d} B={B} p1={p1:.2f} p2={p2:.2f} "
            f"mode={mode} push={push}")
        net = rac.Net.from_u8(n, d, inst.edges, rel, path=path, mode=mode)
        if B == 1 or c % 3 == 0:
            one, it, st = net.enforce(doms[0])
            got, iters, status, B = one[None], np.array([it]), np.array([st]), 1
        else:
            got, iters, status = net.enforce_batch(doms)
        net.close()
        for s in range(B):
            exp, e_it, e_st, _, _ = oracle_expect(n, d, inst.edges, rel, doms[s], mode)
            assert np.array_equal(got[s], exp), f"case {c} state {s}"
            assert iters[s] == e_it and status[s] == e_st, f"case {c} state {s}"


def test_random_groups_with_member_calls():
    # Seeded random groups (2..23 uneven networks, d up to 64), each enforced
    # twice with a single-state call on one member net in between (the member
    # rebuilds its own work items; the group keeps its tables); everything
    # against the oracle.
    rng = np.random.default_rng(2026)
    for c in range(8):
        k = int(rng.integers(2, 24))
        insts, doms = [], []
        for i in range(k):
            n, d = int(rng.integers(10, 300)), int(rng.integers(2, 65))
            inst = gen.model_b(5000 + 100 * c + i, n, d, float(rng.uniform(0.05, 1.0)),
                               float(rng.uniform(0.05, 0.6)))
            dd, _ = gen.partial_assign_states(6000 + 100 * c + i, n, d, 1,
                                              min(n, int(rng.integers(0, 15))))
            insts.append(inst)
            doms.append(dd[0])
        say(f"[gpu] random group {c}: {k} nets")
        nets = [rac.Net.from_instance(i) for i in insts]
        exps = [oracle_expect(i.n, i.d, i.edges, i.rel_u8(), doms[j])[:3] for j, i in enumerate(insts)]
        grp = rac.Group(nets)
        for rep in range(2):
            got, iters, status = grp.enforce(doms)
            for j, (exp, e_it, e_st) in enumerate(exps):
                assert np.array_equal(got[j], exp), f"group {c} rep {rep} net {j}"
                assert iters[j] == e_it and status[j] == e_st, f"group {c} rep {rep} net {j}"
            j = int(rng.integers(0, k))
            one, it, st = nets[j].enforce(doms[j])
            assert np.array_equal(one, exps[j][0]) and (it, st) == exps[j][1:], f"net {j}"
        grp.close()
        for nt in nets:
            nt.close()


def test_batch_states_mfma_random_shapes(monkeypatch):
    # Seeded random shapes on the matrix-core path (n 8..319, d 2..32, B
    # 1..299, density and tightness across their range), each with a random
    # hand-off, forced split, Proposition 2 skip setting and mode; every
    # state against the oracle. Odd block counts, partial superblocks and
    # partial state tiles all occur.
    rng = np.random.default_rng(2024)
    for c in range(24):
        n = int(rng.integers(8, 320))
        d = int(rng.integers(2, 33))
        B = int(rng.integers(1, 300))
        p1, p2 = float(rng.uniform(0.05, 1.0)), float(rng.uniform(0.05, 0.6))
        mode = int(rng.integers(0, 2))
        handoff = str(rng.choice(["0", "32", "100000"]))
        seg = str(rng.choice(["0", "0", "2", "3", "4"]))
        skip = str(rng.choice(["1", "1", "0"]))
        monkeypatch.setenv("RAC_MFMA_HANDOFF", handoff)
        monkeypatch.setenv("RAC_MFMA_SEGMENTS", seg)
        monkeypatch.setenv("RAC_MFMA_SKIP", skip)
        inst = gen.model_b(1000 + c, n, d, p1, p2)
        doms, _ = gen.partial_assign_states(2000 + c, n, d, B, min(n, int(rng.integers(0, 25))))
        rel = inst.rel_u8()
        say(f"[gpu] batch mfma random {c}: n={n} d={d} B={B} p1={p1:.2f} p2={p2:.2f} "
            f"mode={mode} handoff={handoff} seg={seg} skip={skip}")
        net = rac.Net.from_u8(n, d, inst.edges, rel, path=rac.PATH_MFMA, mode=mode)
        got, iters, status = net.enforce_batch(doms)
        net.close()
        for s in range(B):
            exp, e_it, e_st, _, _ = oracle_expect(n, d, inst.edges, rel, doms[s], mode)
            assert np.array_equal(got[s], exp), f"case {c} state {s}"
            assert iters[s] == e_it and status[s] == e_st, f"case {c} state {s}"


def frontier_states(inst, doms, seed):
    """States one removal away from arc consistency: the closure of each
    state (the oracle's), then one value of one variable with at least two
    values removed (a search node just after its branching decision). After
    the first step only a few variables change."""
    import oracle
    rng = np.random.default_rng(seed)
    rel = inst.rel_u8()
    out = []
    for s in range(doms.shape[0]):
        dac, status, _, _ = oracle.ac3(inst.n, inst.d, inst.edges, rel, masks_to_u8(doms[s], inst.d))
        m = u8_to_masks(dac)
        if status == 0:
            sizes = np.array([bin(int(v)).count("1") for v in m])
            cand = np.flatnonzero(sizes >= 2)
            if len(cand):
                x = int(rng.choice(cand))
                m[x] &= ~(np.uint64(1) << np.uint64(int(m[x]).bit_length() - 1))
        out.append(m)
    return np.array(out, dtype=np.uint64)


@pytest.mark.parametrize("skip", ["0", "1"])
@pytest.mark.parametrize("n,d,B,p1,p2", [(100, 32, 130, 0.8, 0.25), (160, 12, 130, 0.5, 0.45),
                                         (2200, 6, 33, 0.006, 0.35)])
def test_batch_states_mfma_prop2_frontier(n, d, B, p1, p2, skip, monkeypatch):
    # Proposition 2 inside the matrix-core step: with skip=1 a tile of states
    # re-examines only the neighbour blocks some of its states changed in the
    # previous step; skip=0 re-examines every arc. Both must equal the oracle.
    monkeypatch.setenv("RAC_MFMA_SKIP", skip)
    monkeypatch.setenv("RAC_MFMA_HANDOFF", "0")
    inst = gen.model_b(50 + n + d, n, d, p1, p2)
    doms, _ = gen.partial_assign_states(51 + B, n, d, B, min(n, 12))
    doms = frontier_states(inst, doms, 52 + n)
    rel = inst.rel_u8()
    say(f"[gpu] batch mfma frontier skip={skip} n={n} d={d} B={B}")
    for mode in (0, 1):
        net = rac.Net.from_u8(n, d, inst.edges, rel, path=rac.PATH_MFMA, mode=mode)
        got, iters, status = net.enforce_batch(doms)
        st = net.stats()
        assert st.path == rac.PATH_MFMA
        total = 0
        for s in range(B):
            exp, e_it, e_st, e_ch, _ = oracle_expect(n, d, inst.edges, rel, doms[s], mode)
            assert np.array_equal(got[s], exp), f"state {s} (mode {mode})"
            assert iters[s] == e_it and status[s] == e_st, f"state {s} (mode {mode})"
            total += e_ch
        assert st.support_checks == total
        # the matrix-core work counts only re-examined arcs: step 1 every arc
        # of every state, later steps at most every arc of the active states
        assert 2 * d * d * inst.m * 2 * B <= st.algo_ops <= 2 * d * d * 2 * inst.m * int(iters.sum())
        net.close()


def test_mfma_rejects_wide_domains():
    inst = gen.model_b(3, 10, 40, 0.5, 0.3)
    net = rac.Net.from_instance(inst, path=rac.PATH_MFMA)
    doms = np.tile(gen.full_domains(10, 40), (4, 1))
    with pytest.raises(rac.RacError) as ei:
        net.enforce_batch(doms)
    assert ei.value.code == rac.RAC_EUNSUPPORTED
    net.close()


def test_mfma_step_cap():
    L, d = 9, 12
    edges = np.array([[i, i + 1] for i in range(L)], np.int32)
    rel = np.zeros((L, d, d), np.uint8)
    for a in range(d):
        rel[:, a, a + 1:] = 1
    doms = np.tile(np.full(L + 1, (1 << d) - 1, np.uint64), (3, 1))
    net = rac.Net.from_u8(L + 1, d, edges, rel, path=rac.PATH_MFMA, max_sweeps=4)
    with pytest.raises(rac.RacError) as ei:
        net.enforce_batch(doms)
    assert ei.value.code == rac.RAC_ENOTCONVERGED
    net.close()


@pytest.mark.parametrize("path", [rac.PATH_BITS, rac.PATH_MFMA, rac.PATH_FUSED])
def test_batch_device_entry_point_matches_host(path):
    torch = pytest.importorskip("torch")
    n, d, B = 60, 32, 200
    inst = gen.model_b(7, n, d, 0.7, 0.3)
    doms, _ = gen.partial_assign_states(8, n, d, B, 10)
    say(f"[gpu] device entry point path={path}")
    net = rac.Net.from_instance(inst, path=path)
    h_dom, h_it, h_st = net.enforce_batch(doms)
    dev = torch.device("cuda:0")
    d_in = torch.from_numpy(doms.view(np.int64)).to(dev)
    d_out = torch.zeros_like(d_in)
    d_it = torch.zeros(B, dtype=torch.int32, device=dev)
    d_st = torch.zeros(B, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(2):
        net.enforce_batch_device(d_in, d_out, d_it, d_st, stream)
        net.sync()
        torch.cuda.synchronize()
        assert np.array_equal(d_out.cpu().numpy().view(np.uint64), h_dom)
        assert np.array_equal(d_it.cpu().numpy(), h_it)
        assert np.array_equal(d_st.cpu().numpy(), h_st)
    assert np.array_equal(d_in.cpu().numpy().view(np.uint64), doms)   # input untouched
    net.close()


def test_group_keeps_its_own_item_tables():
    # A group builds its own work-item tables for its item size. Calls on a
    # member net that rebuild the net's tables for another size (here the
    # default size of one state, against the group's 512 bytes) must leave the
    # group's launches reading valid tables.
    insts, doms, nets = [], [], []
    for i in range(6):
        n, d = 50 + 7 * i, [5, 12, 32, 33, 64, 20][i]
        inst = gen.model_b(300 + i, n, d, 0.5, 0.45 if d < 12 else 0.8)
        insts.append(inst)
        doms.append(gen.preremove(310 + i, n, d, (n * d) // 6))
        nets.append(rac.Net.from_instance(inst))
    say("[gpu] group item tables vs calls on member nets")
    grp = rac.Group(nets, item_bytes=512)
    for rep in range(3):
        for i, net in enumerate(nets):
            got, it, stt = net.enforce(doms[i])
            exp, e_it, e_st, _, _ = oracle_expect(insts[i].n, insts[i].d, insts[i].edges,
                                                  insts[i].rel_u8(), doms[i])
            assert np.array_equal(got, exp) and it == e_it and stt == e_st
        outs, iters, status = grp.enforce(doms)
        for i, inst in enumerate(insts):
            exp, e_it, e_st, _, _ = oracle_expect(inst.n, inst.d, inst.edges, inst.rel_u8(), doms[i])
            assert np.array_equal(outs[i], exp), f"call {rep}, instance {i}"
            assert iters[i] == e_it and status[i] == e_st
    grp.close()
    for net in nets:
        net.close()


@pytest.mark.parametrize("path", [rac.PATH_BITS, rac.PATH_MFMA, rac.PATH_FUSED])
def test_host_call_after_device_call(path):
    # A host-pointer call made while a device-pointer call on the same net is
    # still in flight (no sync in between) waits for it before reusing the
    # net's workspace; both results equal the oracle's.
    torch = pytest.importorskip("torch")
    n, d, B = 60, 16, 96
    inst = gen.model_b(17, n, d, 0.7, 0.45)
    rel = inst.rel_u8()
    doms, _ = gen.partial_assign_states(18, n, d, B, 8)
    dev = torch.device("cuda:0")
    net = rac.Net.from_instance(inst, path=path)
    d_in = torch.from_numpy(doms.view(np.int64)).to(dev)
    d_out = torch.zeros_like(d_in)
    d_it = torch.zeros(B, dtype=torch.int32, device=dev)
    d_st = torch.zeros(B, dtype=torch.int32, device=dev)
    say(f"[gpu] host call after device call path={path}")
    for rep in range(2):
        net.enforce_batch_device(d_in, d_out, d_it, d_st, torch.cuda.current_stream().cuda_stream)
        got1, it1, st1 = net.enforce(doms[rep])
        got2, it2, st2 = net.enforce_batch(doms[:5])
        torch.cuda.synchronize()
        res = d_out.cpu().numpy().view(np.uint64)
        its, sts = d_it.cpu().numpy(), d_st.cpu().numpy()
        for s in range(B):
            exp, e_it, e_st, _, _ = oracle_expect(n, d, inst.edges, rel, doms[s])
            assert np.array_equal(res[s], exp) and its[s] == e_it and sts[s] == e_st, f"state {s}"
            if s == rep:
                assert np.array_equal(got1, exp) and it1 == e_it and st1 == e_st
            if s < 5:
                assert np.array_equal(got2[s], exp) and it2[s] == e_it and st2[s] == e_st
    net.close()


@pytest.mark.parametrize("n", [rac.SMALL_MAX_N, rac.SMALL_MAX_N + 1])
def test_fused_size_limit(n):
    # The fused path holds a state of at most SMALL_MAX_N variables in LDS:
    # at the limit it equals the oracle (a sparse network with a few
    # hundred groups), one variable more is refused with RAC_EUNSUPPORTED.
    d = 6
    inst = gen.model_b(41, n, d, 3.0 / n, 0.5)
    dom = gen.preremove(42, n, d, n // 2)
    if n > rac.SMALL_MAX_N:
        say(f"[gpu] fused refuses n={n}")
        net = rac.Net.from_instance(inst, path=rac.PATH_FUSED)
        with pytest.raises(rac.RacError) as ei:
            net.enforce(dom)
        assert ei.value.code == rac.RAC_EUNSUPPORTED
        net.close()
        return
    for mode in (0, 1):
        gpu_vs_oracle(f"fused-n{n}", n, d, inst.edges, inst.rel_u8(), dom, rac.PATH_FUSED, mode)


def test_fused_dense_multi_group_variables():
    # Variables with several 64-arc groups (degree up to 119) and uint64 rows:
    # every wave of the workgroup takes groups of one variable, their failures
    # meet in the LDS word of the variable.
    for n, d, p2 in ((120, 10, 0.55), (120, 40, 0.85), (90, 64, 0.9)):
        inst = gen.model_b(50 + d, n, d, 1.0, p2)
        dom = gen.preremove(51 + d, n, d, (n * d) // 8)
        for mode in (0, 1):
            gpu_vs_oracle(f"fused-dense-d{d}", n, d, inst.edges, inst.rel_u8(), dom,
                          rac.PATH_FUSED, mode)
