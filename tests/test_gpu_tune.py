"""The autotuner: a shape not in the table is measured on the call's own
inputs (every candidate path and work-item size, which give identical
results) and the fastest is stored in the table file; later calls of the
shape reuse it. Results are checked against the oracle; every candidate is
also forced directly (path, work-item size, matrix-core hand-off)."""
import os
import sys

import numpy as np
import pytest

from paper_2407_11388_amd import gen

from helpers import oracle_expect

pytestmark = pytest.mark.gpu

rac = pytest.importorskip("paper_2407_11388_amd.rac")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def table_lines(kind):
    path = os.environ["RAC_TUNE_CACHE"]
    with open(path) as f:
        return [ln.split() for ln in f if ln.startswith(f"gfx950/{kind}/")]


def check_states(inst, doms, got, iters, status, mode=0):
    rel = inst.rel_u8()
    for s in range(doms.shape[0]):
        exp, e_it, e_st, _, _ = oracle_expect(inst.n, inst.d, inst.edges, rel, doms[s], mode)
        assert np.array_equal(got[s], exp), f"state {s}"
        assert iters[s] == e_it and status[s] == e_st, f"state {s}"


@pytest.mark.parametrize("n,d,p1,p2,B", [(120, 24, 0.6, 0.3, 96), (90, 40, 0.5, 0.2, 40)])
def test_batch_tuner_measures_then_reuses(n, d, p1, p2, B):
    inst = gen.model_b(300 + n + d, n, d, p1, p2)
    doms, _ = gen.partial_assign_states(301 + B, n, d, B, 10)
    before = len(table_lines("batch"))
    say(f"[gpu] tuner: batch n={n} d={d} B={B}, measured")
    net = rac.Net.from_instance(inst, tune=rac.TUNE_MEASURE)
    got, iters, status = net.enforce_batch(doms)
    st = net.stats()
    assert st.tune_source == 3 and st.path in (rac.PATH_BITS, rac.PATH_INT8, rac.PATH_MFMA,
                                               rac.PATH_FUSED)
    check_states(inst, doms, got, iters, status)
    lines = table_lines("batch")
    assert len(lines) == before + 1 and lines[-1][1] == f"path={st.path}"
    net.close()
    say("[gpu] tuner: the same shape again, from the table")
    net2 = rac.Net.from_instance(inst)
    got2, it2, st2 = net2.enforce_batch(doms)
    s2 = net2.stats()
    assert s2.tune_source == 2 and s2.path == st.path
    assert np.array_equal(got2, got) and np.array_equal(it2, iters) and np.array_equal(st2, status)
    net2.close()


def test_single_tuner_measures_then_reuses():
    inst = gen.model_b(310, 150, 20, 0.4, 0.35)
    dom = gen.preremove(311, 150, 20, 200)
    say("[gpu] tuner: single state, measured")
    net = rac.Net.from_instance(inst, tune=rac.TUNE_MEASURE)
    got, it, status = net.enforce(dom)
    assert net.stats().tune_source == 3
    exp, e_it, e_st, _, _ = oracle_expect(inst.n, inst.d, inst.edges, inst.rel_u8(), dom)
    assert np.array_equal(got, exp) and (it, status) == (e_it, e_st)
    net.close()
    net2 = rac.Net.from_instance(inst)
    got2, it2, st2 = net2.enforce(dom)
    assert net2.stats().tune_source == 2
    assert np.array_equal(got2, exp) and (it2, st2) == (e_it, e_st)
    net2.close()


@pytest.mark.parametrize("n,expect", [(64, rac.PATH_FUSED), (200, rac.PATH_MFMA)])
def test_rules_mode_does_not_measure(n, expect):
    # The fixed rules: many states of a network with at most 2 MiB of bit
    # rows (n=64: 64 groups of 4 KiB) take the fused path; of a larger dense
    # one with d <= 32 (n=200: 600 groups, 2.4 MiB), the matrix cores.
    inst = gen.model_b(320, n, 16, 0.7, 0.3)
    doms, _ = gen.partial_assign_states(321, n, 16, 70, 8)
    before = len(table_lines("batch"))
    net = rac.Net.from_instance(inst, tune=rac.TUNE_RULES)
    got, iters, status = net.enforce_batch(doms)
    st = net.stats()
    assert st.tune_source == 0 and st.path == expect
    assert len(table_lines("batch")) == before
    check_states(inst, doms, got, iters, status)
    net.close()


def test_capped_call_does_not_measure():
    # A call capped below the step bound is no sample of the shape's full
    # runs: it takes the fixed rules and stores nothing; the next uncapped
    # call of the shape is measured.
    inst = gen.model_b(330, 140, 12, 0.6, 0.3)
    doms, _ = gen.partial_assign_states(331, 140, 12, 72, 8)
    before = len(table_lines("batch"))
    say("[gpu] tuner: capped call, not measured")
    net = rac.Net.from_instance(inst, max_sweeps=1)
    try:
        net.enforce_batch(doms)
    except rac.RacError as e:
        assert e.code == rac.RAC_ENOTCONVERGED
    assert net.stats().tune_source == 0
    assert len(table_lines("batch")) == before
    net.close()
    say("[gpu] tuner: the same shape uncapped, measured")
    net2 = rac.Net.from_instance(inst)
    got, iters, status = net2.enforce_batch(doms)
    assert net2.stats().tune_source == 3
    assert len(table_lines("batch")) == before + 1
    check_states(inst, doms, got, iters, status)
    net2.close()


# every candidate the tuner can pick, forced: bit rows and int8 rows with
# small, default and large work items, the matrix cores with hand-off at 32
# states and never, the fused path
@pytest.mark.parametrize("path,item_bytes,handoff", [
    (rac.PATH_BITS, 4096, None), (rac.PATH_BITS, 0, None), (rac.PATH_BITS, 1 << 20, None),
    (rac.PATH_INT8, 0, None), (rac.PATH_INT8, 1 << 20, None),
    (rac.PATH_MFMA, 0, "32"), (rac.PATH_MFMA, 0, "0"), (rac.PATH_FUSED, 0, None)])
def test_tuner_candidates_forced(path, item_bytes, handoff, monkeypatch):
    if handoff is not None:
        monkeypatch.setenv("RAC_MFMA_HANDOFF", handoff)
    inst = gen.model_b(330, 200, 32, 0.5, 0.25)
    doms, _ = gen.partial_assign_states(331, 200, 32, 100, 12)
    say(f"[gpu] tuner candidate path={path} items={item_bytes} handoff={handoff}")
    net = rac.Net.from_instance(inst, path=path, item_bytes=item_bytes)
    got, iters, status = net.enforce_batch(doms)
    assert net.stats().path == path and net.stats().tune_source == 0
    check_states(inst, doms, got, iters, status)
    net.close()
