"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times: whole results where the oracle finishes in seconds, and
sampled states / instances (each checked in full) for the 1024-state batch
and the 256-instance uneven batch."""
import sys

import numpy as np
import pytest

from paper_2407_11388_amd import gen
from paper_2407_11388_amd.gen import workloads

from helpers import oracle_expect

pytestmark = pytest.mark.gpu

rac = pytest.importorskip("paper_2407_11388_amd.rac")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_single(w, path, mode=0):
    inst, dom = w.instances[0], w.domains[0]
    say(f"[gpu] {w.name} path={path} mode={mode}")
    net = rac.Net.from_instance(inst, path=path, mode=mode)
    got, iters, status = net.enforce(dom)
    st = net.stats()
    net.close()
    exp, e_it, e_st, e_ch, _ = oracle_expect(inst.n, inst.d, inst.edges, inst.rel_u8(), dom, mode)
    assert np.array_equal(got, exp)
    assert (iters, status) == (e_it, e_st)
    assert st.support_checks == e_ch


def test_single_small_full():
    w = workloads.single_small()
    for path in (rac.PATH_BITS, rac.PATH_INT8):
        for mode in (0, 1):
            check_single(w, path, mode)


def test_single_mid_full():
    w = workloads.single_mid()
    for path in (rac.PATH_BITS, rac.PATH_INT8):
        check_single(w, path)


@pytest.mark.timeout(600)
def test_single_large_full():
    w = workloads.single_large()
    for path in (rac.PATH_BITS, rac.PATH_INT8):
        check_single(w, path)


@pytest.mark.timeout(600)
def test_batch_states_full_sampled():
    w = workloads.batch_states()
    inst, doms = w.instances[0], w.domains[0]
    B = doms.shape[0]
    say(f"[gpu] {w.name} auto path")
    net = rac.Net.from_instance(inst)
    got, iters, status = net.enforce_batch(doms)
    st = net.stats()
    assert st.path == rac.PATH_MFMA
    net.close()
    rel = inst.rel_u8()
    # every 48th state, plus the states that took the most steps
    sample = sorted(set(range(0, B, 48)) | set(np.argsort(-iters)[:6].tolist()))
    for s in sample:
        exp, e_it, e_st, _, _ = oracle_expect(inst.n, inst.d, inst.edges, rel, doms[s])
        assert np.array_equal(got[s], exp), f"state {s}"
        assert iters[s] == e_it and status[s] == e_st, f"state {s}"
    # the same states through the plain per-state loop agree exactly
    plain = rac.Net.from_instance(inst, path=rac.PATH_BITS)
    for s in sample[:8]:
        g2, i2, s2 = plain.enforce(doms[s])
        assert np.array_equal(g2, got[s]) and i2 == iters[s] and s2 == status[s]
    plain.close()


@pytest.fixture(scope="module")
def uneven():
    return workloads.uneven_multi()


@pytest.mark.timeout(900)
def test_uneven_multi_full_sampled(uneven):
    w = uneven
    say(f"[gpu] {w.name}: creating {len(w.instances)} networks")
    nets = [rac.Net.from_instance(inst) for inst in w.instances]
    grp = rac.Group(nets)
    say("[gpu] group enforce")
    outs, iters, status = grp.enforce(w.domains)
    outs2, iters2, status2 = grp.enforce(w.domains)   # replay of the captured graph
    for i in range(len(nets)):
        assert np.array_equal(outs[i], outs2[i]) and iters[i] == iters2[i]
    k = len(w.instances)
    sample = sorted(set(range(0, k, 16)) | set(np.argsort(-iters)[:4].tolist()))
    for i in sample:
        inst = w.instances[i]
        exp, e_it, e_st, _, _ = oracle_expect(inst.n, inst.d, inst.edges, inst.rel_u8(), w.domains[i])
        assert np.array_equal(outs[i], exp), f"instance {i} (n={inst.n}, d={inst.d})"
        assert iters[i] == e_it and status[i] == e_st, f"instance {i}"
    grp.close()
    for n in nets:
        n.close()
