"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times: every state of the 1024-state batch and every instance of
the 256-instance uneven batch against the oracle (computed from a pool of
threads: the C oracle runs without the interpreter lock), through the host
entry points and through the device-pointer entry points the benchmark
times."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2407_11388_amd import gen
from paper_2407_11388_amd.gen import workloads

import oracle
from helpers import masks_to_u8, oracle_expect, u8_to_masks

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


POOL = max(1, min(16, os.cpu_count() or 1))


def oracle_many(jobs):
    """Oracle results of many (n, d, edges, rel_u8, dom_masks) states, in order:
    (dom masks, iters, status, checks). The Eq. (1) recurrence gives the step
    count, status and support checks; AC-3 gives the domains, and the two
    must agree. A job may be a callable returning the tuple (built inside the
    worker, so that large relation tensors are not all held at once)."""
    def one(job):
        n, d, edges, rel, dom = job() if callable(job) else job
        du8 = masks_to_u8(dom, d)
        r = oracle.rac_sync(n, d, edges, rel, du8)
        dac, status, _, _ = oracle.ac3(n, d, edges, rel, du8)
        assert r["converged"] and np.array_equal(dac, r["dom"]) and status == r["status"]
        return u8_to_masks(r["dom"]), r["iters"], r["status"], r["checks"]
    with ThreadPoolExecutor(max_workers=POOL) as ex:
        return list(ex.map(one, jobs))


@pytest.fixture(scope="module")
def batch_states():
    w = workloads.batch_states()
    inst, doms = w.instances[0], w.domains[0]
    rel = inst.rel_u8()
    say(f"[gpu] {w.name}: oracle on {doms.shape[0]} states ({POOL} threads)")
    exp = oracle_many([(inst.n, inst.d, inst.edges, rel, doms[s]) for s in range(doms.shape[0])])
    return w, exp


def check_batch(name, exp, got, iters, status, checks=None):
    bad = [s for s in range(len(exp))
           if not (np.array_equal(got[s], exp[s][0]) and iters[s] == exp[s][1]
                   and status[s] == exp[s][2])]
    assert not bad, f"{name}: {len(bad)} states differ from the oracle, first {bad[:8]}"
    if checks is not None:
        assert checks == sum(e[3] for e in exp), f"{name}: support checks"


@pytest.mark.timeout(900)
def test_batch_states_full(batch_states):
    w, exp = batch_states
    inst, doms = w.instances[0], w.domains[0]
    say(f"[gpu] {w.name}: host entry point, auto path")
    net = rac.Net.from_instance(inst)
    got, iters, status = net.enforce_batch(doms)
    st = net.stats()
    assert st.path == rac.PATH_MFMA
    check_batch("rac_enforce_batch", exp, got, iters, status, st.support_checks)
    net.close()


@pytest.mark.timeout(900)
def test_batch_states_full_device_entry_point(batch_states):
    # the entry point and launch configuration the benchmark times: device
    # buffers, torch's current stream, repeated calls on one net
    torch = pytest.importorskip("torch")
    w, exp = batch_states
    inst, doms = w.instances[0], w.domains[0]
    B = doms.shape[0]
    dev = torch.device("cuda:0")
    say(f"[gpu] {w.name}: rac_enforce_batch_device, auto path")
    net = rac.Net.from_instance(inst, profile=True)
    d_in = torch.from_numpy(doms.view(np.int64)).to(dev)
    d_out = torch.empty_like(d_in)
    d_it = torch.empty(B, dtype=torch.int32, device=dev)
    d_st = torch.empty(B, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    for rep in range(2):
        net.enforce_batch_device(d_in, d_out, d_it, d_st, stream)
        net.sync()
        torch.cuda.synchronize()
        st = net.stats()
        assert st.path == rac.PATH_MFMA
        check_batch(f"rac_enforce_batch_device (call {rep})", exp,
                    d_out.cpu().numpy().view(np.uint64), d_it.cpu().numpy(),
                    d_st.cpu().numpy(), st.support_checks)
    assert np.array_equal(d_in.cpu().numpy().view(np.uint64), doms)   # input untouched
    net.close()


@pytest.mark.timeout(900)
def test_batch_states_plain_loop_agrees(batch_states):
    # the plain per-state loop the benchmark compares with: sequential
    # rac_enforce calls on the bit-row path, on a sample of the states
    w, exp = batch_states
    inst, doms = w.instances[0], w.domains[0]
    say(f"[gpu] {w.name}: plain rac_enforce loop")
    plain = rac.Net.from_instance(inst, path=rac.PATH_BITS)
    for s in range(0, doms.shape[0], 16):
        g2, i2, s2 = plain.enforce(doms[s])
        assert np.array_equal(g2, exp[s][0]) and i2 == exp[s][1] and s2 == exp[s][2], f"state {s}"
    plain.close()


@pytest.fixture(scope="module")
def uneven():
    w = workloads.uneven_multi()
    say(f"[gpu] {w.name}: oracle on {len(w.instances)} instances ({POOL} threads)")
    exp = oracle_many([(lambda i=i, dom=dom: (i.n, i.d, i.edges, i.rel_u8(), dom))
                       for i, dom in zip(w.instances, w.domains)])
    return w, exp


@pytest.mark.timeout(900)
def test_uneven_multi_full(uneven):
    torch = pytest.importorskip("torch")
    w, exp = uneven
    say(f"[gpu] {w.name}: creating {len(w.instances)} networks")
    nets = [rac.Net.from_instance(inst) for inst in w.instances]
    grp = rac.Group(nets)
    say("[gpu] group enforce (host entry point), twice")
    for rep in range(2):   # the second call replays the captured graphs
        outs, iters, status = grp.enforce(w.domains)
        check_batch(f"rac_group_enforce (call {rep})", exp, outs, iters, status,
                    grp.stats().support_checks)
    say("[gpu] group enforce (device entry point)")
    dev = torch.device("cuda:0")
    flat = np.concatenate(w.domains).view(np.int64)
    d_dom = torch.from_numpy(flat).to(dev)
    d_it = torch.empty(len(nets), dtype=torch.int32, device=dev)
    d_st = torch.empty(len(nets), dtype=torch.int32, device=dev)
    grp.enforce_device(d_dom, d_it, d_st, torch.cuda.current_stream().cuda_stream)
    grp.sync()
    torch.cuda.synchronize()
    res = d_dom.cpu().numpy().view(np.uint64)
    off = np.concatenate([[0], np.cumsum([i.n for i in w.instances])])
    check_batch("rac_group_enforce_device", exp, [res[off[i]:off[i + 1]] for i in range(len(nets))],
                d_it.cpu().numpy(), d_st.cpu().numpy())
    grp.close()
    for n in nets:
        n.close()
