"""rac_enforce_batch_noalloc (workspace in the library's fixed device array)
against rac_enforce_batch_device, the entry point it is a variant of: equal
domains, step counts and statuses on consecutive calls, the later ones on
smaller inputs (so that whatever the array holds from an earlier call must not
leak into a later one), plus the oracle on a sample and the size limit."""
import sys

import numpy as np
import pytest

from paper_2407_11388_amd import gen
from paper_2407_11388_amd.gen import workloads

from helpers import oracle_expect

pytestmark = pytest.mark.gpu

rac = pytest.importorskip("paper_2407_11388_amd.rac")
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_both(net, doms):
    """(noalloc, device entry point) results of the same states: each a tuple
    (dom [B, n] uint64, iters [B], status [B])."""
    dev = torch.device("cuda:0")
    B, n = doms.shape
    stream = torch.cuda.current_stream().cuda_stream
    d_in = torch.from_numpy(np.ascontiguousarray(doms).view(np.int64)).to(dev)
    out = []
    for which in ("noalloc", "device"):
        d_out = torch.full((B, n), -1, dtype=torch.int64, device=dev)
        d_it = torch.full((B,), -7, dtype=torch.int32, device=dev)
        d_st = torch.full((B,), -7, dtype=torch.int32, device=dev)
        if which == "noalloc":
            net.enforce_batch_noalloc(d_in, d_out, d_it, d_st, stream)
        else:
            net.enforce_batch_device(d_in, d_out, d_it, d_st, stream)
            net.sync()
        torch.cuda.synchronize()
        out.append((d_out.cpu().numpy().view(np.uint64), d_it.cpu().numpy(), d_st.cpu().numpy()))
    assert np.array_equal(d_in.cpu().numpy().view(np.uint64), doms)   # input untouched
    return out


def assert_same(name, a, b):
    assert np.array_equal(a[1], b[1]), f"{name}: step counts differ"
    assert np.array_equal(a[2], b[2]), f"{name}: statuses differ"
    bad = [s for s in range(a[0].shape[0]) if not np.array_equal(a[0][s], b[0][s])]
    assert not bad, f"{name}: domains of {len(bad)} states differ, first {bad[:8]}"


def test_noalloc_matches_device_entry_point():
    # call 1: the 1024-state batch of the n=1000, d=32 network
    w = workloads.batch_states()
    inst, doms = w.instances[0], w.domains[0]
    net = rac.Net.from_instance(inst)
    say(f"[gpu] noalloc call 1: {w.name}, B={doms.shape[0]}")
    na, dv = run_both(net, doms)
    assert_same("call 1", na, dv)
    for s in (0, 511, 1023):   # and the oracle on a few states
        e_dom, e_it, e_st, _, _ = oracle_expect(inst.n, inst.d, inst.edges, inst.rel_u8(), doms[s])
        assert np.array_equal(na[0][s], e_dom) and na[1][s] == e_it and na[2][s] == e_st, f"state {s}"

    # call 2: fewer, different states of the same network
    doms2, _ = gen.partial_assign_states(91, inst.n, inst.d, 100, 30)
    say("[gpu] noalloc call 2: same network, B=100")
    na2, dv2 = run_both(net, doms2)
    assert_same("call 2", na2, dv2)
    net.close()

    # call 3: a much smaller network, stop-on-wipe-out, B=33
    small = gen.model_b(92, 60, 8, 0.3, 0.45)
    doms3, _ = gen.partial_assign_states(93, small.n, small.d, 33, 6)
    say("[gpu] noalloc call 3: n=60 d=8, stop on wipe-out, B=33")
    net3 = rac.Net.from_instance(small, mode=rac.RAC_STOP_ON_WIPEOUT)
    na3, dv3 = run_both(net3, doms3)
    assert_same("call 3", na3, dv3)
    for s in range(33):
        e_dom, e_it, e_st, _, _ = oracle_expect(small.n, small.d, small.edges, small.rel_u8(),
                                                doms3[s], mode=rac.RAC_STOP_ON_WIPEOUT)
        assert np.array_equal(na3[0][s], e_dom) and na3[1][s] == e_it and na3[2][s] == e_st, f"state {s}"
    net3.close()


def test_noalloc_rejects_oversized_batch():
    inst = gen.model_b(94, 2000, 4, 0.01, 0.3)
    net = rac.Net.from_instance(inst)
    B = 1000   # 1000 states x 2000 variables x 40 bytes > 64 MiB
    dev = torch.device("cuda:0")
    d_in = torch.zeros((B, inst.n), dtype=torch.int64, device=dev)
    d_out = torch.zeros_like(d_in)
    d_it = torch.zeros(B, dtype=torch.int32, device=dev)
    d_st = torch.zeros(B, dtype=torch.int32, device=dev)
    say("[gpu] noalloc oversized call (refused on the host)")
    with pytest.raises(rac.RacError) as ei:
        net.enforce_batch_noalloc(d_in, d_out, d_it, d_st)
    assert ei.value.code == rac.RAC_EINVAL
    # a call that fits still works afterwards
    doms, _ = gen.partial_assign_states(95, inst.n, inst.d, 8, 5)
    na, dv = run_both(net, doms)
    assert_same("after refusal", na, dv)
    net.close()
