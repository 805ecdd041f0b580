"""GPU batched MAC search vs the oracle's MAC search: solution count, node
and failure counts, and the lexicographically smallest solution, on the
closed-form families and random instances, for several batch sizes (the
explored tree of a complete search does not depend on the batch)."""
import sys

import numpy as np
import pytest

from oracle.search import mac_search
from paper_2407_11388_amd import gen

from helpers import cycle_colouring, instance_from_pairs, masks_to_u8, queens

pytestmark = pytest.mark.gpu

rac = pytest.importorskip("paper_2407_11388_amd.rac")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def full_masks(n, d):
    return np.full(n, (1 << d) - 1 if d < 64 else 0xFFFFFFFFFFFFFFFF, dtype=np.uint64)


def check(name, n, d, edges, rel, dom_masks, batches=(1, 5, 256), path=None, **opts):
    exp = mac_search(n, d, edges, rel, masks_to_u8(dom_masks, d))
    kw = dict(opts) if path is None else dict(path=path, **opts)
    net = rac.Net.from_u8(n, d, edges, rel, **kw)
    for b in batches:
        say(f"[gpu] search {name} n={n} d={d} batch={b}")
        res, sol = net.search(dom_masks, batch=b)
        assert res.complete == 1
        assert res.solutions == exp["solutions"], f"{name} batch {b}"
        assert res.nodes == exp["nodes"], f"{name} batch {b}: nodes {res.nodes} != {exp['nodes']}"
        assert res.failures == exp["failures"]
        assert res.sweeps == exp["steps"], f"{name} batch {b}: steps {res.sweeps} != {exp['steps']}"
        if exp["best"] is None:
            assert sol is None
        else:
            assert [int(v).bit_length() - 1 for v in sol] == exp["best"].tolist()
    net.close()


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8])
def test_queens(n):
    edges, rel = queens(n)
    check(f"queens{n}", n, n, edges, rel, full_masks(n, n))


def test_queens10_large_batches():
    # 5889 nodes: rounds of up to 1024 open nodes, and the stack growing past
    # its first allocation with batch 1
    edges, rel = queens(10)
    check("queens10", 10, 10, edges, rel, full_masks(10, 10), batches=(1, 1024))


@pytest.mark.parametrize("n,k", [(3, 3), (5, 3), (6, 2), (7, 2), (6, 3)])
def test_cycle_colourings(n, k):
    edges, rel = cycle_colouring(n, k)
    check(f"cycle{n}-{k}", n, k, edges, rel, full_masks(n, k))


# model-B instances with small trees: many solutions, none, long failures
RANDOM = [(12, 4, 0.5, 0.3, 0), (12, 4, 0.5, 0.3, 1), (12, 4, 0.5, 0.3, 2),
          (30, 5, 0.2, 0.35, 2), (20, 6, 0.4, 0.4, 2), (25, 8, 0.3, 0.45, 1),
          (16, 33, 0.6, 0.6, 0), (16, 33, 0.6, 0.6, 2), (20, 40, 0.5, 0.7, 1)]


@pytest.mark.parametrize("n,d,p1,p2,seed", RANDOM)
def test_random(n, d, p1, p2, seed):
    inst = gen.model_b(800 + seed + 10 * n, n, d, p1, p2)
    check(f"random-n{n}-d{d}-s{seed}", n, d, inst.edges, inst.rel_u8(), full_masks(n, d),
          batches=(3, 64))


def test_int8_path():
    edges, rel = queens(6)
    check("queens6-int8", 6, 6, edges, rel, full_masks(6, 6), batches=(4,), path=rac.PATH_INT8)


def test_fused_rounds_without_graphs():
    # The device-driven rounds of the fused path enqueued kernel by kernel
    # (use_graph=0) instead of as captured batches of rounds.
    edges, rel = queens(7)
    check("queens7-fused-direct", 7, 7, edges, rel, full_masks(7, 7), batches=(1, 5, 256),
          path=rac.PATH_FUSED, use_graph=False)


def test_search_limits_device_rounds():
    # max_nodes / max_solutions are checked before each device-driven round:
    # the search stops at the first round boundary past the limit, as on the
    # round-by-round path.
    edges, rel = queens(8)
    for path in (rac.PATH_FUSED, rac.PATH_BITS):
        net = rac.Net.from_u8(8, 8, edges, rel, path=path)
        say(f"[gpu] search limits path={path}")
        full, _ = net.search(full_masks(8, 8), batch=4)
        res, _ = net.search(full_masks(8, 8), batch=4, max_nodes=50)
        assert res.complete == 0 and 50 <= res.nodes < full.nodes
        res2, sol = net.search(full_masks(8, 8), batch=4, max_solutions=3)
        assert res2.complete == 0 and res2.solutions >= 3 and sol is not None
        net.close()
    # both paths stop at the same round
    got = []
    for path in (rac.PATH_FUSED, rac.PATH_BITS):
        net = rac.Net.from_u8(8, 8, edges, rel, path=path)
        r, _ = net.search(full_masks(8, 8), batch=4, max_nodes=50)
        got.append((r.nodes, r.solutions, r.rounds, r.sweeps))
        net.close()
    assert got[0] == got[1]


@pytest.mark.parametrize("which", ["queens7", "random-n25", "random-n16-d33"])
def test_fused_path(which):
    # Every search round's enforcements in one fused launch (one workgroup
    # per child, @changed = its assigned variable, stop on the first wipe-out).
    if which == "queens7":
        edges, rel = queens(7)
        check("queens7-fused", 7, 7, edges, rel, full_masks(7, 7), batches=(1, 5, 256),
              path=rac.PATH_FUSED)
        return
    n, d, p1, p2, seed = (25, 8, 0.3, 0.45, 1) if which == "random-n25" else (16, 33, 0.6, 0.6, 2)
    inst = gen.model_b(800 + seed + 10 * n, n, d, p1, p2)
    check(f"{which}-fused", n, d, inst.edges, inst.rel_u8(), full_masks(n, d), batches=(3, 64),
          path=rac.PATH_FUSED)


def test_root_cases():
    # root wiped out
    edges, rel = instance_from_pairs(2, 2, [(0, 1, [(0, 1)])])
    net = rac.Net.from_u8(2, 2, edges, rel)
    res, sol = net.search(np.array([1, 1], np.uint64))   # x0 = 0 needs x1 = 1
    assert (res.solutions, res.nodes, res.failures, res.complete) == (0, 1, 1, 1) and sol is None
    # root already a solution
    res, sol = net.search(np.array([1, 2], np.uint64))
    assert (res.solutions, res.nodes, res.failures, res.complete) == (1, 1, 0, 1)
    assert sol.tolist() == [1, 2]
    net.close()


def test_limits():
    edges, rel = queens(8)
    net = rac.Net.from_u8(8, 8, edges, rel)
    res, sol = net.search(full_masks(8, 8), max_solutions=1, batch=1)
    assert res.solutions >= 1 and res.complete == 0
    s = [int(v).bit_length() - 1 for v in sol]
    for i in range(8):
        for j in range(i + 1, 8):
            assert s[i] != s[j] and abs(s[i] - s[j]) != j - i
    res, _ = net.search(full_masks(8, 8), max_nodes=50, batch=4)
    assert res.nodes >= 50 and res.complete == 0
    net.close()


def test_repeated_searches_on_one_net():
    # Consecutive searches with one batch size launch the step kernels with
    # the same arguments and replay the same captured step graphs; a single
    # enforcement in between rebuilds them. Every search is checked against
    # the oracle.
    n = 8
    edges, rel = queens(n)
    net = rac.Net.from_u8(n, n, edges, rel)
    full = full_masks(n, n)
    roots = [full, full.copy(), full.copy(), full.copy()]
    roots[1][0] = 0b00001111          # x0 in {0..3}
    roots[2][3] = (1 << 2) | (1 << 5)  # x3 in {2, 5}
    roots[3][7] = 1 << 6               # x7 = 6
    for rep in range(2):
        for i, root in enumerate(roots):
            say(f"[gpu] repeated search rep={rep} root={i}")
            exp = mac_search(n, n, edges, rel, masks_to_u8(root, n))
            res, sol = net.search(root, batch=64)
            assert (res.solutions, res.nodes, res.failures, res.sweeps) == \
                (exp["solutions"], exp["nodes"], exp["failures"], exp["steps"]), (rep, i)
            if exp["best"] is None:
                assert sol is None
            else:
                assert [int(v).bit_length() - 1 for v in sol] == exp["best"].tolist()
        say(f"[gpu] enforce between searches rep={rep}")
        dom, iters, status = net.enforce(full)
        assert status == 0 and (dom == full).all()
    net.close()


@pytest.mark.parametrize("which", ["queens11", "modelB-n100"])
def test_bench_search_workloads(which):
    # The two search workloads of the bench at its batch (4096 open nodes per
    # round), in full against the oracle's search (about 2 s and 30 s of CPU).
    if which == "queens11":
        n, d = 11, 11
        edges, rel = queens(11)
    else:
        n, d = 100, 10
        inst = gen.model_b(110, 100, 10, 0.1, 0.4)
        edges, rel = inst.edges, inst.rel_u8()
    say(f"[gpu] bench search workload {which}: oracle")
    exp = mac_search(n, d, edges, rel, np.ones((n, d), np.uint8))
    net = rac.Net.from_u8(n, d, edges, rel)
    say(f"[gpu] bench search workload {which}: batch 4096")
    res, sol = net.search(full_masks(n, d), batch=4096)
    assert res.complete == 1
    assert (res.solutions, res.nodes, res.failures, res.sweeps) == \
        (exp["solutions"], exp["nodes"], exp["failures"], exp["steps"])
    if exp["best"] is None:
        assert sol is None
    else:
        assert [int(v).bit_length() - 1 for v in sol] == exp["best"].tolist()
    net.close()


@pytest.mark.parametrize("n,p1", [(100, 0.5), (100, 0.75), (100, 1.0), (250, 0.5), (500, 0.5),
                                  (1000, 1.0)])
def test_table1_cells_complete(n, p1):
    # Cells of the Table 1 grid (model-B stand-ins, d = 10, p2 = 0.3) whose
    # whole search tree the oracle explores in seconds: the GPU search's
    # recurrence steps per assignment (and nodes, failures, solutions) equal
    # the oracle's, at the batch the grid is run with (n = 100 and 250: the
    # fused path's rounds; n = 500 and 1000: the bit-row path's).
    import bench
    inst = bench.table1_instance(n, p1)
    d = bench.TABLE1_D
    rel = inst.rel_u8()
    say(f"[gpu] table 1 cell n={n} density={p1}: oracle")
    exp = mac_search(n, d, inst.edges, rel, np.ones((n, d), np.uint8))
    net = rac.Net.from_u8(n, d, inst.edges, rel)
    say(f"[gpu] table 1 cell n={n} density={p1}: batch {bench.SEARCH_BATCH}")
    res, _ = net.search(full_masks(n, d), batch=bench.SEARCH_BATCH)
    net.close()
    assert res.complete == 1 and exp["complete"]
    assert (res.solutions, res.nodes, res.failures, res.sweeps) == \
        (exp["solutions"], exp["nodes"], exp["failures"], exp["steps"])
    assert res.sweeps / res.nodes == exp["steps"] / exp["nodes"]   # steps per assignment


def test_random_instances_random_batches():
    # Seeded small model-B instances (n 4..12, d 2..4, d^n <= 2e5, density
    # and tightness across their range) searched completely with a random path and batch
    # size; counts, recurrence steps and the smallest solution against the
    # oracle's MAC search.
    rng = np.random.default_rng(2027)
    for c in range(16):
        n, d = int(rng.integers(4, 13)), int(rng.integers(2, 5))
        while d ** n > 200000:   # keeps the oracle's tree small
            n -= 1
        p1, p2 = float(rng.uniform(0.1, 0.9)), float(rng.uniform(0.1, 0.5))
        path = int(rng.choice([rac.PATH_AUTO, rac.PATH_BITS, rac.PATH_FUSED]))
        b = int(rng.choice([1, 3, 64, 4096]))
        inst = gen.model_b(7000 + c, n, d, p1, p2)
        check(f"random{c}", n, d, inst.edges, inst.rel_u8(), full_masks(n, d), batches=(b,),
              path=path)
