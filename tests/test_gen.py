"""Seeded generator: SplitMix64 against its published test vector, model-B
counts and structure, determinism."""
import numpy as np
import pytest

from paper_2407_11388_amd import gen
from paper_2407_11388_amd.gen import workloads


def test_splitmix64_published_vector():
    # First outputs of SplitMix64 seeded with 1234567, as published with the
    # algorithm's reference description (Steele, Lea & Flood 2014).
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    assert gen.splitmix64_stream(1234567, 5).tolist() == expect


def test_rand_below_in_range_and_roughly_uniform():
    r = gen.rand_below(7, 10, 20000)
    assert r.min() >= 0 and r.max() <= 9
    counts = np.bincount(r.astype(np.int64), minlength=10)
    assert counts.min() > 1800 and counts.max() < 2200


@pytest.mark.parametrize("n,d,p1,p2", [(50, 10, 0.5, 0.3), (30, 7, 1.0, 0.6), (40, 64, 0.2, 0.1),
                                       (12, 1, 0.5, 0.0), (9, 5, 0.0, 0.5), (25, 33, 0.7, 0.9)])
def test_model_b_counts_and_structure(n, d, p1, p2):
    inst = gen.model_b(11, n, d, p1, p2)
    m = int(np.floor(p1 * n * (n - 1) / 2 + 0.5))
    f = int(np.floor(p2 * d * d + 0.5))
    assert inst.m == m == gen.num_edges(n, p1)
    assert gen.num_forbidden(d, p2) == f
    e = inst.edges
    if m:
        assert (e[:, 0] < e[:, 1]).all() and e.min() >= 0 and e.max() < n
        keys = e[:, 0].astype(np.int64) * n + e[:, 1]
        assert (np.diff(keys) > 0).all()          # sorted, no duplicate pairs
        u8 = inst.rel_u8()
        assert ((u8 == 0).sum(axis=(1, 2)) == f).all()
        if d < 64:
            assert (inst.rel >> np.uint64(d) == 0).all()
        assert np.array_equal(gen.rel_u8_to_bits(u8), inst.rel)


def test_model_b_deterministic_and_seed_sensitive():
    a = gen.model_b(3, 60, 8, 0.4, 0.3)
    b = gen.model_b(3, 60, 8, 0.4, 0.3)
    c = gen.model_b(4, 60, 8, 0.4, 0.3)
    assert np.array_equal(a.edges, b.edges) and np.array_equal(a.rel, b.rel)
    assert not (np.array_equal(a.edges, c.edges) and np.array_equal(a.rel, c.rel))


def test_workload_sizes_match_their_definitions():
    w = workloads.single_small()
    assert w.instances[0].m == 613 and gen.num_forbidden(10, 0.3) == 30
    assert gen.num_edges(500, 1.0) == 124750 and gen.num_forbidden(20, 0.35) == 140
    assert gen.num_edges(2000, 0.9) == 1799100 and gen.num_forbidden(32, 0.2) == 205
    assert gen.num_edges(1000, 0.8) == 399600 and gen.num_forbidden(32, 0.25) == 256


def test_preremove_exact_count():
    dom = gen.preremove(20, 500, 20, 1000)
    present = sum(bin(int(v)).count("1") for v in dom)
    assert present == 500 * 20 - 1000


def test_partial_assignment_states():
    dom, k = gen.partial_assign_states(40, 100, 32, 64, 20)
    full = np.uint64((1 << 32) - 1)
    for s in range(64):
        single = [x for x in range(100) if dom[s, x] != full]
        assert len(single) == k[s] and 0 <= k[s] <= 20
        for x in single:
            v = int(dom[s, x])
            assert v != 0 and v & (v - 1) == 0


def test_uneven_params_ranges():
    n, d, p1, p2 = gen.uneven_params(5, 256, 20, 800, 4, 64, 0.1, 1.0, 0.1, 0.6)
    assert n.min() >= 20 and n.max() <= 800 and d.min() >= 4 and d.max() <= 64
    assert p1.min() >= 0.1 and p1.max() < 1.0 and p2.min() >= 0.1 and p2.max() < 0.6
