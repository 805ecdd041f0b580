"""Seeded synthetic inputs for the RAC library and its oracle.

Model-B random binary CSPs and initial domain states (see ``modelb.c`` for the
definition of every draw). This module produces inputs only: it holds none of
the arc-consistency arithmetic, and both the HIP path and the CPU oracle are
fed from it.

The paper's benchmark is random binary CSPs whose variable pairs are each
constrained with a given density (Section 5.2); domain size and tightness are
not given there, so the model-B parameters of each workload are stated
explicitly in ``workloads.py``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmodelb.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libmodelb.so`` in place with gcc."""
    import subprocess

    src = os.path.join(_HERE, "modelb.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fvisibility=hidden",
           src, "-o", tmp, "-lm"]
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.mb_splitmix64.argtypes = [u64p]
    lib.mb_splitmix64.restype = ctypes.c_uint64
    lib.mb_rand_below.argtypes = [u64p, ctypes.c_uint64]
    lib.mb_rand_below.restype = ctypes.c_uint64
    lib.mb_substream.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.mb_substream.restype = ctypes.c_uint64
    lib.mb_num_edges.argtypes = [ctypes.c_int32, ctypes.c_double]
    lib.mb_num_edges.restype = ctypes.c_int64
    lib.mb_num_forbidden.argtypes = [ctypes.c_int32, ctypes.c_double]
    lib.mb_num_forbidden.restype = ctypes.c_int32
    lib.mb_generate.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_double, ctypes.c_double, i32p, u64p]
    lib.mb_generate.restype = ctypes.c_int
    lib.mb_full_domains.argtypes = [ctypes.c_int32, ctypes.c_int32, u64p]
    lib.mb_full_domains.restype = None
    lib.mb_preremove.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int64, u64p]
    lib.mb_preremove.restype = ctypes.c_int
    lib.mb_partial_assign_states.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32, u64p, i32p]
    lib.mb_partial_assign_states.restype = ctypes.c_int
    lib.mb_uneven_params.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, i32p, i32p, f64p, f64p]
    lib.mb_uneven_params.restype = None
    _lib = lib
    return lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    """The first ``count`` SplitMix64 outputs of a stream seeded with ``seed``."""
    lib = _load()
    st = ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF)
    return np.array([lib.mb_splitmix64(ctypes.byref(st)) for _ in range(count)], dtype=np.uint64)


def rand_below(seed: int, bound: int, count: int) -> np.ndarray:
    lib = _load()
    st = ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF)
    return np.array([lib.mb_rand_below(ctypes.byref(st), bound) for _ in range(count)],
                    dtype=np.uint64)


def substream(seed: int, idx: int) -> int:
    return int(_load().mb_substream(seed & 0xFFFFFFFFFFFFFFFF, idx))


def num_edges(n: int, p1: float) -> int:
    return int(_load().mb_num_edges(n, p1))


def num_forbidden(d: int, p2: float) -> int:
    return int(_load().mb_num_forbidden(d, p2))


@dataclass
class Instance:
    """A binary CSP: ``edges[m,2]`` (x<y) and ``rel[m,d]`` uint64 rows, where bit b of
    ``rel[e,a]`` is 1 iff the pair (x_e=a, y_e=b) is allowed."""

    n: int
    d: int
    edges: np.ndarray
    rel: np.ndarray
    p1: float = float("nan")
    p2: float = float("nan")
    seed: int = 0

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])

    def rel_u8(self) -> np.ndarray:
        """The same relations as 0/1 bytes ``[m, d, d]`` (rel[e,a,b])."""
        return rel_bits_to_u8(self.rel, self.d)


def rel_bits_to_u8(rel: np.ndarray, d: int) -> np.ndarray:
    """Bit rows [m, d] uint64 (bit b of row a) -> 0/1 bytes [m, d, d]."""
    m = rel.shape[0]
    le = np.ascontiguousarray(rel, dtype="<u8").reshape(m, d).view(np.uint8).reshape(m, d, 8)
    return np.ascontiguousarray(np.unpackbits(le, axis=2, bitorder="little")[:, :, :d])


def rel_u8_to_bits(rel_u8: np.ndarray) -> np.ndarray:
    m, d, d2 = rel_u8.shape
    assert d == d2
    w = (np.uint64(1) << np.arange(d, dtype=np.uint64)).reshape(1, 1, d)
    return (rel_u8.astype(np.uint64) * w).sum(axis=2, dtype=np.uint64)


def model_b(seed: int, n: int, d: int, p1: float, p2: float) -> Instance:
    lib = _load()
    m = num_edges(n, p1)
    edges = np.zeros((m, 2), dtype=np.int32)
    rel = np.zeros((m, d), dtype=np.uint64)
    rc = lib.mb_generate(seed, n, d, p1, p2, _p(edges, ctypes.c_int32), _p(rel, ctypes.c_uint64))
    if rc != 0:
        raise ValueError(f"model_b generation failed (n={n}, d={d})")
    return Instance(n=n, d=d, edges=edges, rel=rel, p1=p1, p2=p2, seed=seed)


def full_domains(n: int, d: int) -> np.ndarray:
    dom = np.zeros(n, dtype=np.uint64)
    _load().mb_full_domains(n, d, _p(dom, ctypes.c_uint64))
    return dom


def preremove(seed: int, n: int, d: int, count: int) -> np.ndarray:
    dom = np.zeros(n, dtype=np.uint64)
    if _load().mb_preremove(seed, n, d, count, _p(dom, ctypes.c_uint64)) != 0:
        raise ValueError("bad pre-removal count")
    return dom


def partial_assign_states(seed: int, n: int, d: int, B: int, max_assign: int):
    """Returns (dom[B,n] uint64, n_assigned[B] int32)."""
    dom = np.zeros((B, n), dtype=np.uint64)
    k = np.zeros(B, dtype=np.int32)
    if _load().mb_partial_assign_states(seed, n, d, B, max_assign, _p(dom, ctypes.c_uint64),
                                        _p(k, ctypes.c_int32)) != 0:
        raise MemoryError("partial_assign_states")
    return dom, k


def uneven_params(seed: int, k: int, nmin: int, nmax: int, dmin: int, dmax: int,
                  p1lo: float, p1hi: float, p2lo: float, p2hi: float):
    n = np.zeros(k, dtype=np.int32)
    d = np.zeros(k, dtype=np.int32)
    p1 = np.zeros(k, dtype=np.float64)
    p2 = np.zeros(k, dtype=np.float64)
    _load().mb_uneven_params(seed, k, nmin, nmax, dmin, dmax, p1lo, p1hi, p2lo, p2hi,
                             _p(n, ctypes.c_int32), _p(d, ctypes.c_int32),
                             _p(p1, ctypes.c_double), _p(p2, ctypes.c_double))
    return n, d, p1, p2


def random_tiny(seed: int, n: int, d: int, p1: float, p2: float, dom_keep: float = 1.0):
    """A model-B instance plus an initial domain state in which every value is
    kept with probability ``dom_keep`` (drawn from the same seeded stream)."""
    inst = model_b(seed, n, d, p1, p2)
    dom = full_domains(n, d)
    if dom_keep < 1.0:
        bits = rand_below(substream(seed, 999), 1 << 20, n * d)
        keep = (bits.astype(np.float64) / float(1 << 20)) < dom_keep
        mask = np.zeros(n, dtype=np.uint64)
        for x in range(n):
            for a in range(d):
                if keep[x * d + a]:
                    mask[x] |= np.uint64(1) << np.uint64(a)
        dom = dom & mask
    return inst, dom


def queens(n: int):
    """The n-queens problem as a binary CSP: variable i is the column of the
    queen in row i; every pair of rows needs different columns and different
    diagonals. Returns (edges int32 [m, 2], relations uint8 [m, n, n])."""
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    edges = np.array(pairs, dtype=np.int32).reshape(-1, 2)
    a = np.arange(n).reshape(-1, 1)
    b = np.arange(n).reshape(1, -1)
    rel = np.zeros((len(pairs), n, n), dtype=np.uint8)
    for e, (i, j) in enumerate(pairs):
        rel[e] = ((a != b) & (np.abs(a - b) != j - i)).astype(np.uint8)
    return edges, rel

