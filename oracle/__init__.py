"""CPU oracle for arc-consistency enforcement — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never imports, links or runs it, and the
two share no code: the only common inputs come from the seeded generator in
``paper_2407_11388_amd.gen``, which holds none of the method's arithmetic.

What it computes (all in plain C on 0/1 bytes, ``rac_oracle.c``):

* ``ac3``       the arc-consistency closure D_ac (Section 3: the union of all
                arc-consistent subsets of D) by the queue-and-revise paradigm
                the paper contrasts with (Section 1), run to an empty queue;
* ``rac_sync``  the recurrence of Eq. (1) stepped as in Algorithm 1, which
                gives the iteration count, the state after every step and the
                stop-on-wipe-out variant;
* ``is_ac``     the definition of arc consistency (Section 3), as a check.

``brute.py`` holds the definitions themselves (union of all arc-consistent
subsets; enumeration of all solutions) for tiny instances; they pin the two
algorithms above. ``search.py`` holds the MAC search of Algorithm 2 (every
node's closure by ``ac3``), pinned by ``brute.solutions`` and closed-form
solution counts.

Pins (see ``tests/test_oracle.py``): brute force on tiny instances, the closed
forms of chains / cliques / empty and universal relations, hand-worked golden
cases under ``tests/golden/``, and the invariants of Lemma 1, Proposition 1
and Proposition 2. AC-3's revision and look-up counters are pinned by the
hand-counted values in every golden fixture and by their closed form for
universal relations; ``is_ac`` by the definition evaluated by brute force (a
set is arc consistent iff it equals its own closure) and by rejecting D_ac
plus any value it lacks. No function here is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

RUN_TO_FIXPOINT = 0
STOP_ON_WIPEOUT = 1


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` in place with gcc (plain C, -O2)."""
    src = os.path.join(_HERE, "rac_oracle.c")
    tmp = _LIB_PATH + ".tmp"
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-fvisibility=hidden", src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.oracle_ac3.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, vp, vp, vp, vp]
    lib.oracle_ac3.restype = ctypes.c_int
    lib.oracle_rac_sync.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, vp, vp, vp,
                                    vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                    vp, vp]
    lib.oracle_rac_sync.restype = ctypes.c_int
    lib.oracle_is_ac.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, vp, vp, vp]
    lib.oracle_is_ac.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def dom_masks_to_u8(dom_masks: np.ndarray, d: int) -> np.ndarray:
    """uint64 masks [n] (bit a = value a present) -> 0/1 bytes [n, d]."""
    dm = np.asarray(dom_masks, dtype=np.uint64)
    out = np.zeros((dm.shape[0], d), dtype=np.uint8)
    for a in range(d):
        out[:, a] = ((dm >> np.uint64(a)) & np.uint64(1)).astype(np.uint8)
    return out


def dom_u8_to_masks(dom_u8: np.ndarray) -> np.ndarray:
    n, d = dom_u8.shape
    out = np.zeros(n, dtype=np.uint64)
    for a in range(d):
        out |= dom_u8[:, a].astype(np.uint64) << np.uint64(a)
    return out


def _prep(edges, rel_u8, dom_u8):
    edges = np.ascontiguousarray(edges, dtype=np.int32)
    rel_u8 = np.ascontiguousarray(rel_u8, dtype=np.uint8)
    dom_u8 = np.array(dom_u8, dtype=np.uint8, copy=True, order="C")
    return edges, rel_u8, dom_u8


def ac3(n: int, d: int, edges, rel_u8, dom_u8):
    """AC-3 to an empty queue. Returns (dom_u8 [n,d], status, revisions, lookups)."""
    edges, rel_u8, dom = _prep(edges, rel_u8, dom_u8)
    stats = np.zeros(2, dtype=np.int64)
    st = _load().oracle_ac3(n, d, edges.shape[0], _ptr(edges), _ptr(rel_u8), _ptr(dom), _ptr(stats))
    if st < 0:
        raise ValueError("oracle_ac3: bad input")
    return dom, int(st), int(stats[0]), int(stats[1])


def rac_sync(n: int, d: int, edges, rel_u8, dom_u8, changed0=None, mode: int = RUN_TO_FIXPOINT,
             incremental: bool = True, max_steps: int = 0, trace: bool = False):
    """Eq. (1) stepped as in Algorithm 1.

    Returns dict(dom, iters, status, converged, checks, trace) where ``trace`` is
    [iters, n, d] (state after each step) when requested.
    """
    edges, rel_u8, dom = _prep(edges, rel_u8, dom_u8)
    if max_steps <= 0:
        max_steps = n * d + 1
    ch = None
    if changed0 is not None:
        ch = np.zeros(n, dtype=np.uint8)
        ch[np.asarray(changed0, dtype=np.int64)] = 1
    tr = np.zeros((max_steps, n, d), dtype=np.uint8) if trace else None
    iters = np.zeros(1, dtype=np.int32)
    status = np.zeros(1, dtype=np.int32)
    checks = np.zeros(1, dtype=np.int64)
    rc = _load().oracle_rac_sync(n, d, edges.shape[0], _ptr(edges), _ptr(rel_u8), _ptr(dom),
                                 _ptr(ch), mode, 1 if incremental else 0, max_steps, _ptr(tr),
                                 _ptr(iters), _ptr(status), _ptr(checks))
    if rc < 0:
        raise ValueError("oracle_rac_sync: bad input")
    k = int(iters[0])
    return dict(dom=dom, iters=k, status=int(status[0]), converged=(rc == 0),
                checks=int(checks[0]), trace=None if tr is None else tr[:k].copy())


def is_ac(n: int, d: int, edges, rel_u8, dom_u8) -> bool:
    edges, rel_u8, dom = _prep(edges, rel_u8, dom_u8)
    r = _load().oracle_is_ac(n, d, edges.shape[0], _ptr(edges), _ptr(rel_u8), _ptr(dom))
    if r < 0:
        raise ValueError("oracle_is_ac: bad input")
    return bool(r)
