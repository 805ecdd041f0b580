"""Python binding of librac (rac.h): argument marshalling only.

Every step of the enforcement runs in the HIP kernels of ``librac.so``; this
module converts numpy arrays / torch tensors to pointers and return codes to
exceptions. If the library has not been built, importing this module fails
loudly: there is no CPU fallback.

The entry points keep the C names (``rac_create``, ``rac_enforce``,
``rac_enforce_batch``, ...); ``Net`` and ``Group`` wrap them for convenience.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RAC_LIB_PATH") or os.path.join(_HERE, "librac.so")

RAC_OK = 0
RAC_EINVAL = -1
RAC_ENOMEM = -2
RAC_EHIP = -3
RAC_EUNSUPPORTED = -4
RAC_ENOTCONVERGED = -5
RAC_ENODEV = -6
RAC_ETIMEOUT = -7

RAC_CONSISTENT = 0
RAC_WIPEOUT = 1
RAC_RUN_TO_FIXPOINT = 0
RAC_STOP_ON_WIPEOUT = 1
PATH_AUTO, PATH_BITS, PATH_INT8, PATH_MFMA, PATH_FUSED = 0, 1, 2, 3, 4
PATH_NAMES = {PATH_AUTO: "auto", PATH_BITS: "bits", PATH_INT8: "int8", PATH_MFMA: "mfma",
              PATH_FUSED: "fused"}
SMALL_MAX_N = 2048   # largest network the fused path (one workgroup per state) holds

EXPORTED = [
    "rac_default_options", "rac_create", "rac_create_bits", "rac_create_dense", "rac_destroy",
    "rac_enforce", "rac_enforce_batch", "rac_enforce_batch_device", "rac_sync_status",
    "rac_enforce_batch_noalloc",
    "rac_enforce_multi", "rac_group_create", "rac_group_enforce", "rac_group_enforce_device",
    "rac_group_sync_status", "rac_group_destroy", "rac_net_stats", "rac_group_stats",
    "rac_net_info", "rac_search", "rac_strerror", "rac_last_error",
]


class RacError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


class rac_options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("path", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("item_bytes", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("tune", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class rac_stats(ctypes.Structure):
    _fields_ = [("support_checks", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("relation_bytes", ctypes.c_int64), ("device_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("kernel_launches", ctypes.c_int64),
                ("algo_ops", ctypes.c_int64), ("path", ctypes.c_int32),
                ("item_bytes", ctypes.c_int32), ("first_kernel_ms", ctypes.c_float),
                ("tune_source", ctypes.c_int32)]


class rac_search_result(ctypes.Structure):
    _fields_ = [("solutions", ctypes.c_int64), ("nodes", ctypes.c_int64),
                ("failures", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("sweeps", ctypes.c_int64),
                ("complete", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("search_ms", ctypes.c_double)]


def _share_runtime_with_torch():
    """PyTorch ships its own HIP runtime. Importing it first makes librac's
    libamdhip64.so.7 / libhsa-runtime64.so.1 resolve to that same runtime (by
    soname), so one process never holds two HIP runtimes; with the order
    reversed, torch would load a second copy and fail to see the GPU."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def _load():
    _share_runtime_with_torch()
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first "
                           "(the library has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "rac_default_options": ([vp], None),
        "rac_create": ([i32, i32, i64, vp, vp, vp, pp], ctypes.c_int),
        "rac_create_bits": ([i32, i32, i64, vp, vp, vp, pp], ctypes.c_int),
        "rac_create_dense": ([i32, i32, vp, i64, vp, vp, pp], ctypes.c_int),
        "rac_destroy": ([vp], None),
        "rac_enforce": ([vp, vp, vp, i32, vp, vp], ctypes.c_int),
        "rac_enforce_batch": ([vp, i32, vp, vp, vp], ctypes.c_int),
        "rac_enforce_batch_device": ([vp, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "rac_sync_status": ([vp], ctypes.c_int),
        "rac_enforce_batch_noalloc": ([vp, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "rac_enforce_multi": ([i32, vp, vp, vp, vp], ctypes.c_int),
        "rac_group_create": ([i32, vp, vp, pp], ctypes.c_int),
        "rac_group_enforce": ([vp, vp, vp, vp], ctypes.c_int),
        "rac_group_enforce_device": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "rac_group_sync_status": ([vp], ctypes.c_int),
        "rac_group_destroy": ([vp], None),
        "rac_net_stats": ([vp, vp], ctypes.c_int),
        "rac_group_stats": ([vp, vp], ctypes.c_int),
        "rac_net_info": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "rac_search": ([vp, vp, i64, i64, i32, vp, vp], ctypes.c_int),
        "rac_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "rac_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _check(rc: int, where: str):
    if rc != RAC_OK:
        msg = lib.rac_last_error().decode(errors="replace") or lib.rac_strerror(rc).decode()
        raise RacError(rc, where, msg)


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())  # torch tensor: device or host pointer


def _check_device_tensors(where: str, specs):
    """specs: (name, tensor, element bytes, exact shape tuple or minimum numel).
    Every tensor must be a contiguous GPU tensor on the same device, with the
    element size and the shape the entry point reads and writes."""
    dev = None
    for name, t, esize, shape in specs:
        if not getattr(t, "is_cuda", False):
            raise ValueError(f"{where}: {name} must be a tensor on the GPU")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{where}: {name} is on {t.device}, expected {dev}")
        if not t.is_contiguous():
            raise ValueError(f"{where}: {name} must be contiguous")
        if t.element_size() != esize or (esize == 4 and str(t.dtype) != "torch.int32"):
            raise ValueError(f"{where}: {name} must have {'int32' if esize == 4 else '8-byte'} elements")
        if isinstance(shape, tuple):
            if tuple(t.shape) != shape:
                raise ValueError(f"{where}: {name} has shape {tuple(t.shape)}, expected {shape}")
        elif t.numel() < shape:
            raise ValueError(f"{where}: {name} has {t.numel()} elements, needs {shape}")


TUNE_AUTO, TUNE_RULES, TUNE_MEASURE = 0, 1, 2
TUNE_SOURCES = {0: "rules", 1: "shipped table", 2: "user table", 3: "measured"}


def options(mode: int = RAC_RUN_TO_FIXPOINT, max_sweeps: int = 0, path: int = PATH_AUTO,
            use_graph: bool = True, item_bytes: int = 0, profile: bool = False,
            tune: int = TUNE_AUTO) -> rac_options:
    o = rac_options()
    lib.rac_default_options(ctypes.byref(o))
    o.mode, o.max_sweeps, o.path = mode, max_sweeps, path
    o.use_graph, o.item_bytes = 1 if use_graph else 0, item_bytes
    o.profile = 1 if profile else 0
    o.tune = tune
    return o


class Net:
    """A network on the GPU (owns a ``rac_net``)."""

    def __init__(self, handle: int, n: int, d: int, m: int, opt: rac_options):
        self.handle = handle
        self.n, self.d, self.m = n, d, m
        self.opt = opt

    @classmethod
    def from_bits(cls, n: int, d: int, edges: np.ndarray, rel_rows: np.ndarray, **kw) -> "Net":
        edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        rel_rows = np.ascontiguousarray(rel_rows, dtype=np.uint64)
        opt = options(**kw)
        h = ctypes.c_void_p()
        _check(lib.rac_create_bits(n, d, edges.shape[0], _ptr(edges), _ptr(rel_rows),
                                   ctypes.byref(opt), ctypes.byref(h)), "rac_create_bits")
        return cls(h.value, n, d, edges.shape[0], opt)

    @classmethod
    def from_u8(cls, n: int, d: int, edges: np.ndarray, rel_u8: np.ndarray, **kw) -> "Net":
        edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        rel_u8 = np.ascontiguousarray(rel_u8, dtype=np.uint8)
        opt = options(**kw)
        h = ctypes.c_void_p()
        _check(lib.rac_create(n, d, edges.shape[0], _ptr(edges), _ptr(rel_u8), ctypes.byref(opt),
                              ctypes.byref(h)), "rac_create")
        return cls(h.value, n, d, edges.shape[0], opt)

    @classmethod
    def from_dense(cls, n: int, d: int, R: np.ndarray, edges: np.ndarray, **kw) -> "Net":
        edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        R = np.ascontiguousarray(R, dtype=np.uint8)
        opt = options(**kw)
        h = ctypes.c_void_p()
        _check(lib.rac_create_dense(n, d, _ptr(R), edges.shape[0], _ptr(edges), ctypes.byref(opt),
                                    ctypes.byref(h)), "rac_create_dense")
        return cls(h.value, n, d, edges.shape[0], opt)

    @classmethod
    def from_instance(cls, inst, **kw) -> "Net":
        return cls.from_bits(inst.n, inst.d, inst.edges, inst.rel, **kw)

    def close(self):
        if self.handle:
            lib.rac_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def enforce(self, dom: np.ndarray, changed: Optional[Sequence[int]] = None):
        """One state: returns (dom [n] uint64, iters, status)."""
        out = np.array(dom, dtype=np.uint64, copy=True).reshape(self.n)
        it = ctypes.c_int32()
        st = ctypes.c_int32()
        ch = None
        nch = 0
        if changed is not None:
            ch = np.ascontiguousarray(changed, dtype=np.int32)
            nch = ch.shape[0]
        _check(lib.rac_enforce(self.handle, _ptr(out), _ptr(ch), nch, ctypes.byref(it),
                               ctypes.byref(st)), "rac_enforce")
        return out, it.value, st.value

    def enforce_batch(self, dom: np.ndarray):
        """B states [B, n]: returns (dom [B, n], iters [B], status [B])."""
        out = np.array(dom, dtype=np.uint64, copy=True)
        B = out.shape[0]
        it = np.zeros(B, dtype=np.int32)
        st = np.zeros(B, dtype=np.int32)
        _check(lib.rac_enforce_batch(self.handle, B, _ptr(out), _ptr(it), _ptr(st)),
               "rac_enforce_batch")
        return out, it, st

    def enforce_batch_device(self, d_in, d_out, d_iters, d_status, stream: int = 0):
        """Device pointers (torch tensors on the GPU): d_in and d_out [B, n] of
        8-byte elements, d_iters and d_status [>= B] int32, all contiguous on
        one GPU. Enqueues the call on `stream` (a hipStream_t as an int)."""
        if getattr(d_in, "dim", None) is None or d_in.dim() != 2 or d_in.shape[1] != self.n:
            raise ValueError(f"d_in must be a [B, {self.n}] tensor")
        B = int(d_in.shape[0])
        _check_device_tensors("enforce_batch_device",
                              [("d_in", d_in, 8, (B, self.n)), ("d_out", d_out, 8, (B, self.n)),
                               ("d_iters", d_iters, 4, B), ("d_status", d_status, 4, B)])
        _check(lib.rac_enforce_batch_device(self.handle, B, _ptr(d_in), _ptr(d_out), _ptr(d_iters),
                                            _ptr(d_status), stream or None),
               "rac_enforce_batch_device")

    def enforce_batch_noalloc(self, d_in, d_out, d_iters, d_status, stream: int = 0):
        """rac_enforce_batch_noalloc: as enforce_batch_device (same tensors), on
        the bit-row path with the library's fixed workspace; returns when the
        results are complete."""
        if getattr(d_in, "dim", None) is None or d_in.dim() != 2 or d_in.shape[1] != self.n:
            raise ValueError(f"d_in must be a [B, {self.n}] tensor")
        B = int(d_in.shape[0])
        _check_device_tensors("enforce_batch_noalloc",
                              [("d_in", d_in, 8, (B, self.n)), ("d_out", d_out, 8, (B, self.n)),
                               ("d_iters", d_iters, 4, B), ("d_status", d_status, 4, B)])
        _check(lib.rac_enforce_batch_noalloc(self.handle, B, _ptr(d_in), _ptr(d_out),
                                             _ptr(d_iters), _ptr(d_status), stream or None),
               "rac_enforce_batch_noalloc")

    def search(self, dom: np.ndarray, max_solutions: int = 0, max_nodes: int = 0,
               batch: int = 0):
        """Batched MAC search from root domains [n]: returns (rac_search_result,
        the lexicographically smallest solution found as [n] uint64, or None)."""
        root = np.ascontiguousarray(dom, dtype=np.uint64).reshape(self.n)
        sol = np.zeros(self.n, dtype=np.uint64)
        res = rac_search_result()
        _check(lib.rac_search(self.handle, _ptr(root), max_solutions, max_nodes, batch, _ptr(sol),
                              ctypes.byref(res)), "rac_search")
        return res, (sol if res.solutions > 0 else None)

    def sync(self):
        _check(lib.rac_sync_status(self.handle), "rac_sync_status")

    def stats(self) -> rac_stats:
        s = rac_stats()
        _check(lib.rac_net_stats(self.handle, ctypes.byref(s)), "rac_net_stats")
        return s


class Group:
    """Several networks enforced together: every step of every network runs in the
    same kernels (captured graphs, one per round of steps)."""

    def __init__(self, nets: Sequence[Net], **kw):
        self.nets = list(nets)
        arr = (ctypes.c_void_p * len(self.nets))(*[n.handle for n in self.nets])
        self._arr = arr
        opt = options(**kw)
        h = ctypes.c_void_p()
        _check(lib.rac_group_create(len(self.nets), arr, ctypes.byref(opt), ctypes.byref(h)),
               "rac_group_create")
        self.handle = h.value
        self.offsets = np.concatenate([[0], np.cumsum([n.n for n in self.nets])]).astype(np.int64)

    def close(self):
        if self.handle:
            lib.rac_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def enforce(self, doms: Sequence[np.ndarray]):
        outs = [np.array(d, dtype=np.uint64, copy=True) for d in doms]
        ptrs = (ctypes.c_void_p * len(outs))(*[o.ctypes.data for o in outs])
        k = len(outs)
        it = np.zeros(k, dtype=np.int32)
        st = np.zeros(k, dtype=np.int32)
        _check(lib.rac_group_enforce(self.handle, ptrs, _ptr(it), _ptr(st)), "rac_group_enforce")
        return outs, it, st

    def enforce_device(self, d_dom, d_iters, d_status, stream: int = 0):
        """d_dom: [sum of n_i] 8-byte elements (the nets' states back to back, in/out);
        d_iters, d_status: [>= k] int32; contiguous tensors on one GPU."""
        k, total = len(self.nets), int(self.offsets[-1])
        _check_device_tensors("Group.enforce_device",
                              [("d_dom", d_dom, 8, (total,)), ("d_iters", d_iters, 4, k),
                               ("d_status", d_status, 4, k)])
        _check(lib.rac_group_enforce_device(self.handle, _ptr(d_dom), _ptr(d_iters),
                                            _ptr(d_status), stream or None),
               "rac_group_enforce_device")

    def sync(self):
        _check(lib.rac_group_sync_status(self.handle), "rac_group_sync_status")

    def stats(self) -> rac_stats:
        s = rac_stats()
        _check(lib.rac_group_stats(self.handle, ctypes.byref(s)), "rac_group_stats")
        return s


def enforce_multi(nets: Sequence[Net], doms: Sequence[np.ndarray]):
    outs = [np.array(d, dtype=np.uint64, copy=True) for d in doms]
    ptrs = (ctypes.c_void_p * len(outs))(*[o.ctypes.data for o in outs])
    arr = (ctypes.c_void_p * len(nets))(*[n.handle for n in nets])
    k = len(nets)
    it = np.zeros(k, dtype=np.int32)
    st = np.zeros(k, dtype=np.int32)
    _check(lib.rac_enforce_multi(k, arr, ptrs, _ptr(it), _ptr(st)), "rac_enforce_multi")
    return outs, it, st
