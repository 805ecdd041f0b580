"""The C-ABI library loads and exports every entry point rac.h declares;
host-side validation rejects bad input before any device work (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2407_11388_amd import rac

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "rac.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rac_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["rac_create", "rac_enforce", "rac_enforce_batch", "rac_enforce_multi",
                 "rac_destroy", "rac_strerror"]:
        assert must in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports_symbol(name):
    lib = ctypes.CDLL(rac.LIB_PATH)
    assert hasattr(lib, name), f"librac.so does not export {name}"
    assert name in rac.EXPORTED


def test_strerror_names_every_code():
    for code in [0, -1, -2, -3, -4, -5, -6, -7]:
        assert rac.lib.rac_strerror(code).decode() not in ("", "unknown error")


def _expect(code, fn):
    with pytest.raises(rac.RacError) as ei:
        fn()
    assert ei.value.code == code, str(ei.value)


E = np.array([[0, 1], [1, 2]], np.int32)
R = np.full((2, 4), 15, np.uint64)


def test_invalid_sizes():
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(0, 4, E, R))
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 0, E, R))
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 65, E, np.zeros((2, 65), np.uint64)))


def test_invalid_edges():
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 4, np.array([[0, 0]], np.int32), R[:1]))
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 4, np.array([[0, 3]], np.int32), R[:1]))
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 4, np.array([[-1, 2]], np.int32), R[:1]))
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 4, np.array([[0, 1], [1, 0]], np.int32), R))
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 4, np.array([[2, 1], [1, 2]], np.int32), R))


def test_relation_bits_beyond_d():
    bad = R.copy()
    bad[1, 2] = 1 << 4
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 4, E, bad))


def test_dense_must_be_symmetric():
    n, d = 2, 2
    Rd = np.zeros((n, d, n, d), np.uint8)
    Rd[0, 0, 1, 1] = 1      # allowed (x0=0, x1=1) ...
    # ... but the reverse block does not say so
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_dense(n, d, Rd, np.array([[0, 1]], np.int32)))


def test_invalid_options():
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 4, E, R, mode=2))
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 4, E, R, path=7))
    _expect(rac.RAC_EINVAL, lambda: rac.Net.from_bits(3, 4, E, R, max_sweeps=-1))


class FakeGpuTensor:
    """Stands in for a torch tensor on the GPU (CPU-only test of the wrapper's
    argument checks; nothing reaches the library)."""

    def __init__(self, shape, esize=8, dtype="torch.int64", device="cuda:0", contiguous=True,
                 is_cuda=True):
        self.shape, self._esize, self.dtype = tuple(shape), esize, dtype
        self.device, self._contig, self.is_cuda = device, contiguous, is_cuda

    def dim(self):
        return len(self.shape)

    def numel(self):
        return int(np.prod(self.shape))

    def element_size(self):
        return self._esize

    def is_contiguous(self):
        return self._contig

    def data_ptr(self):
        raise AssertionError("the wrapper must refuse before passing a pointer")


def _fake_net(n):
    net = rac.Net.__new__(rac.Net)
    net.handle, net.n, net.d, net.m = None, n, 8, 0
    return net


def _i32(numel, **kw):
    return FakeGpuTensor((numel,), esize=4, dtype="torch.int32", **kw)


@pytest.mark.parametrize("case", [
    "wrong_n", "one_dim", "out_shape", "on_cpu", "other_device", "not_contiguous",
    "four_byte_domains", "short_iters", "float_status"])
def test_device_entry_point_refuses_bad_tensors(case):
    n, B = 10, 6
    args = dict(d_in=FakeGpuTensor((B, n)), d_out=FakeGpuTensor((B, n)), d_iters=_i32(B),
                d_status=_i32(B))
    if case == "wrong_n":
        args["d_in"] = FakeGpuTensor((B, n - 1))
    elif case == "one_dim":
        args["d_in"] = FakeGpuTensor((B * n,))
    elif case == "out_shape":
        args["d_out"] = FakeGpuTensor((B - 1, n))
    elif case == "on_cpu":
        args["d_out"] = FakeGpuTensor((B, n), is_cuda=False, device="cpu")
    elif case == "other_device":
        args["d_iters"] = _i32(B, device="cuda:1")
    elif case == "not_contiguous":
        args["d_out"] = FakeGpuTensor((B, n), contiguous=False)
    elif case == "four_byte_domains":
        args["d_out"] = FakeGpuTensor((B, n), esize=4, dtype="torch.int32")
    elif case == "short_iters":
        args["d_iters"] = _i32(B - 1)
    elif case == "float_status":
        args["d_status"] = FakeGpuTensor((B,), esize=4, dtype="torch.float32")
    with pytest.raises(ValueError):
        _fake_net(n).enforce_batch_device(**args)


def test_group_device_entry_point_refuses_bad_tensors():
    grp = rac.Group.__new__(rac.Group)
    grp.nets = [_fake_net(4), _fake_net(7)]
    grp.offsets = np.array([0, 4, 11], np.int64)
    grp.handle = None
    with pytest.raises(ValueError):
        grp.enforce_device(FakeGpuTensor((10,)), _i32(2), _i32(2))
    with pytest.raises(ValueError):
        grp.enforce_device(FakeGpuTensor((11,)), _i32(1), _i32(2))
    with pytest.raises(ValueError):
        grp.enforce_device(FakeGpuTensor((11,), is_cuda=False), _i32(2), _i32(2))


def test_shipped_tuner_table_format():
    # every entry of the autotuner table shipped beside librac.so parses the
    # way the library reads it, once per key, with valid choices
    import re
    path = os.path.join(ROOT, "paper_2407_11388_amd", "rac_tune_gfx950.txt")
    keys = set()
    pat = re.compile(r"^gfx950/(single|batch)/d(\d+)/n(\d+)/dens(0\.05|0\.1|0\.25|0\.5|0\.75|1)/B(\d+) "
                     r"path=([1234]) items=(-?\d) handoff=(-?\d+) ms=(\d+\.\d+)$")
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            m = pat.match(line.rstrip("\n"))
            assert m, line
            kind, d, n, _, B, p, items, handoff, _ = m.groups()
            for v in (int(d), int(n), int(B)):
                assert v & (v - 1) == 0           # powers of 2
            assert not (kind == "single" and (p == "3" or B != "1"))
            assert -4 <= int(items) <= 4 and int(handoff) >= -1
            key = line.split()[0]
            assert key not in keys
            keys.add(key)
    assert any(k.startswith("gfx950/batch/d32/n1024/dens1/B1024") for k in keys)
