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
