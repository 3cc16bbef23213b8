"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import oracle
from paper_2510_11513_amd import snx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "snx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(snx_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = ct.CDLL(snx.LIB_PATH)
    names = header_functions()
    assert len(names) >= 16
    for name in names:
        assert hasattr(L, name), name
    assert set(snx.EXPORTS) <= set(names)


@pytest.mark.parametrize("npol,naz", [(1, 1), (2, 2), (3, 4), (4, 8), (4, 4), (8, 8)])
def test_library_quadrature_matches_oracle(npol, naz):
    om, w = snx.quadrature_product(npol, naz)
    omr, wr = oracle.quadrature(npol, naz)
    assert np.abs(om - omr).max() < 1e-15
    assert np.abs(w - wr).max() < 1e-15


def test_library_quadrature_rejects_bad_sizes():
    om = np.zeros((8, 3))
    w = np.zeros(8)
    assert snx.load().snx_quadrature_product(0, 1, om, w) == -1
    assert snx.load().snx_quadrature_product(1, 0, om, w) == -1


def test_create_without_device_fails_cleanly():
    """On a host without a GPU, creating a problem reports an error instead of crashing."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ct.c_void_p()
    rc = snx.load().snx_create(ct.byref(h), 0)
    assert rc in (-1, -5)
    assert snx.load().snx_last_error(None)
