"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and its host-only helper agrees with the oracle's plane lists."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import crystal

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "laueot.h")
LIB = os.path.join(ROOT, "paper_2404_06478_amd", "liblaueot.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(laue_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblaueot.so is not built (python -m paper_2404_06478_amd.build)")
    from paper_2404_06478_amd import _abi
    return _abi.load(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    from paper_2404_06478_amd import _abi
    assert set(names) == set(_abi.SIGNATURES), "binding and header disagree"


def test_version(lib):
    assert lib.laue_version() == 200


@pytest.mark.parametrize("a,cen,nmax", [(2.87, "I", 14), (2.87, "I", 30), (3.52, "F", 40), (4.05, "F", 30)])
def test_plane_list_matches_oracle(lib, a, cen, nmax):
    n = ctypes.c_int32()
    assert lib.laue_planes_cubic(a, cen.encode(), nmax, ctypes.byref(n), None, None, None, None) == 0
    hkl = np.zeros((n.value, 3), np.int32)
    w = np.zeros((n.value, 3), np.float32)
    d = np.zeros(n.value, np.float32)
    prev = np.zeros(n.value, np.int32)
    assert lib.laue_planes_cubic(a, cen.encode(), nmax, ctypes.byref(n), hkl.ctypes.data,
                                 w.ctypes.data, d.ctypes.data, prev.ctypes.data) == 0
    ref = crystal.cubic_planes(a, cen, nmax)
    assert np.array_equal(hkl, ref["hkl"])
    assert np.array_equal(prev, ref["harmonic_prev"])
    assert np.array_equal(w, ref["w"].astype(np.float32))
    assert np.array_equal(d, ref["d"].astype(np.float32))


def test_bad_arguments_are_rejected(lib):
    n = ctypes.c_int32()
    assert lib.laue_planes_cubic(2.87, b"X", 14, ctypes.byref(n), None, None, None, None) == -1
    assert b"centering" in lib.laue_last_error()
    assert lib.laue_planes_cubic(-1.0, b"I", 14, ctypes.byref(n), None, None, None, None) == -1
    assert lib.laue_planes_cubic(2.87, b"I", 14, None, None, None, None, None) == -1
    from paper_2404_06478_amd import _abi
    g = _abi.laue_geometry()
    g.n_rot = 0
    assert lib.laue_forward_workspace_size(ctypes.byref(g), 10, 10) == 0
    assert lib.laue_sinkhorn_workspace_size(ctypes.byref(g), 10, 10, 1) == 0


def test_ot_defaults_match_the_oracle(lib):
    """laue_ot_defaults (host only): the outlier row and column of Sec. 7 equal
    the oracle's c_out (3-sigma miss) and T_b = ceil(0.4 |J|); bad input is
    rejected."""
    from oracle import cost, sinkhorn
    from paper_2404_06478_amd import _abi
    p = _abi.laue_ot_params()
    for sigma, D, J in ((1.0, 150.0, 496312), (0.3, 150.0, 238), (0.4, 160.0, 0)):
        assert lib.laue_ot_defaults(sigma, D, J, ctypes.byref(p)) == 0
        assert p.c_out == pytest.approx(cost.c_out(sigma, D), rel=1e-14)
        assert p.c_sink == p.c_out and p.c_unm == 0.0
        assert p.t_b == sinkhorn.default_tb(J)
        assert p.eps == pytest.approx(2.0 * sigma ** 2, rel=1e-15)
        assert (p.tol, p.n_max, p.rho, p.outlier_model) == (1e-5, 2000, 0, 0)
    assert lib.laue_ot_defaults(0.0, 150.0, 10, ctypes.byref(p)) == _abi.LAUE_EINVAL
    assert lib.laue_ot_defaults(1.0, 150.0, -1, ctypes.byref(p)) == _abi.LAUE_EINVAL
