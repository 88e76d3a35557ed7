"""Host-side checks of the D3Q19 C ABI (no GPU): the library exports every function
include/btrt3.h declares, validates problems, and derives the 3x3 K1 of Eq. (30) and the k2 of
Eq. (62)."""
import os
import re

import numpy as np
import pytest

from paper_1902_09813_amd import btrt, btrt3
from paper_1902_09813_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "btrt3.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(btrt3_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(btrt3.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = btrt3.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def _inval(p):
    with pytest.raises(btrt.BtrtError) as e:
        p.validate()
    assert e.value.code == btrt.E_INVAL
    return str(e.value)


def test_validation():
    good = dict(A0=(0.02, 0.0, 0.0, 0.02, 0.0, 0.02))
    btrt3.Problem3(4, 5, 6, **good).validate()
    _inval(btrt3.Problem3(0, 5, 6, **good))
    _inval(btrt3.Problem3(4, 5, 6, precision=btrt.F16DEV, **good))
    _inval(btrt3.Problem3(1024, 1024, 1024, **good))  # 19 planes beyond 2^31 elements
    _inval(btrt3.Problem3(4, 4, 4, A0=(0.02, 0.03, 0.0, 0.02, 0.0, 0.02)))  # not positive definite
    _inval(btrt3.Problem3(4, 4, 4, A0=(0.02, 0.0, 0.0, 0.02, 0.0, -0.01)))
    _inval(btrt3.Problem3(4, 4, 4, beta=-1.0, **good))
    _inval(btrt3.Problem3(4, 4, 4, flux_a=(0.0, np.nan, 0.0), **good))
    _inval(btrt3.Problem3(4, 4, 4, k0=2.0, **good))
    _inval(btrt3.Problem3(4, 4, 4, k2=(1, 1, 1, 1, 1, 1, 1, 1, 2.5), **good))
    _inval(btrt3.Problem3(4, 4, 4, k2=(1, 3, 1, 1, 1, 1, 1, 1, 1), **good))  # (k2_12 + k2_21)/2 = 2
    btrt3.Problem3(4, 4, 4, k2=(1, 3, 1, -2, 1, 1, 1, 1, 1), **good).validate()  # 0.5: only the mean counts
    _inval(btrt3.Problem3(4, 4, 4, bc_type=(1, 0, 0, 0, 0, 0), **good))
    _inval(btrt3.Problem3(4, 4, 4, bc_type=(1,) * 6, bc_value=(0, 0, 0, np.inf, 0, 0), **good))
    assert "HBB" in _inval(btrt3.Problem3(4, 4, 4, A0=(0.02, 0.0, 0.0, 0.03, 0.0, 0.02), k2="hbb"))
    _inval(btrt3.Problem3(4, 4, 4, A0=(0.02, 0.0, 0.0, 0.02, 0.0, 0.02), beta=1.0, k2="hbb"))
    bad = np.zeros((4, 4, 4))
    bad[1, 2, 3] = np.nan
    assert "node 27" in _inval(btrt3.Problem3(4, 4, 4, source=bad, **good))


def test_eq30_and_eq62_constants():
    w = W.d3_walls()
    info = btrt3.problem_from_workload3(w).validate()
    A = W.D3_A0
    np.testing.assert_allclose(np.array(info.K1).reshape(3, 3), np.linalg.inv(3 * A + 0.5 * np.eye(3)), rtol=1e-14)
    assert info.k1_per_node == 1
    assert info.bytes_per_node_launch == (19 * 2 + 2 + 1) * 8
    alpha = 0.1
    info = btrt3.Problem3(4, 4, 4, A0=(alpha, 0, 0, alpha, 0, alpha), k2="hbb").validate()
    k1 = 1.0 / (3 * alpha + 0.5)
    assert info.K1[0] == pytest.approx(k1, rel=1e-15) and info.K1[1] == 0.0
    assert list(info.K2) == pytest.approx([8 * (k1 - 2) / (3 * (k1 - 4))] * 9, rel=1e-14)
    assert btrt3.Problem3(4, 4, 4, precision=btrt.F32, **dict(A0=(0.02, 0, 0, 0.02, 0, 0.02))).validate() \
        .bytes_per_node_launch == 40 * 4
