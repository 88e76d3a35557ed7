"""Host-side checks of the C-ABI library (no GPU): it loads, exports every symbol that
include/btrt.h declares, validates problems, and derives the constants of Eq. (30) and
Eq. (62) as the paper states them."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "btrt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(btrt_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(btrt.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = btrt.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_strerror_covers_codes():
    L = btrt.lib()
    for code in range(6):
        assert L.btrt_strerror(code).decode()
    assert L.btrt_strerror(99).decode() == "unknown error code"


def _expect_inval(p):
    with pytest.raises(btrt.BtrtError) as e:
        p.validate()
    assert e.value.code == btrt.E_INVAL
    return str(e.value)


def test_validation_rejects_bad_problems():
    good = dict(A0=(0.01, 0.0, 0.01))
    _expect_inval(btrt.Problem(0, 4, **good))
    _expect_inval(btrt.Problem(4, -1, **good))
    _expect_inval(btrt.Problem(4, 4, precision=7, **good))
    _expect_inval(btrt.Problem(70000, 70000, **good))  # more than 2^31 - 1 nodes
    _expect_inval(btrt.Problem(4, 4, A0=(0.01, 0.02, 0.01)))  # not positive definite
    _expect_inval(btrt.Problem(4, 4, A0=(-0.01, 0.0, 0.01)))
    _expect_inval(btrt.Problem(4, 4, beta=-1.0, **good))
    _expect_inval(btrt.Problem(4, 4, flux_a=(np.nan, 0.0), **good))
    _expect_inval(btrt.Problem(4, 4, k0=2.0, **good))
    _expect_inval(btrt.Problem(4, 4, k0=0.0, **good))
    _expect_inval(btrt.Problem(4, 4, k2=2.5, **good))
    _expect_inval(btrt.Problem(4, 4, k2=(1.0, -1.0, -1.5, 1.0), **good))  # (k2_12 + k2_21)/2 < 0
    _expect_inval(btrt.Problem(4, 4, check_interval=0, **good))
    # A periodic side must be paired with the opposite side.
    _expect_inval(btrt.Problem(4, 4, bc_type=(btrt.PERIODIC, btrt.DIRICHLET, 0, 0), **good))
    _expect_inval(btrt.Problem(4, 4, bc_type=(1, 1, 1, 1), bc_value=(0, np.inf, 0, 0), **good))
    # Eq. (62) only for a constant isotropic A.
    assert "K2_HBB" in _expect_inval(btrt.Problem(4, 4, A0=(0.01, 0.002, 0.01), k2="hbb"))
    _expect_inval(btrt.Problem(4, 4, A0=(0.01, 0.0, 0.01), beta=1.0, k2="hbb"))
    _expect_inval(btrt.Problem(4, 4, A0=(0.01, 0.0, 0.02), k2="hbb"))
    bad_field = np.zeros((4, 4))
    bad_field[2, 3] = np.nan
    _expect_inval(btrt.Problem(4, 4, source=bad_field, **good))
    p = btrt.Problem(4, 4, **good)
    p.dterm.kind = 3
    _expect_inval(p)


def test_eq30_and_eq62_constants():
    # Eq. (30): K1 = (A / c_s^2 + I / 2)^-1; Eq. (62) for the isotropic case.
    A = np.array([[0.02, 0.008], [0.008, 0.01]])
    info = btrt.problem_from_workload(W.c2()).validate()
    np.testing.assert_allclose(np.array(info.K1).reshape(2, 2), np.linalg.inv(3 * A + 0.5 * np.eye(2)), rtol=1e-15)
    info = btrt.problem_from_workload(W.c1("hbb")).validate()
    k1 = 1.0 / 0.53
    assert info.K1[0] == pytest.approx(k1, rel=1e-15) and info.K1[1] == 0.0
    assert list(info.K2) == pytest.approx([8 * (k1 - 2) / (3 * (k1 - 4))] * 4, rel=1e-14)
    assert info.K2[0] == pytest.approx(1.0 / 7.0, rel=1e-13)  # D = 0.01: tau = 0.53, k2 = 1/7
    info = btrt.problem_from_workload(W.c3()).validate()
    assert info.k1_per_node == 1


def test_bytes_and_workspace():
    for prec, es in ((btrt.F64, 8), (btrt.F32, 4)):
        p = btrt.problem_from_workload(W.c3(), precision=prec)
        info = p.validate()
        assert info.bytes_per_node_launch == 20 * es
        assert info.workspace_bytes == p.workspace_size()
        # Two population buffers of 9 planes dominate the footprint.
        assert info.workspace_bytes >= 2 * 9 * 4096 * 4096 * es
    # A ragged width is padded to 256-byte rows.
    assert btrt.Problem(100, 3, A0=(0.01, 0, 0.01)).validate().pitch == 128
    assert btrt.Problem(100, 3, precision=btrt.F32, A0=(0.01, 0, 0.01)).validate().pitch == 128
    assert btrt.Problem(65, 3, A0=(0.01, 0, 0.01)).validate().pitch == 96


def test_space_dependent_tensor_and_growing_source_reach_the_library():
    # The A0 field and the source growth travel through the structures: a non-SPD node is
    # named, the field adds three planes to the workspace and to the bytes per launch, and
    # batches refuse both (checked on the host, before any device work).
    w = W.c6(1e-3, 16)
    p = btrt.problem_from_workload(w)
    info = p.validate()
    assert info.k1_per_node == 1
    assert info.bytes_per_node_launch == (18 + 2 + 1 + 3) * 8  # plus the source field and A0(x)
    plain = btrt.Problem(16, 16, A0=(0.01, 0.0, 0.01), source=w.source[1])
    assert p.workspace_size() - plain.workspace_size() >= 3 * 16 * 16 * 8
    bad = w.A0_field.copy()
    bad[3, 5, 1] = 1.0  # a12^2 > a11 a22 at node (5, 3)
    msg = _expect_inval(btrt.Problem(16, 16, A0_field=bad, source=w.source))
    assert "node 53" in msg
    _expect_inval(btrt.Problem(16, 16, A0_field=w.A0_field, k2="hbb"))
    _expect_inval(btrt.Problem(16, 16, A0=(0.01, 0.0, 0.01), source=("field", w.source[1], np.inf)))


def test_general_model_parameters_reach_the_library():
    # The power-law flux and the phi-dependent source of the Burgers-Fisher problem (Eq. (67))
    # pass validation with plain storage, and their exponents and storage formats are checked
    # on the host.
    w = W.bfe(n=20)
    p = btrt.problem_from_workload(w)
    info = p.validate()
    k1 = 1.0 / (3 * w.A0[0] + 0.5)
    assert info.K1[0] == pytest.approx(k1, rel=1e-15)
    assert info.K2[0] == pytest.approx(8 * (k1 - 2) / (3 * (k1 - 4)), rel=1e-14)
    assert (p.flux.c[0], p.flux.q, p.source.r, p.source.p) == (w.flux_c[0], w.flux_q, w.src_r, w.src_p)
    btrt.problem_from_workload(w, precision=btrt.F32).validate()
    good = dict(A0=(0.01, 0.0, 0.01))
    assert "exponent q" in _expect_inval(btrt.Problem(4, 4, flux_c=(0.1, 0.0), flux_q=0.5, **good))
    _expect_inval(btrt.Problem(4, 4, flux_c=(0.1, 0.0), flux_q=np.nan, **good))
    _expect_inval(btrt.Problem(4, 4, flux_c=(np.inf, 0.0), flux_q=2.0, **good))
    assert "exponent p" in _expect_inval(btrt.Problem(4, 4, src_r=0.01, src_p=0.0, **good))
    _expect_inval(btrt.Problem(4, 4, src_r=np.nan, **good))
    for prec in (btrt.F16DEV, btrt.BF16DEV):
        assert "BTRT_F64 or BTRT_F32" in _expect_inval(btrt.Problem(4, 4, precision=prec, src_r=0.01, **good))
        _expect_inval(btrt.Problem(4, 4, precision=prec, flux_c=(0.1, 0.0), flux_q=2.0, **good))
    # Exponents are read only where their term is present.
    btrt.Problem(4, 4, flux_q=0.0, src_p=-1.0, **good).validate()


def test_general_d_reaches_the_library():
    good = dict(A0=(0.01, 0.0, 0.01))
    btrt.Problem(4, 4, dterm=(1.0, 0.2, 3.0), **good).validate()
    btrt.Problem(4, 4, precision=btrt.F32, dterm=(0.5, 0.0, 0.0), **good).validate()  # s unread when e = 0
    assert "exponent s" in _expect_inval(btrt.Problem(4, 4, dterm=(1.0, 0.2, 0.5), **good))
    _expect_inval(btrt.Problem(4, 4, dterm=(np.nan, 0.0, 1.0), **good))
    _expect_inval(btrt.Problem(4, 4, dterm=(1.0, np.inf, 2.0), **good))
    for prec in (btrt.F16DEV, btrt.BF16DEV):
        assert "BTRT_F64 or BTRT_F32" in _expect_inval(btrt.Problem(4, 4, precision=prec, dterm=(1.0, 0.1, 2.0), **good))
