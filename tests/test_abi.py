"""The C ABI on the CPU: the library loads, exports every symbol the header
declares, and host-side validation rejects bad problems before any GPU call."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2002_00352_amd as kp

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "kp.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kp_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = kp.lib()
    names = _declared()
    assert "kp_eval_dual" in names and "kp_scd_sweep" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_limits():
    assert kp.lib().kp_max_items() == 64
    assert kp.lib().kp_max_knapsacks_scd() >= 20


def _host_problem(N=4, M=3, K=2, B=(1.0, 1.0), parent=(-1,), cap=(1,), leaf=None, fmt=0, row_nnz=0):
    s = kp.kp_problem()
    s.N, s.M, s.K = N, M, K
    keep = []
    dummy = np.zeros(16, np.float32)
    keep.append(dummy)
    s.p = dummy.ctypes.data
    s.b = dummy.ctypes.data
    s.b_format = fmt
    s.b_row_nnz = row_nnz
    if fmt == 1:
        rp = np.arange(N * M + 1, dtype=np.int64)
        keep.append(rp)
        s.b_rowptr, s.b_col, s.b_val = rp.ctypes.data, dummy.ctypes.data, dummy.ctypes.data
    Ba = np.array(B, np.float64)
    par = np.array(parent, np.int32)
    cp = np.array(cap, np.int32)
    lf = np.array(leaf if leaf is not None else [0] * M, np.int32)
    keep += [Ba, par, cp, lf]
    s.B, s.parent, s.cap, s.leaf_of_item = Ba.ctypes.data, par.ctypes.data, cp.ctypes.data, lf.ctypes.data
    s.L = len(par)
    return s, keep


@pytest.mark.parametrize("kw,code", [
    (dict(B=(1.0, 0.0)), -1),                 # budget must be > 0
    (dict(B=(1.0, float("nan"))), -1),
    (dict(cap=(0,)), -1),                     # C_l >= 1
    (dict(parent=(0,)), -1),                  # self loop
    (dict(parent=(1, 0), cap=(1, 1)), -1),    # cycle
    (dict(leaf=[0, 5, 0]), -1),               # leaf out of range
    (dict(M=65, leaf=[0] * 65), -5),          # over the item limit
    (dict(N=-1), -1),
    (dict(K=0, B=(1.0,)), -1),
    (dict(row_nnz=1), -1),                    # a row count is declared for CSR costs only
    (dict(fmt=1, row_nnz=3), -1),             # 1 or 2 entries per item row
    (dict(fmt=1, row_nnz=-1), -1),
])
def test_validation_rejects_bad_problems(kw, code):
    L = kp.lib()
    ctx = ctypes.c_void_p()
    assert L.kp_create(ctypes.byref(ctx), None, 0) == 0
    s, keep = _host_problem(**kw)
    lam = np.zeros(4)
    rc = L.kp_eval_dual(ctx, ctypes.byref(s), lam.ctypes.data, None, None, None, None)
    assert rc == code, L.kp_last_error()
    assert L.kp_last_error()
    L.kp_destroy(ctx)


def test_scd_rejects_too_many_knapsacks():
    L = kp.lib()
    ctx = ctypes.c_void_p()
    L.kp_create(ctypes.byref(ctx), None, 0)
    K = L.kp_max_knapsacks_scd() + 1
    s, keep = _host_problem(K=K, B=tuple([1.0] * K))
    lam = np.zeros(K)
    rc = L.kp_scd_sweep(ctx, ctypes.byref(s), lam.ctypes.data, lam.ctypes.data, None, None, None)
    assert rc == -5
    L.kp_destroy(ctx)


def test_tree_from_sets_laminar_and_not():
    par, cap, leaf = kp.kp_tree_from_sets(6, [[0, 1, 2, 3, 4, 5], [0, 1, 2], [3, 4, 5], [0]], [3, 2, 2, 1])
    # root is the full set; {0,1,2} and {3,4,5} hang below it; {0} below {0,1,2}
    assert list(cap) == [3, 2, 2, 1]
    assert list(par) == [-1, 0, 0, 1]
    assert list(leaf) == [3, 1, 1, 2, 2, 2]
    # identical sets merge with the smaller cap
    par, cap, leaf = kp.kp_tree_from_sets(3, [[0, 1], [1, 0]], [2, 1])
    assert list(cap) == [1] and list(leaf) == [0, 0, -1]
    with pytest.raises(kp.KPError) as e:
        kp.kp_tree_from_sets(4, [[0, 1], [1, 2]], [1, 1])
    assert e.value.status == -2


def test_product_path_has_no_cpu_fallback(monkeypatch, tmp_path):
    """Without the built library the binding raises instead of computing."""
    monkeypatch.setattr(kp, "_lib", None)
    monkeypatch.setattr(kp, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        kp.lib()
