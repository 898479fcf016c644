"""Device-side generation of the large workloads (same bytes as the host
generator in kpgen/__init__.py; checked by a test on sampled users)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

import kpgen

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkpgen.so")
SRC = os.path.join(_HERE, "csrc", "kpgen.hip")
_lib = None


def build() -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-o", tmp, SRC])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, i64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
        L.kpgen_values.argtypes = [u64, i32, u64, i64, vp, vp, vp]
        L.kpgen_csr.argtypes = [u64, u64, i64, i32, i32, vp, vp, vp, vp]
        L.kpgen_colsum_dense.argtypes = [vp, i64, i32, vp, vp]
        L.kpgen_colsum_csr.argtypes = [vp, vp, i64, i32, vp, vp]
        _lib = L
    return _lib


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ok(rc):
    if rc != 0:
        raise RuntimeError(f"kpgen device call failed ({rc})")


_DEV_TABLES = {}


def _table(dist):
    import torch
    if dist == kpgen.DIST_UNIFORM:
        return None
    if dist not in _DEV_TABLES:
        _DEV_TABLES[dist] = torch.from_numpy(kpgen.dist_table(dist)).to("cuda")
    return _DEV_TABLES[dist]


def device_instance(c: int, run: int = 0, N=None):
    """Generate workload c on the GPU.  Returns (tensors dict, B, tree, meta);
    tensors: p, and b or (rowptr, col, val)."""
    import torch
    cfg = dict(kpgen.CONFIGS[c])
    Nn = cfg["N"] if N is None else int(N)
    M, K = cfg["M"], cfg["K"]
    seed = 1000 * c + run
    dist = {"uniform": kpgen.DIST_UNIFORM, "exp1": kpgen.DIST_EXP1,
            "lognormal": kpgen.DIST_LOGNORMAL}[cfg["p_dist"]]
    L = lib()
    st = _stream()
    p = torch.empty(Nn * M, dtype=torch.float32, device="cuda")
    tab = _table(dist)
    _ok(L.kpgen_values(seed, kpgen.S_P, 0, Nn * M, None if tab is None else tab.data_ptr(),
                       p.data_ptr(), st))
    sums = torch.zeros(K, dtype=torch.int64, device="cuda")
    out = dict(p=p)
    if cfg["csr_d"]:
        d = cfg["csr_d"]
        nrows = Nn * M
        col = torch.empty(nrows * d, dtype=torch.int32, device="cuda")
        val = torch.empty(nrows * d, dtype=torch.float32, device="cuda")
        rowptr = torch.empty(nrows + 1, dtype=torch.int64, device="cuda")
        _ok(L.kpgen_csr(seed, 0, nrows, K, d, col.data_ptr(), val.data_ptr(), rowptr.data_ptr(), st))
        _ok(L.kpgen_colsum_csr(col.data_ptr(), val.data_ptr(), nrows * d, K, sums.data_ptr(), st))
        out.update(rowptr=rowptr, col=col, val=val)
    else:
        b = torch.empty(Nn * M * K, dtype=torch.float32, device="cuda")
        _ok(L.kpgen_values(seed, kpgen.S_B, 0, Nn * M * K, None, b.data_ptr(), st))
        _ok(L.kpgen_colsum_dense(b.data_ptr(), Nn * M, K, sums.data_ptr(), st))
        out["b"] = b
    D = sums.cpu().numpy().astype(np.float64) * 2.0 ** -24
    B = kpgen.budgets(D, cfg["budget_frac"], M if cfg["budget_per_item_mean"] else 1)
    tree = kpgen.tree_hier_2_2_3(M) if cfg.get("hier") else kpgen.tree_topq(M, cfg["Q"])
    meta = dict(N=Nn, M=M, K=K, seed=seed, name=cfg["name"], dist=dist, csr_d=cfg["csr_d"])
    return out, B, tree, meta


def device_batched(run: int = 0, n: int = 256):
    """The batched ragged workload generated on the GPU: the same bytes and
    budgets as kpgen.batched_instances (dense U(0,1) p and b, B_k = 0.1 D_k,
    one top-Q cap).  Returns a list of (tensors, B, tree, meta)."""
    import torch
    seed = 1000 * 5 + run
    L = lib()
    st = _stream()
    out = []
    for s_, (N, M, K, Q, sd) in enumerate(kpgen.batched_shapes(seed, n)):
        p = torch.empty(N * M, dtype=torch.float32, device="cuda")
        b = torch.empty(N * M * K, dtype=torch.float32, device="cuda")
        _ok(L.kpgen_values(sd, kpgen.S_P, 0, N * M, None, p.data_ptr(), st))
        _ok(L.kpgen_values(sd, kpgen.S_B, 0, N * M * K, None, b.data_ptr(), st))
        sums = torch.zeros(K, dtype=torch.int64, device="cuda")
        _ok(L.kpgen_colsum_dense(b.data_ptr(), N * M, K, sums.data_ptr(), st))
        D = sums.cpu().numpy().astype(np.float64) * 2.0 ** -24
        B = kpgen.budgets(D, 0.1, 1)
        tree = kpgen.tree_topq(M, Q)
        meta = dict(N=N, M=M, K=K, Q=Q, seed=sd, name=f"c5 instance {s_}", dist=kpgen.DIST_UNIFORM, csr_d=0)
        out.append((dict(p=p, b=b), B, tree, meta))
    return out


def host_users(meta, B, tree, users):
    """Host-generated copy of the given users of a device instance (for the
    oracle), with the full instance's budgets."""
    users = np.asarray(users, np.int64)
    M, K, seed = meta["M"], meta["K"], meta["seed"]
    rows = (users[:, None] * M + np.arange(M)[None, :]).reshape(-1)
    p = kpgen.values(kpgen.u24(seed, kpgen.S_P, rows.astype(np.uint64)), meta["dist"])
    inst = kpgen.Instance(N=len(users), M=M, K=K, p=p, B=np.asarray(B, np.float64), tree=tree,
                          seed=seed, name=meta["name"] + " (sampled users)")
    if meta["csr_d"]:
        d = meta["csr_d"]
        col = kpgen.gen_csr_cols(seed, rows.astype(np.uint64), K, d).reshape(-1)
        vidx = (rows[:, None].astype(np.uint64) * np.uint64(d) + np.arange(d, dtype=np.uint64)[None, :]).reshape(-1)
        inst.col = col
        inst.val = kpgen.values(kpgen.u24(seed, kpgen.S_VAL, vidx), kpgen.DIST_UNIFORM)
        inst.rowptr = np.arange(len(rows) + 1, dtype=np.int64) * d
    else:
        idx = (rows[:, None] * K + np.arange(K)[None, :]).reshape(-1).astype(np.uint64)
        inst.b = kpgen.values(kpgen.u24(seed, kpgen.S_B, idx), kpgen.DIST_UNIFORM)
    return inst
