"""CPU oracle for the per-user subproblem sweep (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke check and the benchmark's cpu_baseline leg may import
this package.  The GPU product path never imports it; the two share no code.

`kp_oracle.c` holds the paper's arithmetic (scoring, Alg.1, the dual
evaluation, DD's Eq.14, Alg.3/4 Map and Reduce, post-processing, Alg.5) in
plain C; this module is a ctypes wrapper around it.  `exact.py` holds the
brute-force and exact-arithmetic tools that pin the C oracle.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kp_oracle.c")
_LIB = os.path.join(_HERE, "libkp_oracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-shared", "-fPIC", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("M", ctypes.c_int32), ("K", ctypes.c_int32),
        ("p", ctypes.c_void_p), ("b_format", ctypes.c_int32), ("b", ctypes.c_void_p),
        ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
        ("B", ctypes.c_void_p), ("L", ctypes.c_int32), ("parent", ctypes.c_void_p),
        ("cap", ctypes.c_void_p), ("leaf_of_item", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_eval.argtypes = [P, vp, vp, vp, vp, vp, vp]
        L.orc_eval.restype = ctypes.c_int
        L.orc_dd_update.argtypes = [ctypes.c_int, d, vp, vp, vp]
        L.orc_dd_update.restype = None
        L.orc_scd_map.argtypes = [P, vp, i64, i64, vp, vp, vp, vp, i64]
        L.orc_scd_map.restype = i64
        L.orc_scd_reduce.argtypes = [i64, vp, vp, d]
        L.orc_scd_reduce.restype = d
        L.orc_scd_sweep.argtypes = [P, vp, vp]
        L.orc_scd_sweep.restype = ctypes.c_int
        L.orc_scd_sweep_mask.argtypes = [P, vp, vp, vp]
        L.orc_scd_sweep_mask.restype = ctypes.c_int
        L.orc_consumption_at.argtypes = [P, vp, ctypes.c_int, d, i64, i64]
        L.orc_consumption_at.restype = d
        L.orc_fixup.argtypes = [P, vp, ctypes.c_int, vp, vp, vp, vp, vp, i64]
        L.orc_fixup.restype = ctypes.c_int
        L.orc_alg5_map_user.argtypes = [P, vp, i64, ctypes.c_int, vp, vp, vp]
        L.orc_alg5_map_user.restype = ctypes.c_int
        L.orc_max_items.restype = ctypes.c_int
        L.orc_scores.argtypes = [P, vp, i64, i64, vp]
        L.orc_scores.restype = None
        L.orc_alg1.argtypes = [P, vp, vp]
        L.orc_alg1.restype = None
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads of the oracle's loops over users (results do not depend on
    it); returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class OracleProblem:
    """Holds contiguous host arrays of an instance and the C struct over them."""

    def __init__(self, inst):
        self.inst = inst
        self.p = np.ascontiguousarray(inst.p, np.float32)
        self.B = np.ascontiguousarray(inst.B, np.float64)
        t = inst.tree
        self.parent = np.ascontiguousarray(t.parent, np.int32)
        self.cap = np.ascontiguousarray(t.cap, np.int32)
        self.leaf = np.ascontiguousarray(t.leaf_of_item, np.int32)
        s = _Problem()
        s.N, s.M, s.K = inst.N, inst.M, inst.K
        s.p = _ptr(self.p)
        if inst.b is not None:
            self.b = np.ascontiguousarray(inst.b, np.float32)
            s.b_format, s.b = 0, _ptr(self.b)
        else:
            self.rowptr = np.ascontiguousarray(inst.rowptr, np.int64)
            self.col = np.ascontiguousarray(inst.col, np.int32)
            self.val = np.ascontiguousarray(inst.val, np.float32)
            s.b_format = 1
            s.rowptr, s.col, s.val = _ptr(self.rowptr), _ptr(self.col), _ptr(self.val)
        s.B = _ptr(self.B)
        s.L = len(self.parent)
        s.parent, s.cap, s.leaf_of_item = _ptr(self.parent), _ptr(self.cap), _ptr(self.leaf)
        self.s = s

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _prob(inst_or_prob) -> OracleProblem:
    return inst_or_prob if isinstance(inst_or_prob, OracleProblem) else OracleProblem(inst_or_prob)


def eval_dual(inst, lam, want_x=True, want_G=False):
    """x (uint8 [N*M]), R [K], g, P (and G [N]) at lambda (Eq.5, Alg.2)."""
    pr = _prob(inst)
    s = pr.s
    lam = np.ascontiguousarray(lam, np.float64)
    x = np.zeros(s.N * s.M, np.uint8) if want_x else None
    G = np.zeros(s.N, np.float64) if want_G else None
    R = np.zeros(s.K, np.float64)
    g, P = ctypes.c_double(), ctypes.c_double()
    rc = lib().orc_eval(pr.ref, _ptr(lam), _ptr(x), _ptr(R), ctypes.addressof(g),
                        ctypes.addressof(P), _ptr(G))
    if rc != 0:
        raise ValueError("oracle: M too large")
    out = dict(x=x, R=R, g=g.value, P=P.value)
    if want_G:
        out["G"] = G
    return out


def scores(inst, lam, u0=0, u1=None):
    """Cost-adjusted profits p~ of users [u0,u1) as fp64 [(u1-u0), M]."""
    pr = _prob(inst)
    u1 = pr.s.N if u1 is None else u1
    lam = np.ascontiguousarray(lam, np.float64)
    out = np.zeros((u1 - u0) * pr.s.M, np.float64)
    lib().orc_scores(pr.ref, _ptr(lam), int(u0), int(u1), _ptr(out))
    return out.reshape(u1 - u0, pr.s.M)


def alg1(inst, z):
    """Algorithm 1 on explicit values z[M] under the instance's local constraints."""
    pr = _prob(inst)
    z = np.ascontiguousarray(z, np.float64)
    x = np.zeros(pr.s.M, np.uint8)
    lib().orc_alg1(pr.ref, _ptr(z), _ptr(x))
    return x


def dd_update(lam, alpha, R, B):
    lam = np.array(lam, np.float64)
    R = np.ascontiguousarray(R, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    lib().orc_dd_update(len(lam), float(alpha), _ptr(R), _ptr(B), _ptr(lam))
    return lam


def scd_map(inst, lam, u0=0, u1=None):
    """All (k, user, v1, v2) pairs emitted by Alg.4's Map for users [u0,u1)."""
    pr = _prob(inst)
    s = pr.s
    u1 = s.N if u1 is None else u1
    lam = np.ascontiguousarray(lam, np.float64)
    cap = max(16, (u1 - u0) * s.K * 4)
    while True:
        kk = np.zeros(cap, np.int32)
        uu = np.zeros(cap, np.int64)
        v1 = np.zeros(cap, np.float64)
        v2 = np.zeros(cap, np.float64)
        n = lib().orc_scd_map(pr.ref, _ptr(lam), u0, u1, _ptr(kk), _ptr(uu), _ptr(v1), _ptr(v2), cap)
        if n < 0:
            raise ValueError("oracle: M too large")
        if n <= cap:
            return kk[:n], uu[:n], v1[:n], v2[:n]
        cap = n


def scd_reduce(v1, v2, Bk):
    v1 = np.array(v1, np.float64)
    v2 = np.array(v2, np.float64)
    return lib().orc_scd_reduce(len(v1), _ptr(v1), _ptr(v2), float(Bk))


def scd_sweep(inst, lam, ks=None):
    """lambda^{t+1} from lambda^t: one synchronous coordinate-descent iteration
    (restricted to coordinates ks when given; the others are kept)."""
    pr = _prob(inst)
    lam = np.ascontiguousarray(lam, np.float64)
    out = np.zeros(pr.s.K, np.float64)
    mask = None
    if ks is not None:
        mask = np.zeros(pr.s.K, np.uint8)
        mask[list(ks)] = 1
    rc = lib().orc_scd_sweep_mask(pr.ref, _ptr(lam), _ptr(out), _ptr(mask))
    if rc != 0:
        raise RuntimeError(f"oracle scd_sweep failed ({rc})")
    return out


def consumption_at(inst, lam, k, value, u0=0, u1=None):
    pr = _prob(inst)
    u1 = pr.s.N if u1 is None else u1
    lam = np.ascontiguousarray(lam, np.float64)
    return lib().orc_consumption_at(pr.ref, _ptr(lam), int(k), float(value), int(u0), int(u1))


def fixup(inst, lam, mode=0, want_x=True):
    """Post-processing for feasibility; mode 0 = violated-consumer prefix, 1 = literal."""
    pr = _prob(inst)
    s = pr.s
    lam = np.ascontiguousarray(lam, np.float64)
    x = np.zeros(s.N * s.M, np.uint8) if want_x else None
    R = np.zeros(s.K, np.float64)
    P = ctypes.c_double()
    nres = ctypes.c_int64()
    lst = np.zeros(s.N, np.int64)
    rc = lib().orc_fixup(pr.ref, _ptr(lam), int(mode), _ptr(x), ctypes.addressof(P), _ptr(R),
                         ctypes.addressof(nres), _ptr(lst), s.N)
    if rc != 0:
        raise ValueError("oracle: M too large")
    return dict(x=x, P=P.value, R=R, n_reset=nres.value, reset=lst[:nres.value])


def alg5_map_user(inst, lam, i, Q):
    pr = _prob(inst)
    lam = np.ascontiguousarray(lam, np.float64)
    K = pr.s.K
    kk = np.zeros(K, np.int32)
    v1 = np.zeros(K, np.float64)
    v2 = np.zeros(K, np.float64)
    n = lib().orc_alg5_map_user(pr.ref, _ptr(lam), int(i), int(Q), _ptr(kk), _ptr(v1), _ptr(v2))
    if n < 0:
        raise ValueError("Alg.5 needs M == K")
    return kk[:n], v1[:n], v2[:n]


def scd_sweep_alg5(inst, lam, Q):
    """One SCD iteration whose map is Alg.5 (Sec. 5.1) for every user (the
    setting M = K, item j consuming only knapsack j, one top-Q cap) and whose
    reduce is Alg.4's: per knapsack, the pairs in user order, then the
    threshold of scd_reduce."""
    pr = _prob(inst)
    K = pr.s.K
    lam = np.ascontiguousarray(lam, np.float64)
    v1s = [[] for _ in range(K)]
    v2s = [[] for _ in range(K)]
    for i in range(pr.s.N):
        kk, a, b = alg5_map_user(pr, lam, i, Q)
        for k, x, y in zip(kk.tolist(), a.tolist(), b.tolist()):
            v1s[k].append(x)
            v2s[k].append(y)
    return np.array([scd_reduce(v1s[k], v2s[k], pr.B[k]) for k in range(K)], np.float64)


def interp_delta(lam):
    """Central bucket half-width of the interpolated reduce (reading A17):
    a power of two 2^-20 of the multiplier (of 2^-20 when the multiplier is
    smaller), the minimal bucket size around lambda_k^t of Sec. 5.2."""
    return np.array([math.ldexp(1.0, math.frexp(max(float(l), 2.0 ** -20))[1] - 1 - 20) for l in lam])


def _bucket_ids(v1, center, delta):
    """Reading A17 of Sec. 5.2's bucket id: 0 when |v1 - center| < delta,
    else sign * (1 + floor(log2(|v1 - center| / delta))), capped at 31; the
    difference is the FP64 one and delta a power of two."""
    d = np.asarray(v1, np.float64) - center
    a = np.abs(d)
    ids = np.zeros(len(d), np.int64)
    big = a >= delta
    if big.any():
        ea = np.frexp(a[big])[1].astype(np.int64)
        ed = math.frexp(delta)[1]
        ids[big] = np.minimum(31, 1 + (ea - ed)) * np.where(d[big] < 0, -1, 1)
    return ids


def scd_reduce_interp(v1, v2, Bk, center, delta):
    """Sec. 5.2's approximate reduce: v2 summed per bucket of v1 (the uneven
    buckets of _bucket_ids around center = lambda_k^t); 0 when the total fits
    B_k, else the bucket where the running sum from the top first exceeds
    B_k, and inside it the point where a linear spread of its sum over its
    interval [lo, hi] would bring the running sum to B_k:
    v = hi - (B_k - above) / S_b * (hi - lo), with lo clamped at 0."""
    v1 = np.asarray(v1, np.float64)
    v2 = np.asarray(v2, np.float64)
    total = 0.0
    for x in v2:
        total = total + float(x)
    if total <= Bk:
        return 0.0
    ids = _bucket_ids(v1, center, delta)
    sums = {}
    for i, x in zip(ids.tolist(), v2.tolist()):
        sums[i] = sums.get(i, 0.0) + x
    above = 0.0
    for b in range(31, -32, -1):
        if b not in sums:
            continue
        if above + sums[b] > Bk:
            if b == 0:
                lo, hi = center - delta, center + delta
            elif b > 0:
                lo, hi = center + math.ldexp(delta, b - 1), center + math.ldexp(delta, b)
            else:
                lo, hi = center - math.ldexp(delta, -b), center - math.ldexp(delta, -b - 1)
            lo = max(lo, 0.0)
            frac = (Bk - above) / sums[b]
            width = hi - lo
            v = hi - frac * width
            return max(v, lo)
        above = above + sums[b]
    return 0.0


def scd_sweep_interp(inst, lam, ks=None):
    """One SCD iteration whose reduce is Sec. 5.2's bucket interpolation
    (the map is Alg.4's, as in scd_sweep) around lambda^t with the central
    half-widths of interp_delta, restricted to coordinates ks when given."""
    pr = _prob(inst)
    lam = np.ascontiguousarray(lam, np.float64)
    delta = interp_delta(lam)
    kk, uu, v1, v2 = scd_map(pr, lam)
    out = lam.copy()
    for k in range(pr.s.K):
        if ks is not None and k not in ks:
            continue
        sel = kk == k
        out[k] = scd_reduce_interp(v1[sel], v2[sel], float(pr.B[k]), float(lam[k]), float(delta[k]))
    return out


def presolve(inst, users, max_iter=100, lam0=None):
    """Pre-solving by sampling (Sec. 5.3): SCD on the sub-instance of the
    sampled users with every budget scaled by n / N, from lam0 until the
    multipliers repeat or max_iter sweeps.  Returns (lambda, sweeps)."""
    users = np.asarray(users, np.int64)
    n, N = len(users), inst.N
    scale = float(n) / float(N)
    sub = inst.subset(users, B=inst.B * scale)
    pr = OracleProblem(sub)
    lam = np.zeros(inst.K) if lam0 is None else np.array(lam0, np.float64)
    it = 0
    while it < max_iter:
        new = scd_sweep(pr, lam)
        it += 1
        if np.array_equal(new, lam):
            break
        lam = new
    return lam, it


def categorical_copies(tree):
    """Categorical variables (Sec. 2, x_ij non-negative integers under the
    laminar caps): the largest count of item j is the smallest cap on the
    sets containing it.  Returns those counts (an item in no set has none:
    ValueError)."""
    M = len(tree.leaf_of_item)
    sets = tree.sets()
    u = []
    for j in range(M):
        caps = [int(tree.cap[l]) for l in range(tree.L) if j in sets[l]]
        if not caps:
            raise ValueError("item %d is in no set" % j)
        u.append(min(caps))
    return np.array(u, np.int64)


def categorical_binary(inst):
    """The binary instance equivalent to a categorical one: item j becomes
    u_j identical items (its profit and costs) inside item j's innermost set,
    so the caps count copies, ordered by item.  Returns (instance,
    item_of_copy)."""
    import dataclasses
    from kpgen import Tree
    u = categorical_copies(inst.tree)
    item_of_copy = np.repeat(np.arange(inst.M), u)
    Mc = len(item_of_copy)
    N, M, K = inst.N, inst.M, inst.K
    p = inst.p.reshape(N, M)[:, item_of_copy].reshape(-1).copy()
    tree = Tree(inst.tree.parent.copy(), inst.tree.cap.copy(),
                np.asarray(inst.tree.leaf_of_item)[item_of_copy].astype(np.int32))
    bd = inst.b_dense().reshape(N, M, K)[:, item_of_copy, :]
    out = dataclasses.replace(inst, M=Mc, p=p, b=bd.reshape(-1).copy(), rowptr=None, col=None,
                              val=None, tree=tree)
    if inst.b is None:
        out = out.to_csr()
    return out, item_of_copy


def categorical_counts(x_bin, N, item_of_copy, M):
    """x_ij = the number of item j's selected copies."""
    x = np.asarray(x_bin).reshape(N, len(item_of_copy)).astype(np.int64)
    out = np.zeros((N, M), np.int64)
    for c, j in enumerate(item_of_copy):
        out[:, j] += x[:, c]
    return out


def solve(inst, method="scd", lam0=None, tol=1e-3, max_iter=100, alpha=1e-3, fix_every=1,
          block=1):
    """Reference driver: coordinate descent (Alg.4 loop) or DD (Alg.2 loop)
    until the relative duality gap g(lambda) - P(fixed-up x) falls below tol,
    lambda stops changing, or max_iter is reached.

    method: "scd" synchronous CD (every coordinate from the same lambda^t),
    "cyclic" (one coordinate per iteration), "block" (`block` consecutive
    coordinates per iteration) -- the CD variants of Sec. 4.3.2 --, "interp"
    (synchronous CD with Sec. 5.2's interpolated reduce) or "dd".
    Tracks the best dual and best feasible primal seen.  Returns the trajectory."""
    pr = OracleProblem(inst)
    K = inst.K
    lam = np.zeros(K) if lam0 is None else np.array(lam0, np.float64)
    best_g, best_P = np.inf, -np.inf
    hist = []
    for t in range(max_iter):
        ev = eval_dual(pr, lam, want_x=False)
        best_g = min(best_g, ev["g"])
        if t % fix_every == 0:
            fx = fixup(pr, lam, want_x=False)
            best_P = max(best_P, fx["P"])
        gap_rel = (best_g - best_P) / abs(best_P) if best_P > 0 else np.inf
        viol = float(np.max(np.maximum(ev["R"] - inst.B, 0) / inst.B))
        hist.append(dict(t=t, lam=lam.copy(), g=ev["g"], P=ev["P"], best_g=best_g, best_P=best_P,
                         gap_rel=gap_rel, max_viol=viol))
        if gap_rel <= tol:
            break
        if method == "dd":
            new = dd_update(lam, alpha, ev["R"], inst.B)
        elif method == "interp":
            new = scd_sweep_interp(pr, lam)
        else:
            if method == "scd":
                new = scd_sweep(pr, lam)
            else:
                w = 1 if method == "cyclic" else block
                new = scd_sweep(pr, lam, ks=[(t * w + q) % K for q in range(w)])
        if method in ("scd", "dd", "interp") and np.array_equal(new, lam):
            break
        lam = new
    return hist
