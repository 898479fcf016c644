"""Brute-force and exact-arithmetic tools that pin the C oracle (TEST
INFRASTRUCTURE ONLY).

Nothing here shares code with kp_oracle.c: these are independent
restatements -- enumeration over all subsets, a matroid greedy written as
"accept if still independent", exact rational arithmetic with fractions.Fraction,
and scipy's HiGHS LP / MILP solvers -- used as the things the oracle is checked
against.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np


def sets_of(tree) -> List[List[int]]:
    return tree.sets()


def feasible(xbits: Sequence[int], sets, caps) -> bool:
    """Local constraints (Eq.3): every set holds at most its cap."""
    return all(sum(xbits[j] for j in S) <= c for S, c in zip(sets, caps))


def brute_user(z: Sequence, sets, caps) -> Tuple[object, List[Tuple[int, ...]]]:
    """Maximum of sum_j z_j x_j over all binary x satisfying the local caps,
    and every maximiser (enumeration of all 2^M vectors)."""
    M = len(z)
    best, arg = None, []
    for bits in itertools.product((0, 1), repeat=M):
        if not feasible(bits, sets, caps):
            continue
        v = sum(z[j] for j in range(M) if bits[j])
        if best is None or v > best:
            best, arg = v, [bits]
        elif v == best:
            arg.append(bits)
    return best, arg


def matroid_greedy(z: Sequence, sets, caps) -> np.ndarray:
    """Greedy for the laminar matroid written independently of Alg.1: visit
    the items by (value descending, index ascending) and accept an item if its
    value is positive and adding it keeps every set within its cap."""
    M = len(z)
    order = sorted(range(M), key=lambda j: (-z[j], j))
    x = [0] * M
    for j in order:
        if not z[j] > 0:
            continue
        x[j] = 1
        if not feasible(x, sets, caps):
            x[j] = 0
    return np.array(x, np.uint8)


def exact_score(p: float, bs: Sequence[float], lam: Sequence[float]) -> Fraction:
    """p - sum_k lambda_k b_k in exact rational arithmetic."""
    acc = Fraction(float(p))
    for l, b in zip(lam, bs):
        acc -= Fraction(float(l)) * Fraction(float(b))
    return acc


def exact_steps(c: Sequence[float], b: Sequence[float], sets, caps):
    """Exact consumption step function of one (user, k): lines
    z_j(t) = c_j - t b_j with c_j, b_j taken as exact rationals.  Returns the
    list of (breakpoint, jump) with jump = C(t-) - C(t+) > 0 over t > 0,
    evaluated with the matroid greedy at exact midpoints (Fractions)."""
    M = len(c)
    C = [Fraction(float(v)) for v in c]
    Bq = [Fraction(float(v)) for v in b]
    cand = set()
    for j in range(M):
        if Bq[j] > 0:
            cand.add(C[j] / Bq[j])
        for jj in range(j + 1, M):
            if Bq[j] != Bq[jj]:
                cand.add((C[j] - C[jj]) / (Bq[j] - Bq[jj]))
    cand = sorted((u for u in cand if u > 0), reverse=True)

    def cons(t):
        z = [C[j] - t * Bq[j] for j in range(M)]
        x = matroid_greedy(z, sets, caps)
        return sum((Bq[j] for j in range(M) if x[j]), Fraction(0))

    out = []
    prev = Fraction(0)  # consumption above every breakpoint is 0 (b >= 0)
    for r, u in enumerate(cand):
        t = (u + cand[r + 1]) / 2 if r + 1 < len(cand) else u / 2
        cur = cons(t)
        if cur != prev:
            out.append((u, cur - prev))
        prev = cur
    return out


def lp_relaxation(inst) -> float:
    """Optimum of the LP relaxation of Eq.1-4 (0 <= x <= 1) with HiGHS."""
    import scipy.optimize
    import scipy.sparse as sp
    N, M, K = inst.N, inst.M, inst.K
    n = N * M
    bd = inst.b_dense().reshape(n, K)
    rows = [sp.csr_matrix(bd.T.astype(np.float64))]
    rhs = [inst.B.astype(np.float64)]
    sets = inst.tree.sets()
    for S, cap in zip(sets, inst.tree.cap):
        if len(S) <= cap:
            continue  # never binds for binary/fractional x in [0,1]
        r = np.repeat(np.arange(N), len(S))
        cidx = (np.arange(N)[:, None] * M + np.array(S)[None, :]).reshape(-1)
        rows.append(sp.csr_matrix((np.ones(len(r)), (r, cidx)), shape=(N, n)))
        rhs.append(np.full(N, float(cap)))
    A = sp.vstack(rows).tocsr()
    res = scipy.optimize.linprog(-inst.p.astype(np.float64), A_ub=A, b_ub=np.concatenate(rhs),
                                 bounds=(0, 1), method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return -res.fun


def ip_optimum(inst) -> float:
    """Optimum of the integer program Eq.1-4 (scipy.optimize.milp, HiGHS)."""
    import scipy.optimize
    import scipy.sparse as sp
    N, M, K = inst.N, inst.M, inst.K
    n = N * M
    bd = inst.b_dense().reshape(n, K)
    rows = [sp.csr_matrix(bd.T.astype(np.float64))]
    ub = [inst.B.astype(np.float64)]
    for S, cap in zip(inst.tree.sets(), inst.tree.cap):
        if len(S) <= cap:
            continue
        r = np.repeat(np.arange(N), len(S))
        cidx = (np.arange(N)[:, None] * M + np.array(S)[None, :]).reshape(-1)
        rows.append(sp.csr_matrix((np.ones(len(r)), (r, cidx)), shape=(N, n)))
        ub.append(np.full(N, float(cap)))
    A = sp.vstack(rows).tocsr()
    cons = scipy.optimize.LinearConstraint(A, -np.inf, np.concatenate(ub))
    res = scipy.optimize.milp(-inst.p.astype(np.float64), constraints=[cons],
                              integrality=np.ones(n), bounds=scipy.optimize.Bounds(0, 1),
                              options=dict(mip_rel_gap=0))
    if res.status != 0:
        raise RuntimeError(res.message)
    return -res.fun


def brute_global(inst) -> float:
    """Optimum of Eq.1-4 by enumerating every user's feasible subsets jointly
    (tiny instances only)."""
    N, M, K = inst.N, inst.M, inst.K
    sets, caps = inst.tree.sets(), list(inst.tree.cap)
    bd = inst.b_dense().astype(np.float64)
    p = inst.p.reshape(N, M).astype(np.float64)
    per_user = []
    for i in range(N):
        opts = []
        for bits in itertools.product((0, 1), repeat=M):
            if feasible(bits, sets, caps):
                xb = np.array(bits, np.float64)
                opts.append((float(p[i] @ xb), bd[i].T @ xb))
        per_user.append(opts)
    best = -np.inf
    for combo in itertools.product(*per_user):
        use = sum(c[1] for c in combo)
        if np.all(use <= inst.B):
            best = max(best, sum(c[0] for c in combo))
    return best


def brute_user_integer(z: Sequence, sets, caps) -> Tuple[object, List[Tuple[int, ...]]]:
    """The integer local IP by enumeration (categorical variables, Sec. 2):
    max sum_j z_j x_j over non-negative integer x with sum_{j in S_l} x_j <=
    C_l.  Every item must lie in some set.  Returns (optimum, maximisers)."""
    import itertools
    M = len(z)
    ub = [min(int(c) for s, c in zip(sets, caps) if j in s) for j in range(M)]
    best, arg = None, []
    for x in itertools.product(*[range(u + 1) for u in ub]):
        if any(sum(x[j] for j in s) > c for s, c in zip(sets, caps)):
            continue
        v = sum(Fraction(z[j]) * x[j] for j in range(M))
        if best is None or v > best:
            best, arg = v, [x]
        elif v == best:
            arg.append(x)
    return best, arg
