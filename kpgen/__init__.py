"""Seeded synthetic knapsack instances (host side).

This module generates the inputs both the CPU oracle and the GPU path consume.
It holds none of the solver's arithmetic: only a counter-based random number
generator, the value distributions, the instance shapes and the budgets.

Generator definition (published SplitMix64 finaliser, Steele/Lea/Flood 2014,
used in counter mode):

    draw(seed, stream, idx) = mix64((seed XOR stream<<56) + (idx+1)*GAMMA)   mod 2^64
    u24 = draw >> 40                                   (24 uniform bits)

Value distributions, all fp32:
  * uniform  U(0,1):  u24 * 2^-24   (a 2^-24 grid that includes 0; sums of these
    values are exact in FP64 while below 2^29)
  * exp1     Exp(1):  table[u24], table[v] = fp32(-log(1 - (v+0.5)/2^24))
  * lognormal LN(0,1): table[v] = fp32(exp(Phi^-1((v+0.5)/2^24)))
The two inverse-CDF tables (2^24 entries each) are built once on the host and
shipped to the device generator, so both sides read identical bytes.

Layouts match the library boundary: p[N*M] (item fastest), dense b[N*M*K]
(k fastest), per-item CSR (rowptr int64[N*M+1], col int32, val fp32) with the
columns of each item strictly ascending.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream ids (8 bits each)
S_P, S_B, S_COL, S_VAL, S_LAMBDA, S_SEED, S_SHAPE, S_SAMPLE = 1, 2, 3, 4, 5, 6, 7, 8

DIST_UNIFORM, DIST_EXP1, DIST_LOGNORMAL = 0, 1, 2
_DIST_NAMES = {"uniform": DIST_UNIFORM, "exp1": DIST_EXP1, "lognormal": DIST_LOGNORMAL}


def mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z ^ (z >> np.uint64(30))
        z = z * _M1
        z = z ^ (z >> np.uint64(27))
        z = z * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def draw(seed: int, stream: int, idx) -> np.ndarray:
    """64 random bits at position idx of (seed, stream)."""
    base = np.uint64((int(seed) ^ (int(stream) << 56)) & 0xFFFFFFFFFFFFFFFF)
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = base + (idx + np.uint64(1)) * GAMMA
    return mix64(z)


def u24(seed: int, stream: int, idx) -> np.ndarray:
    return (draw(seed, stream, idx) >> np.uint64(40)).astype(np.int64)


def draw_scalar(seed: int, stream: int, idx: int) -> int:
    return int(draw(seed, stream, np.array([idx], dtype=np.uint64))[0])


_TABLES = {}


def dist_table(dist: int) -> Optional[np.ndarray]:
    """fp32[2^24] inverse-CDF table for a non-uniform distribution (None for uniform)."""
    if dist == DIST_UNIFORM:
        return None
    if dist not in _TABLES:
        q = (np.arange(1 << 24, dtype=np.float64) + 0.5) * 2.0 ** -24
        if dist == DIST_EXP1:
            t = -np.log1p(-q)
        elif dist == DIST_LOGNORMAL:
            import scipy.special
            t = np.exp(scipy.special.ndtri(q))
        else:
            raise ValueError(dist)
        _TABLES[dist] = t.astype(np.float32)
    return _TABLES[dist]


def values(u: np.ndarray, dist: int) -> np.ndarray:
    if dist == DIST_UNIFORM:
        return (u.astype(np.float64) * 2.0 ** -24).astype(np.float32)
    return dist_table(dist)[u]


# ----------------------------------------------------------------------------
# local-constraint forests
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Tree:
    """Laminar family of item sets as a forest: node l has cap[l] and parent[l]
    (-1 for a root); leaf_of_item[j] is the innermost node containing item j, or
    -1 when j is in no set. Set S_l = all items whose ancestor chain meets l."""
    parent: np.ndarray
    cap: np.ndarray
    leaf_of_item: np.ndarray

    @property
    def L(self) -> int:
        return int(len(self.parent))

    def sets(self) -> List[List[int]]:
        M = len(self.leaf_of_item)
        out: List[List[int]] = [[] for _ in range(self.L)]
        for j in range(M):
            l = int(self.leaf_of_item[j])
            while l >= 0:
                out[l].append(j)
                l = int(self.parent[l])
        return out


def tree_topq(M: int, Q: int) -> Tree:
    return Tree(np.array([-1], np.int32), np.array([Q], np.int32), np.zeros(M, np.int32))


def tree_hier_2_2_3(M: int = 10) -> Tree:
    """Root cap 3 over two halves of the items with cap 2 each, plus a cap-1
    node per item (the hierarchical 'C=[2,2,3]' local constraints)."""
    half = M // 2
    parent = [-1, 0, 0] + [1 if j < half else 2 for j in range(M)]
    cap = [3, 2, 2] + [1] * M
    leaf = [3 + j for j in range(M)]
    return Tree(np.array(parent, np.int32), np.array(cap, np.int32), np.array(leaf, np.int32))


# ----------------------------------------------------------------------------
# instances
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Instance:
    N: int
    M: int
    K: int
    p: np.ndarray                 # fp32 [N*M]
    B: np.ndarray                 # fp64 [K]
    tree: Tree
    b: Optional[np.ndarray] = None        # dense fp32 [N*M*K]
    rowptr: Optional[np.ndarray] = None   # int64 [N*M+1]
    col: Optional[np.ndarray] = None      # int32 [nnz]
    val: Optional[np.ndarray] = None      # fp32 [nnz]
    seed: int = 0
    name: str = ""

    @property
    def dense(self) -> bool:
        return self.b is not None

    def b_dense(self) -> np.ndarray:
        """Dense [N,M,K] view (materialised from CSR when needed; small N only)."""
        if self.b is not None:
            return self.b.reshape(self.N, self.M, self.K)
        out = np.zeros(self.N * self.M * self.K, np.float32)
        rows = np.repeat(np.arange(self.N * self.M, dtype=np.int64), np.diff(self.rowptr))
        out[rows * self.K + self.col] = self.val
        return out.reshape(self.N, self.M, self.K)

    def to_csr(self) -> "Instance":
        """Same instance with b stored per-item CSR (zeros dropped)."""
        bd = self.b_dense().reshape(self.N * self.M, self.K)
        nz = bd != 0
        rowptr = np.zeros(self.N * self.M + 1, np.int64)
        rowptr[1:] = np.cumsum(nz.sum(axis=1))
        r, c = np.nonzero(nz)
        return dataclasses.replace(self, b=None, rowptr=rowptr, col=c.astype(np.int32),
                                   val=bd[r, c].astype(np.float32))

    def subset(self, users: Sequence[int], B: Optional[np.ndarray] = None) -> "Instance":
        """The instance restricted to the given users (budgets kept unless given)."""
        users = np.asarray(users, np.int64)
        M, K = self.M, self.K
        p = self.p.reshape(self.N, M)[users].reshape(-1).copy()
        BB = self.B.copy() if B is None else np.asarray(B, np.float64)
        if self.b is not None:
            b = self.b.reshape(self.N, M * K)[users].reshape(-1).copy()
            return dataclasses.replace(self, N=len(users), p=p, b=b, B=BB)
        rows = (users[:, None] * M + np.arange(M)[None, :]).reshape(-1)
        cnt = self.rowptr[rows + 1] - self.rowptr[rows]
        rowptr = np.zeros(len(rows) + 1, np.int64)
        rowptr[1:] = np.cumsum(cnt)
        idx = np.concatenate([np.arange(self.rowptr[r], self.rowptr[r + 1]) for r in rows]) \
            if len(rows) else np.zeros(0, np.int64)
        return dataclasses.replace(self, N=len(users), p=p, rowptr=rowptr,
                                   col=self.col[idx].copy(), val=self.val[idx].copy(), B=BB)


def gen_p(seed: int, N: int, M: int, dist: int, first_user: int = 0) -> np.ndarray:
    idx = np.arange(first_user * M, (first_user + N) * M, dtype=np.uint64)
    return values(u24(seed, S_P, idx), dist)


def gen_b_dense(seed: int, N: int, M: int, K: int, first_user: int = 0) -> np.ndarray:
    idx = np.arange(first_user * M * K, (first_user + N) * M * K, dtype=np.uint64)
    return values(u24(seed, S_B, idx), DIST_UNIFORM)


def gen_csr_cols(seed: int, rows: np.ndarray, K: int, d: int) -> np.ndarray:
    """d distinct columns per item row, ascending: int32 [len(rows), d]."""
    rows = np.asarray(rows, np.uint64)
    n = len(rows)
    chosen = np.zeros((n, 0), np.int64)
    for t in range(d):
        u = u24(seed, S_COL, rows * np.uint64(d) + np.uint64(t))
        k = (u * (K - t)) >> 24
        # map the draw from the K-t remaining columns onto [0,K) skipping chosen ones
        for s in range(t):
            k = k + (k >= chosen[:, s])
        chosen = np.sort(np.concatenate([chosen, k[:, None]], axis=1), axis=1)
    return chosen.astype(np.int32)


def gen_csr(seed: int, N: int, M: int, K: int, d: int, first_user: int = 0):
    rows = np.arange(first_user * M, (first_user + N) * M, dtype=np.uint64)
    col = gen_csr_cols(seed, rows, K, d).reshape(-1)
    vidx = (rows[:, None] * np.uint64(d) + np.arange(d, dtype=np.uint64)[None, :]).reshape(-1)
    val = values(u24(seed, S_VAL, vidx), DIST_UNIFORM)
    rowptr = np.arange(N * M + 1, dtype=np.int64) * d
    return rowptr, col, val


def demand(inst: Instance) -> np.ndarray:
    """D_k = sum_i sum_j b_ijk, exact (values are on the 2^-24 grid)."""
    if inst.b is not None:
        q = np.rint(inst.b.astype(np.float64) * 2.0 ** 24).astype(np.int64).reshape(-1, inst.K)
        s = q.sum(axis=0)
    else:
        q = np.rint(inst.val.astype(np.float64) * 2.0 ** 24).astype(np.int64)
        s = np.zeros(inst.K, np.int64)
        np.add.at(s, inst.col.astype(np.int64), q)
    return s.astype(np.float64) * 2.0 ** -24


def make_instance(N: int, M: int, K: int, *, seed: int, p_dist: str = "uniform",
                  tree: Optional[Tree] = None, Q: int = 1, csr_d: int = 0,
                  budget_frac: float = 0.1, budget_per_item_mean: bool = False,
                  name: str = "") -> Instance:
    """Generate a whole instance on the host.

    budget: B_k = budget_frac * D_k (or budget_frac * D_k / M when
    budget_per_item_mean, i.e. a fraction of sum_i mean_j b_ijk)."""
    dist = _DIST_NAMES[p_dist]
    tree = tree if tree is not None else tree_topq(M, Q)
    p = gen_p(seed, N, M, dist)
    inst = Instance(N=N, M=M, K=K, p=p, B=np.zeros(K), tree=tree, seed=seed, name=name)
    if csr_d:
        inst.rowptr, inst.col, inst.val = gen_csr(seed, N, M, K, csr_d)
    else:
        inst.b = gen_b_dense(seed, N, M, K)
    inst.B = budgets(demand(inst), budget_frac, M if budget_per_item_mean else 1)
    return inst


def budgets(D: np.ndarray, frac: float, div: int) -> np.ndarray:
    B = np.array([(frac * float(d)) / div for d in D], np.float64)
    # a knapsack nobody consumes still needs a strictly positive budget
    return np.where(B > 0, B, 1.0)


# ----------------------------------------------------------------------------
# the five workloads (seed = 1000*config + run)
# ----------------------------------------------------------------------------

CONFIGS = {
    1: dict(N=10_000, M=10, K=2, Q=1, p_dist="uniform", csr_d=0, budget_frac=0.2,
            budget_per_item_mean=True, name="c1 plain SCD+DD N=1e4 M=10 K=2 Q=1"),
    2: dict(N=10_000_000, M=10, K=10, Q=3, p_dist="lognormal", csr_d=0, budget_frac=0.1,
            budget_per_item_mean=True, name="c2 plain SCD N=1e7 M=10 K=10 Q=3 dense"),
    3: dict(N=100_000_000, M=10, K=20, Q=0, p_dist="exp1", csr_d=2, budget_frac=0.05,
            budget_per_item_mean=False, hier=True,
            name="c3 hierarchical N=1e8 M=10 K=20 CSR(2/item) caps 3>(2,2)>1"),
    4: dict(N=10_000_000, M=20, K=50, Q=5, p_dist="uniform", csr_d=0, budget_frac=0.1,
            budget_per_item_mean=True, name="c4 autograd dual N=1e7 M=20 K=50 Q=5 dense"),
}


def config_instance(c: int, run: int = 0, N: Optional[int] = None) -> Instance:
    """Host-generated instance of workload c (optionally with fewer users N;
    budgets are then computed from the generated users)."""
    cfg = dict(CONFIGS[c])
    name = cfg.pop("name")
    hier = cfg.pop("hier", False)
    if N is not None:
        cfg["N"] = N
    Q = cfg.pop("Q")
    tree = tree_hier_2_2_3(cfg["M"]) if hier else None
    return make_instance(seed=1000 * c + run, tree=tree, Q=max(Q, 1), name=name, **cfg)


def batched_shapes(seed: int, n: int = 256):
    """Ragged shapes of the batched workload: N log-uniform in [1e3,1e6),
    M uniform in {4..32}, K uniform in {1..16}, Q uniform in {1..4}."""
    out = []
    for s in range(n):
        u = u24(seed, S_SHAPE, np.arange(4 * s, 4 * s + 4, dtype=np.uint64))
        N = int(math.floor(10.0 ** (3.0 + 3.0 * (float(u[0]) * 2.0 ** -24))))
        M = 4 + int((int(u[1]) * 29) >> 24)
        K = 1 + int((int(u[2]) * 16) >> 24)
        Q = 1 + int((int(u[3]) * 4) >> 24)
        out.append((N, M, K, Q, draw_scalar(seed, S_SEED, s)))
    return out


def batched_instances(run: int = 0, n: int = 256, max_N: Optional[int] = None) -> List[Instance]:
    seed = 1000 * 5 + run
    insts = []
    for s, (N, M, K, Q, sd) in enumerate(batched_shapes(seed, n)):
        if max_N is not None:
            N = min(N, max_N)
        insts.append(make_instance(N, M, K, seed=sd, Q=Q, budget_frac=0.1,
                                   name=f"c5 instance {s}"))
    return insts


def random_lambdas(seed: int, n: int, K: int, hi: float) -> np.ndarray:
    """n points lambda ~ U(0, hi)^K, fp64 built from 24-bit draws."""
    u = u24(seed, S_LAMBDA, np.arange(n * K, dtype=np.uint64)).astype(np.float64)
    return (u * 2.0 ** -24 * hi).reshape(n, K)


def sample_users(seed: int, N: int, n: int) -> np.ndarray:
    """n distinct users of [0, N) for pre-solving by sampling: one user drawn
    uniformly from each of n consecutive strata [floor(s N / n), floor((s+1) N / n)).
    (The draw is an input of the pre-solve, so every side uses the same sample.)"""
    if not 1 <= n <= N:
        raise ValueError("need 1 <= n <= N")
    s = np.arange(n, dtype=np.int64)
    lo = (s * N) // n
    hi = ((s + 1) * N) // n
    u = draw(seed, S_SAMPLE, s.astype(np.uint64)) >> np.uint64(11)        # 53 bits
    off = (u.astype(np.float64) * 2.0 ** -53 * (hi - lo)).astype(np.int64)
    return lo + np.minimum(off, hi - lo - 1)


def checksum(a: np.ndarray) -> str:
    """BLAKE2b-64 of the array bytes (records which inputs a result used)."""
    import hashlib
    return hashlib.blake2b(np.ascontiguousarray(a).view(np.uint8), digest_size=8).hexdigest()
