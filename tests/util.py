"""Small instance builders shared by the tests (inputs only, no solver math)."""
import numpy as np

import kpgen


def random_laminar(M, rng, max_nodes=None):
    """A random laminar family over M items as a forest (parent, cap, leaf)."""
    perm = rng.permutation(M)
    nodes = []  # (lo, hi, parent) over positions of perm

    def split(lo, hi, parent, depth):
        if hi - lo <= 0 or depth > 3:
            return
        if rng.random() < 0.85 or parent < 0:
            nid = len(nodes)
            nodes.append([lo, hi, parent])
            par = nid
        else:
            par = parent
        if hi - lo >= 2:
            cuts = sorted(rng.choice(np.arange(lo + 1, hi), size=min(rng.integers(1, 3), hi - lo - 1),
                                     replace=False).tolist())
            bounds = [lo] + cuts + [hi]
            for a, b in zip(bounds[:-1], bounds[1:]):
                if rng.random() < 0.7:
                    split(a, b, par, depth + 1)

    split(0, M, -1, 0)
    if rng.random() < 0.3 and M >= 3:  # a second root over a few items
        pass
    L = len(nodes)
    parent = np.array([n[2] for n in nodes], np.int32)
    size = np.array([n[1] - n[0] for n in nodes])
    cap = np.array([int(rng.integers(1, max(2, s))) for s in size], np.int32)
    leaf = np.full(M, -1, np.int32)
    for pos in range(M):
        best, bs = -1, M + 1
        for l, (lo, hi, _) in enumerate(nodes):
            if lo <= pos < hi and hi - lo < bs:
                best, bs = l, hi - lo
        leaf[perm[pos]] = best
    return kpgen.Tree(parent, cap, leaf)


def make(p, b, B, tree, name="hand"):
    """Instance from explicit arrays: p [N,M], b [N,M,K]."""
    p = np.asarray(p, np.float32)
    b = np.asarray(b, np.float32)
    N, M = p.shape
    K = b.shape[2]
    return kpgen.Instance(N=N, M=M, K=K, p=p.reshape(-1).copy(), b=b.reshape(-1).copy(),
                          B=np.asarray(B, np.float64), tree=tree, name=name)


def random_instance(rng, N, M, K, tree=None, Q=2, grid=24, frac=0.3, zero_frac=0.0):
    """Uniform values on a 2^-grid grid, optional exact zeros in b."""
    p = rng.integers(0, 1 << grid, size=(N, M)) / float(1 << grid)
    b = rng.integers(0, 1 << grid, size=(N, M, K)) / float(1 << grid)
    if zero_frac:
        b[rng.random(b.shape) < zero_frac] = 0.0
    tree = tree if tree is not None else kpgen.tree_topq(M, Q)
    D = b.sum(axis=(0, 1))
    B = np.maximum(frac * D, 1e-3)
    return make(p, b, B, tree)
