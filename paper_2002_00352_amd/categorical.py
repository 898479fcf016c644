"""Categorical (non-negative integer) decision variables (Sec. 2): x_ij in
{0, 1, 2, ...} under the same laminar caps sum_{j in S_l} x_ij <= C_l.

Item j can take at most u_j copies, the smallest cap on its chain of sets.
It is represented by u_j binary copies that carry item j's profit and costs
and hang from item j's innermost set, so every cap counts copies.  Copies of
one item have identical lines; ties go to the lower index, so the laminar
greedy (Alg.1) takes them in order and its selection is the integer greedy
solution (the laminar caps on integer vectors form an integer polymatroid,
for which the greedy is optimal, as for the binary case of Sec. 4.2).  Every
sweep (evaluation, DD, SCD, fix-up) then runs unchanged on the copies, and
x_ij is the number of item j's copies selected.

Only the data layout happens here (an index gather of p and b per user, and
the count of selected copies afterwards); the sweep runs in the library."""
from __future__ import annotations

import dataclasses

import numpy as np


def copy_counts(parent, cap, leaf_of_item) -> np.ndarray:
    """u_j = the smallest cap over item j's chain of sets.  Raises ValueError
    for an item in no set (its count would be unbounded)."""
    parent = np.asarray(parent, np.int64)
    cap = np.asarray(cap, np.int64)
    u = np.zeros(len(leaf_of_item), np.int64)
    for j, l in enumerate(np.asarray(leaf_of_item, np.int64)):
        if l < 0:
            raise ValueError(f"item {j} is in no set: its count is unbounded")
        best = None
        while l >= 0:
            best = int(cap[l]) if best is None else min(best, int(cap[l]))
            l = int(parent[l])
        u[j] = best
    return u


@dataclasses.dataclass
class CategoricalProblem:
    binary: object            # Problem over the copies
    item_of_copy: np.ndarray  # [M'] item of every copy (ascending)
    u: np.ndarray             # [M] copies per item
    M: int                    # items of the categorical instance

    def counts(self, x_copies):
        """x_ij (int32 [N, M]) from the selection of the copies (uint8 [N*M'])."""
        import torch
        N = self.binary.N
        xc = x_copies.view(N, -1).to(torch.int32)
        out = torch.zeros(N, self.M, dtype=torch.int32, device=xc.device)
        idx = torch.as_tensor(self.item_of_copy, device=xc.device)
        out.index_add_(1, idx, xc)
        return out


def expand(prob) -> CategoricalProblem:
    """The binary instance of copies of a categorical Problem (p [N*M], dense
    b [N*M*K] or per-item CSR, the laminar forest), on the same device."""
    import torch
    from . import Problem
    N, M, K = prob.N, prob.M, prob.K
    u = copy_counts(prob.parent, prob.cap, prob.leaf)
    item_of_copy = np.repeat(np.arange(M, dtype=np.int64), u)
    Mc = int(len(item_of_copy))
    if Mc > 64:
        raise ValueError(f"{Mc} copies per user exceed the 64 items a user may have")
    dev = prob.p.device
    ic = torch.as_tensor(item_of_copy, device=dev)
    p = prob.p.view(N, M).index_select(1, ic).contiguous().view(-1)
    leaf = np.asarray(prob.leaf, np.int32)[item_of_copy]
    kw = {}
    if prob.b is not None:
        kw["b"] = prob.b.view(N, M, K).index_select(1, ic).contiguous().view(-1)
    else:
        rp = prob.rowptr
        ln = (rp[1:] - rp[:-1]).view(N, M).index_select(1, ic).reshape(-1)
        rowptr = torch.zeros(N * Mc + 1, dtype=torch.int64, device=dev)
        rowptr[1:] = torch.cumsum(ln, 0)
        src = rp[:-1].view(N, M).index_select(1, ic).reshape(-1)      # first entry of every source row
        nnz = int(rowptr[-1].item())
        row = torch.repeat_interleave(torch.arange(N * Mc, device=dev), ln)
        ent = src[row] + (torch.arange(nnz, device=dev) - rowptr[:-1][row])
        kw.update(rowptr=rowptr, col=prob.col[ent].contiguous(), val=prob.val[ent].contiguous())
    binary = Problem(p, prob.B, prob.parent, prob.cap, leaf, N=N, M=Mc, K=K, **kw)
    return CategoricalProblem(binary=binary, item_of_copy=item_of_copy, u=u, M=M)
