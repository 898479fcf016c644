"""Dual function as a torch.autograd.Function, and the iteration loop that
drives the sweep (Alg.2 / Alg.4 master loop, Sec. 4.3, with the
post-processing of Sec. 5.4).  Every step calls the C ABI; this file only
sequences the calls and does the O(K) bookkeeping of the gap check."""
from __future__ import annotations

import time
from typing import Optional

import numpy as np


class DualFn:
    """g = DualFn.apply(lam, prob): the Lagrangian dual
    g(lambda) = sum_i max_x (p_i - lambda b_i) x + lambda . B  (Eq.5).
    backward: dg/dlambda = B - R(lambda), computed by the backward kernel from
    the consumption R saved by the forward pass (no second pass over b)."""

    _fn = None

    @staticmethod
    def apply(lam, prob):
        if DualFn._fn is None:
            import torch
            from . import kp_eval_dual, kp_dual_backward

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, lam_, prob_):
                    out = kp_eval_dual(prob_, lam_.detach().contiguous())
                    ctx.prob = prob_
                    ctx.save_for_backward(out["R"])
                    return out["g"].reshape(())

                @staticmethod
                def backward(ctx, grad_out):
                    (R,) = ctx.saved_tensors
                    go = grad_out.reshape(1).to(torch.float64).contiguous()
                    return kp_dual_backward(ctx.prob, R, go), None

            DualFn._fn = _F
        return DualFn._fn.apply(lam, prob)


def solve(prob, method: str = "scd", lam0=None, tol: float = 1e-3, max_iter: int = 100,
          alpha: float = 1e-3, block: int = 1, log=None, presolve_users=None, presolve_iter: int = 30,
          ctx=None):
    """Iterate until the relative duality gap (best dual - best feasible
    primal) / |best feasible primal| <= tol, lambda stops changing, or
    max_iter.  method: "scd" | "cyclic" | "block" | "interp" (synchronous CD
    with Sec. 5.2's interpolated reduce, on a context of its own unless ctx
    is given) | "dd".  The feasible primal
    of an iterate is P(x) when x already meets every budget, else the
    post-processed value.  presolve_users: sampled users whose pre-solve
    (Sec. 5.3) replaces lam0 as the starting point.  Returns (lambda, history)."""
    import torch
    from . import Context, kp_scd_sweep, kp_dd_step, kp_primal_fixup, kp_presolve
    K = prob.K
    sweep_ctx = ctx
    if method == "interp" and sweep_ctx is None:
        sweep_ctx = Context()
        sweep_ctx.set_reduce("interp")
    B = prob.B
    lam = torch.zeros(K, dtype=torch.float64, device="cuda") if lam0 is None else \
        torch.as_tensor(np.asarray(lam0, np.float64)).to("cuda").clone()
    if presolve_users is not None:
        kp_presolve(prob, presolve_users, lam, max_iter=presolve_iter)
    best_g, best_P = np.inf, -np.inf
    hist = []
    t0 = time.perf_counter()
    for t in range(max_iter):
        if method == "dd":
            old = lam.clone()
            st = kp_dd_step(prob, alpha, lam)
            new = lam
            lam_t = old
        else:
            kmask = None
            if method in ("cyclic", "block"):
                w = 1 if method == "cyclic" else block
                kmask = np.zeros(K, np.uint8)
                kmask[[(t * w + q) % K for q in range(w)]] = 1
            st = kp_scd_sweep(prob, lam, kmask=kmask, ctx=sweep_ctx)
            new = st["lam"]
            lam_t = lam
        R = st["R"].cpu().numpy()
        g = float(st["g"].item())
        P = float(st["P"].item())
        best_g = min(best_g, g)
        if np.all(R <= B):
            best_P = max(best_P, P)
        elif P > 0 and (g - P) <= 10 * tol * abs(P):
            fx = kp_primal_fixup(prob, lam_t)
            best_P = max(best_P, float(fx["P"].item()))
        gap = (best_g - best_P) / abs(best_P) if best_P > 0 else np.inf
        viol = float(np.max(np.maximum(R - B, 0) / B))
        rec = dict(t=t, g=g, P=P, best_g=best_g, best_P=best_P, gap_rel=gap, max_viol=viol,
                   wall=time.perf_counter() - t0, lam=lam_t.cpu().numpy())
        hist.append(rec)
        if log:
            log(rec)
        if gap <= tol:
            return lam_t, hist
        if method in ("scd", "dd", "interp") and torch.equal(new, lam_t):
            return lam_t, hist
        lam = new.clone() if method != "dd" else new
    return lam, hist
