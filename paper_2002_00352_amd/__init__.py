"""MI355X (gfx950) per-user subproblem sweep of the Lagrangian-dual knapsack
solver ("Solving Billion-Scale Knapsack Problems", Zhang et al., WWW'20).

Thin Python binding of the C ABI in include/kp.h: argument marshalling only.
Every step of the sweep runs in the HIP kernels of libkp.so; PyTorch provides
device memory and the current HIP stream.  If the library is not built the
calls raise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_REPO = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libkp.so")
SOURCES = [os.path.join(_HERE, "csrc", f) for f in
           ("kp_kernels.hip", "kp_ell.hip", "kp_ell_m0.hip", "kp_ell_m1.hip", "kp_ell_m2.hip",
            "kp_ell_m3.hip", "kp_ell_m4.hip", "kp_dense.hip", "kp_batched.hip", "kp_capi.hip")]
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-result"]

KP_OK = 0
STATUS = {0: "KP_OK", -1: "KP_ERR_INVALID", -2: "KP_ERR_NOT_LAMINAR", -3: "KP_ERR_NONFINITE",
          -4: "KP_ERR_NEGATIVE", -5: "KP_ERR_UNSUPPORTED", -6: "KP_ERR_NOMEM", -7: "KP_ERR_HIP",
          -8: "KP_ERR_INTERNAL"}
KP_B_DENSE, KP_B_CSR = 0, 1
KP_ERR_INVALID, KP_ERR_UNSUPPORTED = -1, -5


def build() -> str:
    """Compile libkp.so for gfx950 with hipcc (always recompiles; the sources
    are compiled in parallel, then linked)."""
    import tempfile
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory() as td:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(td, os.path.basename(src) + ".o")
            objs.append(obj)
            procs.append(subprocess.Popen([hipcc, *flags, "-c", "-o", obj, src]))
        rcs = [p.wait() for p in procs]
        if any(rcs):
            raise subprocess.CalledProcessError(max(rcs, key=abs), hipcc)
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class KPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class kp_problem(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("M", ctypes.c_int32), ("K", ctypes.c_int32),
        ("p", ctypes.c_void_p), ("b_format", ctypes.c_int32), ("b", ctypes.c_void_p),
        ("b_rowptr", ctypes.c_void_p), ("b_col", ctypes.c_void_p), ("b_val", ctypes.c_void_p),
        ("B", ctypes.c_void_p), ("L", ctypes.c_int32), ("parent", ctypes.c_void_p),
        ("cap", ctypes.c_void_p), ("leaf_of_item", ctypes.c_void_p), ("b_row_nnz", ctypes.c_int32),
    ]


_lib = None
EXPORTS = ["kp_last_error", "kp_create", "kp_destroy", "kp_set_stream", "kp_eval_dual",
           "kp_scd_sweep", "kp_scd_sweep_masked", "kp_dd_step", "kp_dual_backward",
           "kp_primal_fixup", "kp_scd_sweep_batched", "kp_validate_inputs", "kp_tree_from_sets",
           "kp_max_items", "kp_max_knapsacks_scd", "kp_set_timing", "kp_get_timing",
           "kp_batched_create", "kp_batched_step", "kp_batched_destroy", "kp_set_tuning",
           "kp_set_kernel_choice", "kp_csr_row_nnz", "kp_set_window",
           "kp_get_window_stats", "kp_presolve", "kp_get_window_listed", "kp_get_launch_shape",
           "kp_set_batched_tuning", "kp_batched_shape", "kp_eval_dual_noalloc", "kp_get_batched_passes",
           "kp_stream_read", "kp_set_alg5", "kp_set_reduce", "kp_set_sampled_start"]


def lib():
    """Load libkp.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER(kp_problem)
        L.kp_last_error.restype = ctypes.c_char_p
        L.kp_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_size_t]
        L.kp_destroy.argtypes = [vp]
        L.kp_set_stream.argtypes = [vp, vp]
        L.kp_eval_dual.argtypes = [vp, P, vp, vp, vp, vp, vp]
        L.kp_eval_dual_noalloc.argtypes = [vp, P, vp, vp, vp, vp, vp]
        L.kp_scd_sweep.argtypes = [vp, P, vp, vp, vp, vp, vp]
        L.kp_scd_sweep_masked.argtypes = [vp, P, vp, vp, vp, vp, vp, vp]
        L.kp_dd_step.argtypes = [vp, P, d, vp, vp, vp, vp]
        L.kp_dual_backward.argtypes = [vp, P, vp, vp, vp]
        L.kp_primal_fixup.argtypes = [vp, P, vp, vp, vp, vp, vp]
        L.kp_scd_sweep_batched.argtypes = [vp, P, i32, vp, vp, vp]
        L.kp_validate_inputs.argtypes = [vp, P]
        L.kp_tree_from_sets.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.kp_batched_create.argtypes = [vp, P, i32, vp, vp, ctypes.POINTER(vp)]
        L.kp_batched_step.argtypes = [vp, i32, vp, i32]
        L.kp_batched_destroy.argtypes = [vp]
        L.kp_set_tuning.argtypes = [vp, i32, i32, i32, i32, i32]
        L.kp_set_kernel_choice.argtypes = [vp, i32]
        L.kp_csr_row_nnz.argtypes = [vp, P, ctypes.POINTER(i32)]
        L.kp_set_window.argtypes = [vp, i32]
        L.kp_set_alg5.argtypes = [vp, i32]
        L.kp_set_reduce.argtypes = [vp, i32]
        L.kp_set_sampled_start.argtypes = [vp, i64]
        L.kp_presolve.argtypes = [vp, P, vp, i64, i32, vp, ctypes.POINTER(i32)]
        L.kp_get_window_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                          ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.kp_get_window_listed.argtypes = [vp, ctypes.POINTER(i64)]
        L.kp_get_launch_shape.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.kp_set_batched_tuning.argtypes = [vp, i32, i32]
        L.kp_batched_shape.argtypes = [vp] + [ctypes.POINTER(i32)] * 4
        L.kp_get_batched_passes.argtypes = [vp, ctypes.POINTER(i64)]
        L.kp_stream_read.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.kp_set_timing.argtypes = [vp, i32]
        L.kp_get_timing.argtypes = [vp, vp, vp, vp]
        L.kp_max_items.restype = i32
        L.kp_max_knapsacks_scd.restype = i32
        for name in EXPORTS:
            if name not in ("kp_last_error", "kp_max_items", "kp_max_knapsacks_scd"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != KP_OK:
        raise KPError(status, lib().kp_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A kp context bound to the current torch HIP stream."""

    def __init__(self, max_workspace_bytes: int = 0):
        self.h = ctypes.c_void_p()
        _check(lib().kp_create(ctypes.byref(self.h), _stream_handle(), max_workspace_bytes))

    def sync_stream(self):
        _check(lib().kp_set_stream(self.h, _stream_handle()))

    def set_timing(self, on: bool):
        _check(lib().kp_set_timing(self.h, 1 if on else 0))

    def timing(self):
        """(sweep kernel ms total, launches, algorithmic bytes total)."""
        ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().kp_get_timing(self.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
        return ms.value, n.value, by.value

    def batched_passes(self) -> int:
        """Sweep passes inside the timed iterations of batched plans."""
        n = ctypes.c_int64()
        _check(lib().kp_get_batched_passes(self.h, ctypes.byref(n)))
        return n.value

    def set_tuning(self, M: int, K: int, b_format: int, users_per_tile: int, grid: int):
        _check(lib().kp_set_tuning(self.h, M, K, b_format, users_per_tile, grid))

    def launch_shape(self):
        """(kernel, users per tile, blocks) of the last sweep launch: kernel 0
        is the general kernel, 1 the uniform-row kernel, 2 the lane-per-user
        evaluation of dense costs, 3 its SCD window pass, -1 none yet."""
        k, u, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().kp_get_launch_shape(self.h, ctypes.byref(k), ctypes.byref(u), ctypes.byref(g)))
        return k.value, u.value, g.value

    def set_batched_tuning(self, lds_bytes: int, block_mult: int):
        _check(lib().kp_set_batched_tuning(self.h, int(lds_bytes), int(block_mult)))

    def set_kernel_choice(self, allow_uniform_rows: bool):
        _check(lib().kp_set_kernel_choice(self.h, 1 if allow_uniform_rows else 0))

    def set_reduce(self, mode: str):
        """"exact" (Alg.4's threshold) or "interp" (Sec. 5.2's bucket
        interpolation)."""
        _check(lib().kp_set_reduce(self.h, {"exact": 0, "interp": 1}[mode]))

    def set_sampled_start(self, min_users: int):
        """Full searches of problems with at least min_users users start from
        a sample's threshold (0: never)."""
        _check(lib().kp_set_sampled_start(self.h, int(min_users)))

    def set_alg5(self, on: bool):
        """Alg.5's map (Sec. 5.1) for the users in its setting."""
        _check(lib().kp_set_alg5(self.h, 1 if on else 0))

    def set_window(self, on: bool):
        _check(lib().kp_set_window(self.h, 1 if on else 0))

    def window_stats(self):
        """(window searches tried, threshold found above, below, breakpoints
        emitted inside windows) since creation."""
        t, a, b, e = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().kp_get_window_stats(self.h, ctypes.byref(t), ctypes.byref(a), ctypes.byref(b),
                                         ctypes.byref(e)))
        return t.value, a.value, b.value, e.value

    def window_listed(self) -> int:
        """Users listed for exact checks by the uniform-row kernel's window
        passes since creation."""
        n = ctypes.c_int64()
        _check(lib().kp_get_window_listed(self.h, ctypes.byref(n)))
        return n.value

    def close(self):
        if self.h:
            lib().kp_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: Optional[Context] = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    _default_ctx.sync_stream()
    return _default_ctx


class Problem:
    """Device-resident instance: p, b (dense or CSR) as torch tensors on the
    GPU; B and the local-constraint forest on the host.

    row_nnz (CSR only): the entries every item row holds at offsets r*D
    (1 or 2), 0 for general rows, or None to ask the library
    (kp_csr_row_nnz, one device pass over rowptr at construction).  The
    declaration lets the lean per-user kernel skip rowptr; it stays valid as
    long as the arrays this object holds are not rewritten in place."""

    def __init__(self, p, B, parent, cap, leaf_of_item, *, b=None, rowptr=None, col=None,
                 val=None, N=None, M=None, K=None, row_nnz=None):
        import torch
        self.p = p
        self.b, self.rowptr, self.col, self.val = b, rowptr, col, val
        self.B = np.ascontiguousarray(B, np.float64)
        self.parent = np.ascontiguousarray(parent, np.int32)
        self.cap = np.ascontiguousarray(cap, np.int32)
        self.leaf = np.ascontiguousarray(leaf_of_item, np.int32)
        self.N, self.M, self.K = int(N), int(M), int(K)
        for t in (p, b, rowptr, col, val):
            if t is not None and not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
                raise TypeError("p/b arrays must be contiguous GPU tensors")
        s = kp_problem()
        s.N, s.M, s.K = self.N, self.M, self.K
        s.p = _ptr(p)
        s.b_format = KP_B_DENSE if b is not None else KP_B_CSR
        s.b, s.b_rowptr, s.b_col, s.b_val = _ptr(b), _ptr(rowptr), _ptr(col), _ptr(val)
        s.B = _ptr(self.B)
        s.L = len(self.parent)
        s.parent, s.cap, s.leaf_of_item = _ptr(self.parent), _ptr(self.cap), _ptr(self.leaf)
        s.b_row_nnz = 0
        self.s = s
        if b is None and row_nnz is None:
            row_nnz = kp_csr_row_nnz(self)
        self.row_nnz = 0 if b is not None else int(row_nnz)
        s.b_row_nnz = self.row_nnz

    @property
    def ref(self):
        return ctypes.byref(self.s)

    @classmethod
    def from_host(cls, inst, device="cuda"):
        """Copy a host instance (kpgen.Instance-like) to the GPU."""
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).to(device)
        kw = {}
        if inst.b is not None:
            kw["b"] = t(inst.b, np.float32)
        else:
            kw.update(rowptr=t(inst.rowptr, np.int64), col=t(inst.col, np.int32),
                      val=t(inst.val, np.float32))
        return cls(t(inst.p, np.float32), inst.B, inst.tree.parent, inst.tree.cap,
                   inst.tree.leaf_of_item, N=inst.N, M=inst.M, K=inst.K, **kw)


# ---------------------------------------------------------------------------
# the C ABI, one Python function per entry point (tensors in, tensors out)
# ---------------------------------------------------------------------------

def _dev_f64(n):
    import torch
    return torch.empty(n, dtype=torch.float64, device="cuda")


def kp_eval_dual(prob: Problem, lam, want_x: bool = False, ctx: Optional[Context] = None):
    """g(lambda), R(lambda), P(x(lambda)) and optionally x (uint8 [N*M])."""
    import torch
    ctx = ctx or default_context()
    R, g, P = _dev_f64(prob.K), _dev_f64(1), _dev_f64(1)
    x = torch.empty(prob.N * prob.M, dtype=torch.uint8, device="cuda") if want_x else None
    _check(lib().kp_eval_dual(ctx.h, prob.ref, _ptr(lam), _ptr(R), _ptr(g), _ptr(P), _ptr(x)))
    return dict(R=R, g=g, P=P, x=x)


def kp_eval_dual_noalloc(prob: Problem, lam, R, g, P, x=None):
    """The allocation-free evaluation on the current torch stream into
    caller-provided tensors R [K], g [1], P [1] (FP64) and x (uint8 [N*M])
    or None."""
    _check(lib().kp_eval_dual_noalloc(_stream_handle(), prob.ref, _ptr(lam), _ptr(R), _ptr(g), _ptr(P),
                                      _ptr(x)))
    return dict(R=R, g=g, P=P, x=x)


def kp_scd_sweep(prob: Problem, lam_in, lam_out=None, kmask=None, ctx: Optional[Context] = None):
    """One SCD iteration: returns lambda_out and the statistics at lambda_in."""
    ctx = ctx or default_context()
    lam_out = _dev_f64(prob.K) if lam_out is None else lam_out
    R, g, P = _dev_f64(prob.K), _dev_f64(1), _dev_f64(1)
    if kmask is None:
        st = lib().kp_scd_sweep(ctx.h, prob.ref, _ptr(lam_in), _ptr(lam_out), _ptr(R), _ptr(g), _ptr(P))
    else:
        km = np.ascontiguousarray(kmask, np.uint8)
        st = lib().kp_scd_sweep_masked(ctx.h, prob.ref, _ptr(lam_in), _ptr(lam_out), _ptr(km),
                                       _ptr(R), _ptr(g), _ptr(P))
    _check(st)
    return dict(lam=lam_out, R=R, g=g, P=P)


def kp_dd_step(prob: Problem, alpha: float, lam, ctx: Optional[Context] = None):
    """One DD step in place on lam; returns the statistics at the old lambda."""
    ctx = ctx or default_context()
    R, g, P = _dev_f64(prob.K), _dev_f64(1), _dev_f64(1)
    _check(lib().kp_dd_step(ctx.h, prob.ref, float(alpha), _ptr(lam), _ptr(R), _ptr(g), _ptr(P)))
    return dict(lam=lam, R=R, g=g, P=P)


def kp_dual_backward(prob: Problem, R, grad_out, ctx: Optional[Context] = None):
    ctx = ctx or default_context()
    gl = _dev_f64(prob.K)
    _check(lib().kp_dual_backward(ctx.h, prob.ref, _ptr(R), _ptr(grad_out), _ptr(gl)))
    return gl


def kp_primal_fixup(prob: Problem, lam, want_x: bool = False, ctx: Optional[Context] = None):
    import torch
    ctx = ctx or default_context()
    x = torch.empty(prob.N * prob.M, dtype=torch.uint8, device="cuda") if want_x else None
    P, R = _dev_f64(1), _dev_f64(prob.K)
    nres = torch.zeros(1, dtype=torch.int64, device="cuda")
    _check(lib().kp_primal_fixup(ctx.h, prob.ref, _ptr(lam), _ptr(x), _ptr(P), _ptr(R), _ptr(nres)))
    return dict(x=x, P=P, R=R, n_reset=nres)


def kp_scd_sweep_batched(probs: Sequence[Problem], lams_in, lams_out=None,
                         ctx: Optional[Context] = None):
    """One SCD iteration for every instance in one persistent launch per
    pass.  Returns (lams_out, stats) with stats the per-instance [R, g, P] at
    lams_in, concatenated."""
    import torch
    ctx = ctx or default_context()
    n = len(probs)
    arr = (kp_problem * n)(*[pr.s for pr in probs])
    lams_out = [_dev_f64(pr.K) for pr in probs] if lams_out is None else lams_out
    pin = (ctypes.c_void_p * n)(*[t.data_ptr() for t in lams_in])
    pout = (ctypes.c_void_p * n)(*[t.data_ptr() for t in lams_out])
    stats = _dev_f64(sum(pr.K + 2 for pr in probs))
    _check(lib().kp_scd_sweep_batched(ctx.h, arr, n, pin, pout, _ptr(stats)))
    return lams_out, stats


class BatchedSCD:
    """Repeated SCD iterations over a batch of instances: device tables built
    once, each iteration (its first pass and up to five later passes, split
    among the open instances on the device) replayed from a captured HIP
    graph; a search still open after them continues from the host."""

    def __init__(self, probs: Sequence[Problem], lam0=None, use_graph: bool = True,
                 ctx: Optional[Context] = None):
        import torch
        # graph capture needs a stream other than the legacy default stream
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.ctx = ctx or Context()
            self.ctx.sync_stream()   # a given context is rebound to the plan's stream
        self.probs = list(probs)
        n = len(self.probs)
        self.a = [torch.zeros(pr.K, dtype=torch.float64, device="cuda") if lam0 is None
                  else torch.as_tensor(np.asarray(lam0[s], np.float64)).to("cuda").clone()
                  for s, pr in enumerate(self.probs)]
        self.b = [torch.zeros(pr.K, dtype=torch.float64, device="cuda") for pr in self.probs]
        self.use_graph = use_graph
        self.dir = 0
        torch.cuda.synchronize()   # buffers made on other streams are ready
        arr = (kp_problem * n)(*[pr.s for pr in self.probs])
        pa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.a])
        pb = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.b])
        self.h = ctypes.c_void_p()
        _check(lib().kp_batched_create(self.ctx.h, arr, n, pa, pb, ctypes.byref(self.h)))
        self.stats = _dev_f64(sum(pr.K + 2 for pr in self.probs))

    def shape(self):
        """(blocks, LDS bytes per block, min and max users per tile) of the
        plan's first pass."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().kp_batched_shape(self.h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    @property
    def lam(self):
        """Current multipliers (the buffer the last step wrote)."""
        return self.a if self.dir == 0 else self.b

    def step(self):
        """One iteration; returns (new lambdas, stats at the old lambdas)."""
        _check(lib().kp_batched_step(self.h, self.dir, _ptr(self.stats), 1 if self.use_graph else 0))
        self.dir ^= 1
        return self.lam, self.stats

    def close(self):
        if self.h:
            lib().kp_batched_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kp_presolve(prob: Problem, users, lam, max_iter: int = 30, ctx: Optional[Context] = None):
    """Pre-solving by sampling (Sec. 5.3): SCD on the sampled users with the
    budgets scaled by n/N, from lam (a K-vector of FP64 on the device, updated
    in place).  users: distinct user indices (host integers).  Returns
    (lam, sweeps)."""
    ctx = ctx or default_context()
    u = np.ascontiguousarray(np.asarray(users, dtype=np.int64))
    it = ctypes.c_int32()
    _check(lib().kp_presolve(ctx.h, prob.ref, u.ctypes.data, len(u), int(max_iter),
                             _ptr(lam), ctypes.byref(it)))
    return lam, it.value


def kp_csr_row_nnz(prob: Problem, ctx: Optional[Context] = None) -> int:
    """D when every item row of the CSR costs holds D in {1, 2} entries at
    r*D, else 0 (one device pass over rowptr)."""
    ctx = ctx or default_context()
    D = ctypes.c_int32()
    _check(lib().kp_csr_row_nnz(ctx.h, prob.ref, ctypes.byref(D)))
    return D.value


def kp_stream_read(t, out=None):
    """Read tensor t once on the current stream (the streaming read probe;
    bytes past the last whole 16-byte word are not read); returns its
    checksum as a device tensor: with (x, y, z, w) the XOR of its 16-byte
    words as four 32-bit words, ((x ^ z) << 32) | (y ^ w)."""
    import torch
    out = torch.zeros(1, dtype=torch.int64, device="cuda") if out is None else out
    nbytes = t.numel() * t.element_size()
    _check(lib().kp_stream_read(_stream_handle(), t.data_ptr(), nbytes - nbytes % 16, out.data_ptr()))
    return out


def kp_validate_inputs(prob: Problem, ctx: Optional[Context] = None):
    ctx = ctx or default_context()
    _check(lib().kp_validate_inputs(ctx.h, prob.ref))


def kp_tree_from_sets(M: int, sets: Sequence[Sequence[int]], caps: Sequence[int]):
    """Explicit local sets -> (parent, cap, leaf_of_item) forest (host helper)."""
    L = len(sets)
    off = np.zeros(L + 1, np.int32)
    off[1:] = np.cumsum([len(s) for s in sets])
    items = np.array([j for s in sets for j in s] or [0], np.int32)
    caps = np.ascontiguousarray(caps, np.int32) if L else np.zeros(1, np.int32)
    Lo = ctypes.c_int32()
    par = np.zeros(max(L, 1), np.int32)
    cp = np.zeros(max(L, 1), np.int32)
    leaf = np.zeros(M, np.int32)
    _check(lib().kp_tree_from_sets(M, L, _ptr(off), _ptr(items), _ptr(caps), ctypes.byref(Lo),
                                   _ptr(par), _ptr(cp), _ptr(leaf)))
    n = Lo.value
    return par[:n].copy(), cp[:n].copy(), leaf


from .driver import DualFn, solve  # noqa: E402  (autograd and the solve loop)
