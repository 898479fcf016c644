"""The allocation-free evaluation entry point (kp_eval_dual_noalloc), called
through the C ABI and compared with kp_eval_dual on the same inputs: x and R
bit-exact, g and P within 1e-9 relative.  Two calls in a row on one GPU, the
second with a smaller instance, so that anything the first call left in the
shared scratch array would show."""
import numpy as np
import pytest

import kpgen

gpu = pytest.mark.gpu
REL = 1e-9


def _kp():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2002_00352_amd as kp
    return kp, torch


CASES = [
    ("dense-topq", lambda: kpgen.make_instance(40000, 10, 12, seed=301, Q=3, budget_frac=0.1),
     lambda: kpgen.make_instance(3001, 10, 5, seed=302, Q=2, budget_frac=0.1)),
    ("csr-two-entries-per-row", lambda: kpgen.config_instance(3, N=60000),
     lambda: kpgen.config_instance(3, N=777)),
    ("dense-then-empty", lambda: kpgen.make_instance(5000, 7, 9, seed=303, Q=1, budget_frac=0.2),
     lambda: kpgen.make_instance(0, 7, 9, seed=304, Q=1, budget_frac=0.2)),
]


def _compare(kp, torch, inst, seed):
    prob = kp.Problem.from_host(inst)
    lam = torch.tensor(np.random.default_rng(seed).random(inst.K) * 0.2, dtype=torch.float64,
                       device="cuda")
    ref = kp.kp_eval_dual(prob, lam, want_x=True, ctx=kp.Context())
    R = torch.full((inst.K,), np.nan, dtype=torch.float64, device="cuda")
    g = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    P = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    x = torch.full((inst.N * inst.M,), 7, dtype=torch.uint8, device="cuda")
    kp.kp_eval_dual_noalloc(prob, lam, R, g, P, x)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), ref["x"].cpu().numpy())
    assert np.array_equal(R.cpu().numpy(), ref["R"].cpu().numpy())
    for a, b in ((g, ref["g"]), (P, ref["P"])):
        assert abs(a.item() - b.item()) <= REL * max(1.0, abs(b.item())), (a.item(), b.item())


@gpu
@pytest.mark.parametrize("name,big,small", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_eval_dual_twice(name, big, small):
    kp, torch = _kp()
    print("case", name, flush=True)
    _compare(kp, torch, big(), 11)
    _compare(kp, torch, small(), 12)


def test_noalloc_rejects_oversized_problems():
    """Sizes beyond what fits are refused on the host before any GPU work."""
    import ctypes
    import paper_2002_00352_amd as kp
    K = 600_000
    B = np.ones(K)
    par, cap, leaf = np.array([-1], np.int32), np.array([1], np.int32), np.zeros(1, np.int32)
    dummy = np.zeros(4, np.float32)
    s = kp.kp_problem()
    s.N, s.M, s.K = 0, 1, K
    s.p, s.b, s.b_format = dummy.ctypes.data, dummy.ctypes.data, 0
    s.B, s.L, s.parent, s.cap, s.leaf_of_item = B.ctypes.data, 1, par.ctypes.data, cap.ctypes.data, leaf.ctypes.data
    out = np.zeros(K + 2)
    rc = kp.lib().kp_eval_dual_noalloc(None, ctypes.byref(s), out.ctypes.data, out.ctypes.data,
                                       out.ctypes.data, out.ctypes.data, None)
    assert rc == kp.KP_ERR_UNSUPPORTED, kp.lib().kp_last_error()
    assert kp.lib().kp_last_error()
