"""GPU path (through the C ABI) against the CPU oracle on the same seeded
inputs.  Bars: decisions x bit-exact; R bit-exact (values on the 2^-24 grid
sum exactly in FP64); g and P within 1e-9 relative; DD and SCD multipliers
bit-exact."""
import dataclasses

import numpy as np
import pytest

import kpgen
import oracle
from util import make, random_instance, random_laminar

gpu = pytest.mark.gpu
REL = 1e-9


def _kp():
    import torch
    import paper_2002_00352_amd as kp
    assert torch.cuda.is_available()
    return kp, torch


def _lamd(torch, lam):
    return torch.tensor(np.asarray(lam, np.float64), device="cuda")


def _cases():
    rng = np.random.default_rng(1234)
    out = [
        ("c1-N10000", kpgen.config_instance(1)),
        ("c3-hier-csr-N3001", kpgen.config_instance(3, N=3001)),
        ("c2-lognormal-N2049", kpgen.config_instance(2, N=2049)),
        ("c4-M20K50-N700", kpgen.config_instance(4, N=700)),
        ("dense-ties-grid4", random_instance(rng, 500, 7, 3, Q=2, grid=4, zero_frac=0.3)),
        ("laminar-random-M12", random_instance(rng, 777, 12, 4, tree=random_laminar(12, rng))),
        ("csr-random-M9", random_instance(rng, 613, 9, 5, tree=random_laminar(9, rng), zero_frac=0.7).to_csr()),
        ("N1", random_instance(rng, 1, 5, 2, Q=2)),
        ("M1-K1", random_instance(rng, 300, 1, 1, Q=1)),
        ("M40-K3", random_instance(rng, 200, 40, 3, Q=7)),
        ("M63-K27-odd-tiles", random_instance(rng, 50, 63, 27, Q=9)),
        ("csr-wide-rows", random_instance(rng, 300, 16, 60, Q=4, zero_frac=0.2).to_csr()),
    ]
    return out


CASES = _cases()


@gpu
@pytest.mark.parametrize("name,inst", CASES, ids=[c[0] for c in CASES])
def test_eval_parity(name, inst):
    kp, torch = _kp()
    print("case", name, flush=True)
    prob = kp.Problem.from_host(inst)
    rng = np.random.default_rng(5)
    for lam in (np.zeros(inst.K), rng.random(inst.K) * 0.3, rng.random(inst.K) * 2.0):
        ev = kp.kp_eval_dual(prob, _lamd(torch, lam), want_x=True)
        ref = oracle.eval_dual(inst, lam)
        assert np.array_equal(ev["x"].cpu().numpy(), ref["x"])
        assert np.array_equal(ev["R"].cpu().numpy(), ref["R"])
        for key in ("g", "P"):
            a, b = ev[key].item(), ref[key]
            assert abs(a - b) <= REL * max(1.0, abs(b)), (key, a, b)


@gpu
@pytest.mark.parametrize("name,inst", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_dd_step_parity(name, inst):
    kp, torch = _kp()
    print("case", name, flush=True)
    prob = kp.Problem.from_host(inst)
    lam = np.full(inst.K, 0.05)
    lam_d = _lamd(torch, lam)
    for t in range(5):
        st = kp.kp_dd_step(prob, 1e-4, lam_d)
        ref = oracle.eval_dual(inst, lam, want_x=False)
        lam = oracle.dd_update(lam, 1e-4, ref["R"], inst.B)
        assert np.array_equal(lam_d.cpu().numpy(), lam), t


@gpu
@pytest.mark.parametrize("name,inst", CASES, ids=[c[0] for c in CASES])
def test_scd_sweep_parity(name, inst):
    """Three SCD iterations along the oracle's own trajectory: the GPU's
    lambda^{t+1} must equal the oracle's bit for bit at each step."""
    kp, torch = _kp()
    print("case", name, flush=True)
    prob = kp.Problem.from_host(inst)
    lam = np.zeros(inst.K)
    for t in range(3):
        sw = kp.kp_scd_sweep(prob, _lamd(torch, lam))
        want = oracle.scd_sweep(inst, lam)
        got = sw["lam"].cpu().numpy()
        assert np.array_equal(got, want), (t, got, want)
        ref = oracle.eval_dual(inst, lam, want_x=False)
        assert np.array_equal(sw["R"].cpu().numpy(), ref["R"])
        lam = want


@gpu
def test_scd_sweep_parity_from_random_points():
    kp, torch = _kp()
    inst = kpgen.config_instance(1, N=5000)
    prob = kp.Problem.from_host(inst)
    rng = np.random.default_rng(9)
    for _ in range(6):
        lam = rng.random(inst.K) * 3
        got = kp.kp_scd_sweep(prob, _lamd(torch, lam))["lam"].cpu().numpy()
        assert np.array_equal(got, oracle.scd_sweep(inst, lam))


@gpu
def test_scd_masked_cyclic_parity():
    kp, torch = _kp()
    inst = kpgen.config_instance(3, N=2000)
    prob = kp.Problem.from_host(inst)
    lam = np.full(inst.K, 0.5)
    for k in (0, 7, 19):
        mask = np.zeros(inst.K, np.uint8)
        mask[k] = 1
        got = kp.kp_scd_sweep(prob, _lamd(torch, lam), kmask=mask)["lam"].cpu().numpy()
        want = oracle.scd_sweep(inst, lam, ks=[k])
        assert np.array_equal(got, want)


@gpu
def test_cd_modes_trajectories():
    """Cyclic and block coordinate descent (Sec. 4.3.2) along whole driver
    trajectories from lambda = 0 on the dense (general kernel) and the
    hierarchical sparse (uniform-row kernel) workloads: every update equals
    the oracle's masked sweep of the same coordinates bit for bit."""
    kp, torch = _kp()
    for inst in (kpgen.config_instance(2, N=3000), kpgen.config_instance(3, N=4000)):
        prob = kp.Problem.from_host(inst)
        K = inst.K
        for w in (1, 4, K // 2):
            ctx = kp.Context()
            lam = np.zeros(K)
            for t in range(6):
                ks = [(t * w + q) % K for q in range(w)]
                mask = np.zeros(K, np.uint8)
                mask[ks] = 1
                got = kp.kp_scd_sweep(prob, _lamd(torch, lam), kmask=mask, ctx=ctx)["lam"].cpu().numpy()
                want = oracle.scd_sweep(inst, lam, ks=ks)
                assert np.array_equal(got, want), (inst.name, w, t)
                lam = want


INTERP_CASES = [
    ("c1-dense", lambda: kpgen.config_instance(1, N=6000)),
    ("c3-csr-uniform-rows", lambda: kpgen.config_instance(3, N=20000)),
    ("c2-dense-general", lambda: kpgen.config_instance(2, N=3000)),
]


@gpu
@pytest.mark.parametrize("name,mk", INTERP_CASES, ids=[c[0] for c in INTERP_CASES])
def test_interp_reduce_trajectory(name, mk):
    """Sec. 5.2's interpolated reduce on the GPU (kp_set_reduce): along a
    trajectory from lambda = 0, every update equals the oracle's interpolated
    SCD (the same buckets around lambda^t and central half-widths) bit for
    bit, and so do the drivers' iterates."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    prob = kp.Problem.from_host(inst)
    ctx = kp.Context()
    ctx.set_reduce("interp")
    lam = np.zeros(inst.K)
    for t in range(8):
        want = oracle.scd_sweep_interp(inst, lam)
        got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
        assert np.array_equal(got, want), (t, np.flatnonzero(got != want), got, want)
        lam = want
    if name == "c1-dense":
        # the drivers' iterates agree at every step they share
        _, h = kp.solve(prob, "interp", tol=1e-3, max_iter=30)
        ref = oracle.solve(inst, "interp", tol=1e-3, max_iter=30)
        for a, b in zip(h, ref):
            assert np.array_equal(a["lam"], b["lam"])


def _off_grid(inst):
    """The instance with every cost divided by 3 in fp32 (values off the
    2^-24 grid, so FP64 sums of them round) and the budgets recomputed."""
    if inst.b is not None:
        b = (inst.b.astype(np.float64) / 3.0).astype(np.float32)
        D = b.astype(np.float64).reshape(-1, inst.K).sum(axis=0)
        out = dataclasses.replace(inst, b=b)
    else:
        val = (inst.val.astype(np.float64) / 3.0).astype(np.float32)
        D = np.bincount(inst.col, weights=val.astype(np.float64), minlength=inst.K)
        out = dataclasses.replace(inst, val=val)
    frac = inst.B.sum() / max(1e-300, float((inst.b.astype(np.float64).reshape(-1, inst.K).sum(axis=0)
                                              if inst.b is not None else
                                              np.bincount(inst.col, weights=inst.val.astype(np.float64),
                                                          minlength=inst.K)).sum()))
    out.B = np.maximum(frac * D, 1e-3)
    return out


OFFGRID_CASES = [
    ("c3-csr-uniform-rows", lambda: _off_grid(kpgen.config_instance(3, N=30000))),
    ("c1-dense", lambda: _off_grid(kpgen.config_instance(1, N=8000))),
    ("c2-dense-general", lambda: _off_grid(kpgen.config_instance(2, N=4000))),
    ("laminar-dense-K9", lambda: _off_grid(random_instance(np.random.default_rng(71), 3000, 12, 9,
                                                           tree=random_laminar(12, np.random.default_rng(72)),
                                                           frac=0.15))),
]


@gpu
@pytest.mark.parametrize("name,mk", OFFGRID_CASES, ids=[c[0] for c in OFFGRID_CASES])
def test_off_grid_costs_trajectory_twice(name, mk):
    """Costs off the 2^-24 grid (every cost divided by 3 in fp32): along an
    SCD trajectory from lambda = 0, with the window search on, every update
    equals the oracle's (whose reduce sums exactly) bit for bit; the same
    trajectory on a second fresh context gives the same multipliers bit for
    bit (the threshold sums are exact integer sums, order-free); decisions
    are bit-exact and consumption within 1e-12 relative."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    prob = kp.Problem.from_host(inst)
    runs = []
    for rep in range(2):
        ctx = kp.Context()
        lam = np.zeros(inst.K)
        traj = []
        for t in range(7):
            if rep == 0:
                ev = kp.kp_eval_dual(prob, _lamd(torch, lam), want_x=True, ctx=ctx)
                ref = oracle.eval_dual(inst, lam)
                assert np.array_equal(ev["x"].cpu().numpy(), ref["x"]), t
                R = ev["R"].cpu().numpy()
                assert np.all(np.abs(R - ref["R"]) <= 1e-12 * np.maximum(1.0, np.abs(ref["R"]))), t
                want = oracle.scd_sweep(inst, lam)
            got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
            if rep == 0:
                assert np.array_equal(got, want), (t, np.flatnonzero(got != want))
            traj.append(got)
            lam = got
        runs.append(traj)
        print("window searches", ctx.window_stats(), flush=True)
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


SAMPLED_CASES = [
    ("c3-csr-declared-rows", lambda: kpgen.config_instance(3, N=20000), None),
    # many users: the sample's window over every user, exact tests and walks
    # that stop below it
    ("c3-csr-300k", lambda: kpgen.config_instance(3, N=300000), None),
    ("c2-dense", lambda: kpgen.config_instance(2, N=4000), None),
    ("c3-csr-general-rows", lambda: kpgen.config_instance(3, N=6000), 0),
    ("laminar-dense-K9", lambda: random_instance(np.random.default_rng(81), 5000, 12, 9,
                                                 tree=random_laminar(12, np.random.default_rng(82)),
                                                 frac=0.15), None),
]


@gpu
@pytest.mark.parametrize("name,mk,row_nnz", SAMPLED_CASES, ids=[c[0] for c in SAMPLED_CASES])
def test_sampled_start_trajectory(name, mk, row_nnz):
    """Full searches that start from a strided sample's threshold
    (kp_set_sampled_start, here on small instances): along SCD trajectories
    from lambda = 0 -- with windows (the sample's threshold opens a window
    away from lambda^t, a miss falls back to buckets around it), and with
    every iteration a full search around it -- every update equals the
    oracle's bit for bit (the sample only decides the cost), for uniform-row
    CSR, general CSR and dense costs."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    if row_nnz is None:
        prob = kp.Problem.from_host(inst)
    else:
        host = kp.Problem.from_host(inst)
        prob = kp.Problem(host.p, inst.B, inst.tree.parent, inst.tree.cap, inst.tree.leaf_of_item,
                          rowptr=host.rowptr, col=host.col, val=host.val, N=inst.N, M=inst.M, K=inst.K,
                          row_nnz=row_nnz)
    ctxs = [kp.Context(), kp.Context()]
    for c in ctxs:
        c.set_sampled_start(1000)
    ctxs[1].set_window(False)
    lam = np.zeros(inst.K)
    for t in range(6):
        want = oracle.scd_sweep(inst, lam)
        for ctx in ctxs:
            got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
            assert np.array_equal(got, want), (t, np.flatnonzero(got != want))
        lam = want


@gpu
def test_dual_autograd_matches_oracle_gradient():
    kp, torch = _kp()
    inst = kpgen.config_instance(4, N=3000)
    prob = kp.Problem.from_host(inst)
    rng = np.random.default_rng(3)
    for _ in range(3):
        lam = rng.random(inst.K) / inst.K
        lam_t = torch.tensor(lam, device="cuda", requires_grad=True)
        g = kp.DualFn.apply(lam_t, prob)
        g.backward()
        ref = oracle.eval_dual(inst, lam, want_x=False)
        assert abs(g.item() - ref["g"]) <= REL * abs(ref["g"])
        assert np.array_equal(lam_t.grad.cpu().numpy(), inst.B - ref["R"])


@gpu
def test_unaligned_dense_costs():
    """A dense cost array that is not 16-byte aligned takes the scalar
    staging path and gives the same results."""
    kp, torch = _kp()
    rng = np.random.default_rng(77)
    inst = random_instance(rng, 900, 9, 5, Q=3)
    prob = kp.Problem.from_host(inst)
    big = torch.empty(inst.N * inst.M * inst.K + 1, dtype=torch.float32, device="cuda")
    big[1:] = prob.b
    prob2 = kp.Problem(prob.p, inst.B, inst.tree.parent, inst.tree.cap, inst.tree.leaf_of_item,
                       b=big[1:], N=inst.N, M=inst.M, K=inst.K)
    assert prob2.b.data_ptr() % 16 != 0
    lam = np.array([0.1, 0.2, 0.05, 0.3, 0.15])
    ev = kp.kp_eval_dual(prob2, _lamd(torch, lam), want_x=True)
    ref = oracle.eval_dual(inst, lam)
    assert np.array_equal(ev["x"].cpu().numpy(), ref["x"])
    assert np.array_equal(ev["R"].cpu().numpy(), ref["R"])
    got = kp.kp_scd_sweep(prob2, _lamd(torch, lam))["lam"].cpu().numpy()
    assert np.array_equal(got, oracle.scd_sweep(inst, lam))


DENSE_LANE_CASES = [
    ("M10-K10-top3-ragged", lambda: random_instance(np.random.default_rng(61), 4099, 10, 10, Q=3)),
    ("M3-K1", lambda: random_instance(np.random.default_rng(62), 777, 3, 1, Q=1)),
    ("M7-K16-laminar", lambda: random_instance(np.random.default_rng(63), 1500, 7, 16,
                                               tree=random_laminar(7, np.random.default_rng(64)))),
    ("M13-K5-ties", lambda: random_instance(np.random.default_rng(65), 2000, 13, 5, Q=4, grid=5)),
    ("M16-K16-zeros", lambda: random_instance(np.random.default_rng(66), 640, 16, 16, Q=6, zero_frac=0.3)),
    ("M12-K4-one-user", lambda: random_instance(np.random.default_rng(67), 1, 12, 4, Q=2)),
    ("c2-like", lambda: kpgen.config_instance(2, N=8000)),
    # exact item and knapsack counts (the kernels with K fixed at compile time)
    ("M8-K10-top2", lambda: random_instance(np.random.default_rng(68), 3001, 8, 10, Q=2)),
    ("M16-K10-top4", lambda: random_instance(np.random.default_rng(69), 2500, 16, 10, Q=4)),
    ("M12-K2-laminar", lambda: random_instance(np.random.default_rng(70), 4000, 12, 2,
                                               tree=random_laminar(12, np.random.default_rng(71)))),
]


@gpu
@pytest.mark.parametrize("name,mk", DENSE_LANE_CASES, ids=[c[0] for c in DENSE_LANE_CASES])
def test_dense_lane_evaluation(name, mk):
    """The lane-per-user evaluation of dense costs (M <= 16, K <= 16): it is
    the kernel that runs, x and R equal the oracle's (and the general
    kernel's) bit for bit, g and P within 1e-9; also from a cost array that
    is not 16-byte aligned, and through DD steps."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    prob = kp.Problem.from_host(inst)
    rng = np.random.default_rng(len(name))
    lam = rng.uniform(0.0, 0.6, inst.K)
    ref = oracle.eval_dual(inst, lam)
    ctx = kp.Context()
    ev = kp.kp_eval_dual(prob, _lamd(torch, lam), want_x=True, ctx=ctx)
    assert ctx.launch_shape()[0] == 2, ctx.launch_shape()
    assert np.array_equal(ev["x"].cpu().numpy(), ref["x"])
    assert np.array_equal(ev["R"].cpu().numpy(), ref["R"])
    assert abs(ev["g"].item() - ref["g"]) <= REL * max(1.0, abs(ref["g"]))
    assert abs(ev["P"].item() - ref["P"]) <= REL * max(1.0, abs(ref["P"]))
    gen = kp.Context()
    gen.set_kernel_choice(False)
    evg = kp.kp_eval_dual(prob, _lamd(torch, lam), want_x=True, ctx=gen)
    assert gen.launch_shape()[0] == 0
    assert np.array_equal(evg["x"].cpu().numpy(), ev["x"].cpu().numpy())
    assert np.array_equal(evg["R"].cpu().numpy(), ev["R"].cpu().numpy())
    # unaligned costs: the scalar staging path
    big = torch.empty(inst.N * inst.M * inst.K + 1, dtype=torch.float32, device="cuda")
    big[1:] = prob.b
    prob2 = kp.Problem(prob.p, inst.B, inst.tree.parent, inst.tree.cap, inst.tree.leaf_of_item,
                       b=big[1:], N=inst.N, M=inst.M, K=inst.K)
    ev2 = kp.kp_eval_dual(prob2, _lamd(torch, lam), want_x=True, ctx=ctx)
    assert ctx.launch_shape()[0] == 2
    assert np.array_equal(ev2["x"].cpu().numpy(), ref["x"])
    assert np.array_equal(ev2["R"].cpu().numpy(), ref["R"])
    # dual descent steps (Eq.14) through the same kernel
    l_gpu = _lamd(torch, lam)
    l_ref = lam.copy()
    alpha = 1e-3
    for _ in range(3):
        kp.kp_dd_step(prob, alpha, l_gpu, ctx=ctx)
        r = oracle.eval_dual(inst, l_ref, want_x=False)
        l_ref = oracle.dd_update(l_ref, alpha, r["R"], inst.B)
        assert np.array_equal(l_gpu.cpu().numpy(), l_ref)


def _random_case(seed):
    """A small instance of random shape: N 1..700, M 1..20, K 1..20, dense
    or CSR (uniform rows declared, or general rows), top-Q or a random
    laminar family, profits of one of the generator's distributions."""
    rng = np.random.default_rng(seed)
    N = int(rng.integers(1, 700))
    M = int(rng.integers(1, 21))
    K = int(rng.integers(1, 21))
    tree = random_laminar(M, rng) if rng.random() < 0.5 else kpgen.tree_topq(M, int(rng.integers(1, M + 1)))
    fmt = int(rng.integers(0, 3))   # 0 dense, 1 CSR with 1-2 entries per row (declared), 2 general CSR
    d = int(rng.integers(1, min(K, 2) + 1))
    inst = kpgen.make_instance(N, M, K, seed=5000 + seed, p_dist=["uniform", "exp1", "lognormal"][seed % 3],
                               tree=tree, csr_d=0 if fmt == 0 else d, budget_frac=float(rng.uniform(0.05, 0.4)))
    return inst, fmt, rng


@gpu
@pytest.mark.parametrize("seed", list(range(40)))
def test_random_shapes_parity(seed):
    """Random shapes (every kernel path: dense lane-per-user, uniform-row,
    general dense and CSR): the evaluation (x, R bit-exact; g, P within
    1e-9) and three SCD iterations from a random point (multipliers
    bit-exact, windows on) equal the oracle's."""
    kp, torch = _kp()
    inst, fmt, rng = _random_case(seed)
    print("case", seed, inst.N, inst.M, inst.K, fmt, flush=True)
    if fmt == 2:
        host = kp.Problem.from_host(inst)
        prob = kp.Problem(host.p, inst.B, inst.tree.parent, inst.tree.cap, inst.tree.leaf_of_item,
                          rowptr=host.rowptr, col=host.col, val=host.val, N=inst.N, M=inst.M, K=inst.K,
                          row_nnz=0)
    else:
        prob = kp.Problem.from_host(inst)
    lam = rng.uniform(0.0, 1.5, inst.K) * (rng.random(inst.K) < 0.8)
    ctx = kp.Context()
    ev = kp.kp_eval_dual(prob, _lamd(torch, lam), want_x=True, ctx=ctx)
    ref = oracle.eval_dual(inst, lam)
    assert np.array_equal(ev["x"].cpu().numpy(), ref["x"])
    assert np.array_equal(ev["R"].cpu().numpy(), ref["R"])
    assert abs(ev["g"].item() - ref["g"]) <= REL * max(1.0, abs(ref["g"]))
    assert abs(ev["P"].item() - ref["P"]) <= REL * max(1.0, abs(ref["P"]))
    for t in range(3):
        want = oracle.scd_sweep(inst, lam)
        got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
        assert np.array_equal(got, want), (t, np.flatnonzero(got != want))
        lam = want


@gpu
@pytest.mark.parametrize("fmt", ["dense", "csr-uniform-rows"])
def test_empty_instance(fmt):
    """N = 0: no consumption, g = lambda.B, every SCD multiplier 0 (dense
    costs, and per-item CSR rows that would take the uniform-row kernel)."""
    kp, torch = _kp()
    rng = np.random.default_rng(0)
    inst = random_instance(rng, 4, 3, 2, Q=1) if fmt == "dense" else \
        kpgen.make_instance(4, 3, 2, seed=5, Q=1, csr_d=1, budget_frac=0.5)
    prob = kp.Problem.from_host(inst)
    prob.s.N = 0
    lam = np.array([0.5, 0.25])
    ctx = kp.Context()
    ev = kp.kp_eval_dual(prob, _lamd(torch, lam), ctx=ctx)
    assert ev["R"].cpu().numpy().tolist() == [0.0, 0.0]
    assert ev["g"].item() == 0.5 * inst.B[0] + 0.25 * inst.B[1]
    for _ in range(2):   # the second call may start with windows
        sw = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)
        assert sw["lam"].cpu().numpy().tolist() == [0.0, 0.0]


@gpu
def test_validate_inputs_flags_bad_values():
    kp, torch = _kp()
    rng = np.random.default_rng(0)
    inst = random_instance(rng, 50, 4, 3, Q=2)
    prob = kp.Problem.from_host(inst)
    kp.kp_validate_inputs(prob)
    prob.b[17] = float("nan")
    with pytest.raises(kp.KPError) as e:
        kp.kp_validate_inputs(prob)
    assert e.value.status == -3
    prob.b[17] = -1.0
    with pytest.raises(kp.KPError) as e:
        kp.kp_validate_inputs(prob)
    assert e.value.status == -4


def _off_grid_fix():
    rng = np.random.default_rng(11)
    N, M, K = 20000, 6, 3
    p = rng.random((N, M)).astype(np.float32)
    b = (rng.random((N, M, K)) * 1.37).astype(np.float32)
    return make(p, b, 0.05 * b.astype(np.float64).sum(axis=(0, 1)), kpgen.tree_topq(M, 2))


def _identical_users_fix():
    # every user the same: one G value, so one bin and ties decided by index
    rng = np.random.default_rng(5)
    M, K = 8, 3
    p = rng.integers(1, 64, size=(1, M)) / 64.0
    b = rng.integers(1, 64, size=(1, M, K)) / 64.0
    N = 30000
    p = np.repeat(p, N, axis=0)
    b = np.repeat(b, N, axis=0)
    return make(p, b, 0.1 * b.sum(axis=(0, 1)), kpgen.tree_topq(M, 3))


FIX_CASES = [
    ("c1-underpriced", lambda: kpgen.config_instance(1, N=6000), [1.2, 1.25]),
    ("c3-hier-csr", lambda: kpgen.config_instance(3, N=4000), None),
    ("dense-ties", lambda: random_instance(np.random.default_rng(3), 700, 6, 4, Q=2, grid=6), None),
    ("feasible-already", lambda: kpgen.config_instance(1, N=3000), [3.0, 3.0]),
    # many bins, a threshold bin of several 4096-user chunks, a strided sample
    ("c3-2M", lambda: kpgen.config_instance(3, N=2_000_000), None),
    ("c3-2M-near", lambda: kpgen.config_instance(3, N=2_000_000), [3.1] * 20),
    ("off-grid", _off_grid_fix, [0.1, 0.1, 0.1]),
    ("identical-users", _identical_users_fix, [0.05, 0.05, 0.05]),
    # many violated knapsacks: one bin and LDS accumulators at 2000 slots,
    # global-memory accumulators past 48 KB at 4000
    ("wide-K2000", lambda: random_instance(np.random.default_rng(71), 300, 3, 2000, Q=2, frac=0.02), [1e-5] * 2000),
    ("wide-K4000", lambda: random_instance(np.random.default_rng(72), 200, 2, 4000, Q=1, frac=0.02), [1e-5] * 4000),
]


@gpu
@pytest.mark.parametrize("name,mk,lam", FIX_CASES, ids=[c[0] for c in FIX_CASES])
def test_primal_fixup_parity(name, mk, lam):
    """Post-processing (Sec. 5.4): the reset users, x, R and n_reset equal the
    oracle's; P within 1e-9; the result is feasible."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    if lam is None:
        lam = np.full(inst.K, 0.05)
    lam = np.asarray(lam, np.float64)
    prob = kp.Problem.from_host(inst)
    fx = kp.kp_primal_fixup(prob, _lamd(torch, lam), want_x=True)
    ref = oracle.fixup(inst, lam, mode=0)
    assert fx["n_reset"].item() == ref["n_reset"]
    assert np.array_equal(fx["x"].cpu().numpy(), ref["x"])
    if name == "off-grid":
        # the consumption left is rounded once here and re-summed there
        assert np.allclose(fx["R"].cpu().numpy(), ref["R"], rtol=REL, atol=0)
    else:
        assert np.array_equal(fx["R"].cpu().numpy(), ref["R"])
    assert abs(fx["P"].item() - ref["P"]) <= REL * abs(ref["P"])
    assert np.all(fx["R"].cpu().numpy() <= inst.B * (1 + 1e-12))


@gpu
def test_solve_to_gap_c1():
    """The driver reaches a relative duality gap <= 1e-3 on the small
    plain-SCD workload, like the oracle's own driver."""
    kp, torch = _kp()
    inst = kpgen.config_instance(1)
    prob = kp.Problem.from_host(inst)
    lam, hist = kp.solve(prob, "scd", tol=1e-3, max_iter=60)
    assert hist[-1]["gap_rel"] <= 1e-3
    ref = oracle.solve(inst, "scd", tol=1e-3, max_iter=60)
    assert ref[-1]["gap_rel"] <= 1e-3
    # same iterates: the multipliers are bit-exact at every step
    for a, b in zip(hist, ref):
        assert np.array_equal(a["lam"], b["lam"])


@gpu
def test_batched_sweep_parity():
    """Ragged batch (uneven N, M, K, Q): one launch per pass; every
    instance's lambda^{t+1} and statistics equal the oracle's."""
    kp, torch = _kp()
    insts = kpgen.batched_instances(run=0, n=24, max_N=2500)
    probs = [kp.Problem.from_host(i) for i in insts]
    lams = [np.zeros(i.K) for i in insts]
    for t in range(2):
        outs, stats = kp.kp_scd_sweep_batched(probs, [_lamd(torch, l) for l in lams])
        stats = stats.cpu().numpy()
        off = 0
        for s, inst in enumerate(insts):
            want = oracle.scd_sweep(inst, lams[s])
            got = outs[s].cpu().numpy()
            assert np.array_equal(got, want), (t, s, got, want)
            ref = oracle.eval_dual(inst, lams[s], want_x=False)
            K = inst.K
            assert np.array_equal(stats[off:off + K], ref["R"])
            assert abs(stats[off + K] - ref["g"]) <= REL * max(1.0, abs(ref["g"]))
            assert abs(stats[off + K + 1] - ref["P"]) <= REL * max(1.0, abs(ref["P"]))
            off += K + 2
            lams[s] = want


@gpu
@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_plan_graph_replays(use_graph):
    """A batched plan stepped several times (graph replays alternating the
    two multiplier buffers, with host work in between) follows the oracle's
    SCD trajectory for every instance at every step.  With the graph, an
    iteration's later passes are split on the device and replayed with the
    first; they run the same passes as the host-split plan."""
    kp, torch = _kp()
    insts = kpgen.batched_instances(run=1, n=12, max_N=2000)
    probs = [kp.Problem.from_host(i) for i in insts]
    ctx = kp.Context()
    ref_ctx = kp.Context()
    ctx.set_timing(True)       # (passes are counted over timed iterations)
    ref_ctx.set_timing(True)
    plan = kp.BatchedSCD(probs, use_graph=use_graph, ctx=ctx)
    ref = kp.BatchedSCD(probs, use_graph=False, ctx=ref_ctx)
    lams = [np.zeros(i.K) for i in insts]
    for t in range(6):
        outs, stats = plan.step()
        routs, _ = ref.step()
        torch.cuda.synchronize()
        for s, inst in enumerate(insts):
            want = oracle.scd_sweep(inst, lams[s])
            assert np.array_equal(outs[s].cpu().numpy(), want), (use_graph, t, s)
            assert np.array_equal(routs[s].cpu().numpy(), want), (t, s)
            lams[s] = want
        assert ctx.batched_passes() == ref_ctx.batched_passes(), t
    print("passes", ctx.batched_passes(), flush=True)
    plan.close()
    ref.close()


@gpu
def test_autotuner_reaches_every_kernel(tmp_path):
    """Every tuning candidate launches the shape it asks for, as the library
    reports it: users per tile and grid of the general kernel (dense costs),
    the grid of the uniform-row kernel (CSR with two entries per item row),
    and the LDS budget and block split of a batched plan.  Every shape gives
    the oracle's decisions, consumption and SCD updates."""
    kp, torch = _kp()
    from paper_2002_00352_amd import autotune
    # general kernel
    inst = kpgen.config_instance(2, N=6000)
    prob = kp.Problem.from_host(inst)
    ctx = kp.Context()
    lam = np.full(inst.K, 0.3)
    want = oracle.scd_sweep(inst, lam)
    ref = oracle.eval_dual(inst, lam)
    shapes = []
    for u, g in [(4, 512), (16, 64), (40, 96)]:
        autotune.apply(ctx, prob, (u, g))
        ev = kp.kp_eval_dual(prob, _lamd(torch, lam), want_x=True, ctx=ctx)
        shape = ctx.launch_shape()
        assert shape == (0, u, min(g, -(-inst.N // u))), (u, g, shape)
        assert np.array_equal(ev["x"].cpu().numpy(), ref["x"])
        assert np.array_equal(ev["R"].cpu().numpy(), ref["R"])
        got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
        assert ctx.launch_shape()[:2] == (0, u)
        assert np.array_equal(got, want), (u, g)
        shapes.append(shape)
    assert len(set(shapes)) == 3
    path = str(tmp_path / "tune.json")
    choice = autotune.tune(prob, ctx=ctx, candidates=[(8, 512), (32, 2048)], path=path)
    assert choice in [(8, 512), (32, 2048)]
    rec = autotune.load_cache(path)[autotune.shape_key(prob) + "|scd"]
    assert rec["kernel"] == "general" and len(rec["tried"]) == 2
    # uniform-row kernel: the grid only
    inst3 = kpgen.config_instance(3, N=20000)
    prob3 = kp.Problem.from_host(inst3)
    assert prob3.row_nnz == 2
    ctx3 = kp.Context()
    lam3 = np.full(inst3.K, 0.05)
    want3 = oracle.scd_sweep(inst3, lam3)
    ref3 = oracle.eval_dual(inst3, lam3)
    grids = []
    for g in (16, 48, 79):
        autotune.apply(ctx3, prob3, (0, g))
        ev = kp.kp_eval_dual(prob3, _lamd(torch, lam3), want_x=True, ctx=ctx3)
        assert ctx3.launch_shape() == (1, 64, g), (g, ctx3.launch_shape())
        assert np.array_equal(ev["x"].cpu().numpy(), ref3["x"])
        assert np.array_equal(ev["R"].cpu().numpy(), ref3["R"])
        got = kp.kp_scd_sweep(prob3, _lamd(torch, lam3), ctx=ctx3)["lam"].cpu().numpy()
        assert ctx3.launch_shape()[0] == 1
        assert np.array_equal(got, want3), g
        grids.append(g)
    choice3 = autotune.tune(prob3, ctx=ctx3, path=path)
    assert choice3[0] == 0 and choice3[1] in autotune.ELL_GRIDS
    assert autotune.load_cache(path)[autotune.shape_key(prob3) + "|scd"]["kernel"] == "uniform-row"
    # batched plan: LDS budget and block split
    rng = np.random.default_rng(91)
    insts = [kpgen.make_instance(int(rng.integers(200, 3000)), int(rng.integers(4, 20)),
                                 int(rng.integers(1, 9)), seed=900 + s, Q=int(rng.integers(1, 4)),
                                 budget_frac=0.1) for s in range(6)]
    probs = [kp.Problem.from_host(i) for i in insts]
    bshapes = []
    for lds, mult in [(16384, 4), (65536, 128)]:
        bctx = kp.Context()
        bctx.set_batched_tuning(lds, mult)
        bs = kp.BatchedSCD(probs, ctx=bctx)
        shape = bs.shape()
        assert shape[1] <= lds, shape
        bshapes.append(shape)
        lams = [np.zeros(i.K) for i in insts]
        for t in range(2):
            outs, _ = bs.step()
            for s_, inst_ in enumerate(insts):
                w = oracle.scd_sweep(inst_, lams[s_])
                assert np.array_equal(outs[s_].cpu().numpy(), w), (lds, mult, t, s_)
                lams[s_] = w
        bs.close()
    assert bshapes[0] != bshapes[1]
    assert bshapes[0][3] < bshapes[1][3], bshapes


@gpu
def test_structure_declaration_not_cached_by_address():
    """A CSR instance with two entries per item row, freed, then one of the
    same shape whose rows are not uniform, allocated on the same default
    context at the recycled addresses (torch's caching allocator): the new
    problem declares no uniform rows, runs the general kernel and matches the
    oracle.  A false declaration is caught by input validation."""
    kp, torch = _kp()
    inst = kpgen.config_instance(3, N=20000)
    prob = kp.Problem.from_host(inst)
    assert prob.row_nnz == 2 and kp.kp_csr_row_nnz(prob) == 2
    lam = np.full(inst.K, 0.05)
    ev = kp.kp_eval_dual(prob, _lamd(torch, lam), want_x=True)
    assert np.array_equal(ev["x"].cpu().numpy(), oracle.eval_dual(inst, lam)["x"])
    assert kp.default_context().launch_shape()[0] == 1
    addrs = (prob.rowptr.data_ptr(), prob.col.data_ptr(), prob.val.data_ptr())
    del prob, ev
    torch.cuda.synchronize()
    # move one stored entry of every even row to the next row: same nnz, same
    # array sizes, rows of 1 and 3 entries (columns kept distinct and ascending)
    col = inst.col.reshape(-1, 2).copy()
    val = inst.val.reshape(-1, 2).copy()
    nrows = inst.N * inst.M
    lens = np.full(nrows, 2, np.int64)
    cols, vals = [], []
    for r in range(0, nrows - 1, 2):
        extra_c, extra_v = col[r, 1], val[r, 1]
        nxt = sorted(set(col[r + 1].tolist()) | {int(extra_c)})
        if len(nxt) != 3:          # the moved column is already in the next row
            cols += [col[r].tolist(), col[r + 1].tolist()]
            vals += [val[r].tolist(), val[r + 1].tolist()]
            continue
        lens[r], lens[r + 1] = 1, 3
        vmap = {int(col[r + 1, 0]): val[r + 1, 0], int(col[r + 1, 1]): val[r + 1, 1], int(extra_c): extra_v}
        cols += [[int(col[r, 0])], nxt]
        vals += [[val[r, 0]], [vmap[c] for c in nxt]]
    if nrows % 2:
        cols.append(col[-1].tolist())
        vals.append(val[-1].tolist())
    bad = dataclasses.replace(inst, rowptr=np.concatenate([[0], np.cumsum(lens)]).astype(np.int64),
                              col=np.array([c for r in cols for c in r], np.int32),
                              val=np.array([v for r in vals for v in r], np.float32))
    assert bad.rowptr[-1] == inst.rowptr[-1] and (lens != 2).any()
    prob2 = kp.Problem.from_host(bad)
    reused = (prob2.rowptr.data_ptr(), prob2.col.data_ptr(), prob2.val.data_ptr()) == addrs
    print("addresses reused:", reused, flush=True)
    assert prob2.row_nnz == 0
    ctx = kp.default_context()
    for t in range(3):
        ev = kp.kp_eval_dual(prob2, _lamd(torch, lam), want_x=True)
        assert ctx.launch_shape()[0] == 0
        ref = oracle.eval_dual(bad, lam)
        assert np.array_equal(ev["x"].cpu().numpy(), ref["x"])
        assert np.array_equal(ev["R"].cpu().numpy(), ref["R"])
        want = oracle.scd_sweep(bad, lam)
        got = kp.kp_scd_sweep(prob2, _lamd(torch, lam))["lam"].cpu().numpy()
        assert np.array_equal(got, want), t
        lam = want
    liar = kp.Problem(prob2.p, bad.B, bad.tree.parent, bad.tree.cap, bad.tree.leaf_of_item,
                      rowptr=prob2.rowptr, col=prob2.col, val=prob2.val, N=bad.N, M=bad.M, K=bad.K,
                      row_nnz=2)
    with pytest.raises(kp.KPError) as e:
        kp.kp_validate_inputs(liar)
    assert e.value.status == kp.KP_ERR_INVALID
    kp.kp_validate_inputs(kp.Problem.from_host(inst))


ELL_CASES = [
    ("c3-ragged-N12345", lambda: kpgen.config_instance(3, N=12345)),
    ("csr-d1-topq", lambda: kpgen.make_instance(3001, 12, 9, seed=41, Q=3, csr_d=1, budget_frac=0.1)),
    ("csr-d2-laminar-M16", lambda: kpgen.make_instance(1500, 16, 7, seed=42, csr_d=2, budget_frac=0.08,
                                                       tree=random_laminar(16, np.random.default_rng(4)))),
    ("c3-single-user", lambda: kpgen.config_instance(3, N=1)),
    # K = 40 with M = 16, D = 2: 33 or more statistics rows in one chunk (one
    # lane per row part) and a short remainder chunk; top-4 takes the
    # compact statistics path, top-6 the other one
    ("csr-d2-M16-K40-top4", lambda: kpgen.make_instance(2100, 16, 40, seed=43, Q=4, csr_d=2, budget_frac=0.1)),
    ("csr-d2-M16-K40-top6", lambda: kpgen.make_instance(2100, 16, 40, seed=44, Q=6, csr_d=2, budget_frac=0.1)),
    # M = 10 with the knapsack count compiled in: K = 10 on the non-compact
    # statistics path, K = 20 with one entry per item row and laminar sets
    ("csr-d2-M10-K10-top6", lambda: kpgen.make_instance(3333, 10, 10, seed=45, Q=6, csr_d=2, budget_frac=0.1)),
    ("csr-d1-M10-K20-laminar", lambda: kpgen.make_instance(2999, 10, 20, seed=46, csr_d=1, budget_frac=0.08,
                                                           tree=random_laminar(10, np.random.default_rng(5)))),
]


@gpu
@pytest.mark.parametrize("name,mk", ELL_CASES, ids=[c[0] for c in ELL_CASES])
def test_uniform_row_kernel_parity(name, mk):
    """CSR with the same number of entries per item row takes the lean
    per-user kernel: decisions, statistics and SCD updates equal the
    oracle's and the general kernel's."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    prob = kp.Problem.from_host(inst)
    lean = kp.Context()
    general = kp.Context()
    general.set_kernel_choice(False)
    lam = np.zeros(inst.K)
    for t in range(3):
        for ctx in (lean, general):
            ev = kp.kp_eval_dual(prob, _lamd(torch, lam), want_x=True, ctx=ctx)
            ref = oracle.eval_dual(inst, lam)
            assert np.array_equal(ev["x"].cpu().numpy(), ref["x"])
            assert np.array_equal(ev["R"].cpu().numpy(), ref["R"])
            for key in ("g", "P"):
                assert abs(ev[key].item() - ref[key]) <= REL * max(1.0, abs(ref[key]))
        want = oracle.scd_sweep(inst, lam)
        for ctx in (lean, general):
            got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
            assert np.array_equal(got, want), (t, got, want)
        lam = want if t < 2 else np.random.default_rng(t).random(inst.K) * 2


def _offset_problem(kp, torch, inst):
    """The instance on the GPU with p, col and val placed one element past a
    16-byte boundary (4-byte aligned views): the uniform-row kernel stages
    every tile with 4-byte loads instead of 16-byte ones."""
    def dev(a, dt):
        a = np.ascontiguousarray(a, dt)
        buf = torch.empty(a.size + 1, dtype={np.float32: torch.float32, np.int32: torch.int32}[dt],
                          device="cuda")
        view = buf[1:]
        view.copy_(torch.from_numpy(a))
        assert view.data_ptr() % 16 != 0
        return view
    rowptr = torch.from_numpy(np.ascontiguousarray(inst.rowptr, np.int64)).cuda()
    return kp.Problem(dev(inst.p, np.float32), inst.B, inst.tree.parent, inst.tree.cap,
                      inst.tree.leaf_of_item, rowptr=rowptr, col=dev(inst.col, np.int32),
                      val=dev(inst.val, np.float32), N=inst.N, M=inst.M, K=inst.K)


LEAN_EXTRA = [
    ("c3-unaligned-N5000", lambda: kpgen.config_instance(3, N=5000), True),
    ("topq6-rank6-N4100", lambda: kpgen.make_instance(4100, 10, 9, seed=47, Q=6, csr_d=2, budget_frac=0.1),
     False),
]


@gpu
@pytest.mark.parametrize("name,mk,offset", LEAN_EXTRA, ids=[c[0] for c in LEAN_EXTRA])
def test_uniform_row_kernel_staging_and_rank(name, mk, offset):
    """The uniform-row kernel's other paths: 4-byte staging of full tiles
    when the arrays are not 16-byte aligned, and the consumption sums over
    all entries when more than 4 items can be selected (top-6).  Decisions,
    statistics and SCD updates (window trajectory) equal the oracle's."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    prob = _offset_problem(kp, torch, inst) if offset else kp.Problem.from_host(inst)
    ctx = kp.Context()
    lam = np.zeros(inst.K)
    for t in range(6):
        ev = kp.kp_eval_dual(prob, _lamd(torch, lam), want_x=True, ctx=ctx)
        ref = oracle.eval_dual(inst, lam)
        assert np.array_equal(ev["x"].cpu().numpy(), ref["x"])
        assert np.array_equal(ev["R"].cpu().numpy(), ref["R"])
        for key in ("g", "P"):
            assert abs(ev[key].item() - ref[key]) <= REL * max(1.0, abs(ref[key]))
        want = oracle.scd_sweep(inst, lam)
        got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
        assert np.array_equal(got, want), (t, np.flatnonzero(got != want))
        lam = want
    print("window searches", ctx.window_stats(), "listed", ctx.window_listed(), flush=True)


WINDOW_CASES = [
    ("c3-N20000", lambda: kpgen.config_instance(3, N=20000)),
    ("csr-d1-topq-N9000", lambda: kpgen.make_instance(9000, 12, 9, seed=43, Q=3, csr_d=1, budget_frac=0.1)),
    ("csr-d2-laminar-M16", lambda: kpgen.make_instance(6000, 16, 7, seed=44, csr_d=2, budget_frac=0.08,
                                                       tree=random_laminar(16, np.random.default_rng(5)))),
]


@gpu
@pytest.mark.parametrize("name,mk", WINDOW_CASES, ids=[c[0] for c in WINDOW_CASES])
def test_scd_window_trajectory(name, mk):
    """SCD iterations whose threshold search starts with a window around the
    previous multiplier (after the first sweep on a context): every update
    equals the oracle's at the same lambda, with the window on and off,
    including after a jump that puts the threshold outside the window."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    prob = kp.Problem.from_host(inst)
    win = kp.Context()
    full = kp.Context()
    full.set_window(False)
    lam = np.zeros(inst.K)
    for t in range(14):
        want = oracle.scd_sweep(inst, lam)
        for ctx in (win, full):
            got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
            assert np.array_equal(got, want), (t, np.flatnonzero(got != want), got, want)
        lam = want
        if t == 9:   # jump: the next windows miss
            lam = lam * np.where(np.arange(inst.K) % 2 == 0, 1.5, 0.5)
    tried, above, below, emitted = win.window_stats()
    print("window searches", tried, "above", above, "below", below, "emitted", emitted, flush=True)
    assert tried > 0 and tried - above - below > 0
    assert full.window_stats() == (0, 0, 0, 0)


def _alg5_instance(N, K, Q, seed):
    """Alg.5's setting (Sec. 5.1): M = K, item j consumes only knapsack j
    (diagonal b, every entry nonzero), one top-Q cap."""
    from util import make
    rng = np.random.default_rng(seed)
    p = rng.integers(1, 1 << 24, (N, K)) / float(1 << 24)
    b = np.zeros((N, K, K))
    for k in range(K):
        b[:, k, k] = rng.integers(1, 1 << 24, N) / float(1 << 24)
    B = 0.15 * b.sum(axis=(0, 1))
    return make(p, b, B, kpgen.tree_topq(K, Q), name="alg5")


@gpu
@pytest.mark.parametrize("K,Q", [(12, 3), (7, 2)])
def test_alg5_setting_scd_trajectory(K, Q):
    """Alg.5's special case on the GPU: stored per-item CSR with one entry per
    row takes the uniform-row kernel (one moving item per knapsack: the
    threshold-element path), dense storage the general kernel; both follow
    the oracle's SCD trajectory bit for bit, window on and off.  The oracle's
    general Map equals its Alg.5 Map on this instance (checked on a sample of
    users at every iterate)."""
    kp, torch = _kp()
    print("case alg5 K", K, "Q", Q, flush=True)
    inst = _alg5_instance(4097, K, Q, seed=50 + K)
    csr = inst.to_csr()
    assert np.all(np.diff(csr.rowptr) == 1)
    pc, pd = kp.Problem.from_host(csr), kp.Problem.from_host(inst)
    ctxs = [kp.Context(), kp.Context(), kp.Context()]
    ctxs[1].set_window(False)
    lam = np.zeros(K)
    for t in range(8):
        want = oracle.scd_sweep(inst, lam)
        kk, uu, v1, v2 = oracle.scd_map(inst, lam)
        for i in range(0, inst.N, 257):
            k5, a5, b5 = oracle.alg5_map_user(inst, lam, i, Q)
            assert sorted(kk[uu == i].tolist()) == sorted(k5.tolist())
        for prob, ctx in ((pc, ctxs[0]), (pc, ctxs[1]), (pd, ctxs[2])):
            got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
            assert np.array_equal(got, want), (t, np.flatnonzero(got != want))
        lam = want
    print("window searches", ctxs[0].window_stats(), flush=True)


def _ulps(a, b):
    return abs(int(np.float64(a).view(np.int64)) - int(np.float64(b).view(np.int64)))


@gpu
@pytest.mark.parametrize("K,Q", [(10, 3), (7, 2), (6, 6)])
def test_alg5_map_trajectory(K, Q):
    """Alg.5's map on the GPU (kp_set_alg5, Sec. 5.1): its SCD updates equal
    the oracle's SCD with Alg.5's map bit for bit, window on and off, along a
    trajectory; cross-checked against the general map (the event walk's
    threshold-element path) from the same multipliers: every coordinate
    within a few ulp, zero where it is zero."""
    kp, torch = _kp()
    print("case alg5 map K", K, "Q", Q, flush=True)
    inst = _alg5_instance(6001, K, Q, seed=60 + K)
    prob = kp.Problem.from_host(inst.to_csr())
    assert prob.row_nnz == 1
    ctxs = [kp.Context(), kp.Context()]
    for c in ctxs:
        c.set_alg5(True)
    ctxs[1].set_window(False)
    general = kp.Context()
    lam = np.zeros(K)
    for t in range(8):
        want = oracle.scd_sweep_alg5(inst, lam, Q)
        for ctx in ctxs:
            got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
            assert np.array_equal(got, want), (t, np.flatnonzero(got != want))
        gen = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=general)["lam"].cpu().numpy()
        assert np.array_equal(gen, oracle.scd_sweep(inst, lam)), t
        assert np.array_equal(gen == 0, want == 0), t
        assert max(_ulps(x, y) for x, y in zip(gen, want)) <= 16, (t, gen, want)
        lam = want
    print("window searches", ctxs[0].window_stats(), flush=True)


@gpu
@pytest.mark.parametrize("c,N", [(1, 10_000), (2, 2049), (3, 3001), (4, 700)])
def test_device_generator_matches_host(c, N):
    """The device generator writes the host generator's bytes and budgets."""
    kp, torch = _kp()
    from kpgen import device as kgd
    print("config", c, "N", N, flush=True)
    arrs, B, tree, meta = kgd.device_instance(c, 0, N=N)
    host = kpgen.config_instance(c, N=N)
    assert np.array_equal(arrs["p"].cpu().numpy(), host.p)
    if host.b is not None:
        assert np.array_equal(arrs["b"].cpu().numpy(), host.b)
    else:
        for key in ("rowptr", "col", "val"):
            assert np.array_equal(arrs[key].cpu().numpy(), getattr(host, key)), key
    assert np.array_equal(np.asarray(B), host.B)


def _full_size_problem(kp, c):
    from kpgen import device as kgd
    arrs, B, tree, meta = kgd.device_instance(c, 0)
    prob = kp.Problem(arrs["p"], B, tree.parent, tree.cap, tree.leaf_of_item, b=arrs.get("b"),
                      rowptr=arrs.get("rowptr"), col=arrs.get("col"), val=arrs.get("val"),
                      row_nnz=meta["csr_d"] if meta["csr_d"] else None,
                      N=meta["N"], M=meta["M"], K=meta["K"])
    return arrs, B, tree, meta, prob


@gpu
@pytest.mark.parametrize("c", [3, 2, 4])
def test_full_size_scd_sampled_parity(c):
    """At the benchmark's full size and launch configuration: decisions of
    sampled users equal the oracle's, g - P = lambda.(B - R), and every SCD
    threshold satisfies coordinate optimality (consumption just above it fits
    B_k, just below it does not), which holds at any size."""
    kp, torch = _kp()
    from kpgen import device as kgd
    print("config", c, "full size", flush=True)
    arrs, B, tree, meta, prob = _full_size_problem(kp, c)
    N, M, K = meta["N"], meta["M"], meta["K"]
    ctx = kp.Context()
    lam = torch.zeros(K, dtype=torch.float64, device="cuda")
    # as far as the benchmark's last timed iteration (windowed searches)
    for t in range(30):
        out = kp.kp_scd_sweep(prob, lam, ctx=ctx)
        lam_prev, lam = lam, out["lam"]
    print("window stats", ctx.window_stats(), flush=True)
    # sampled users at lambda^t
    ev = kp.kp_eval_dual(prob, lam_prev, want_x=True, ctx=ctx)
    users = np.sort(np.random.default_rng(7).choice(N, 4096, replace=False))
    sub = kgd.host_users(meta, B, tree, users)
    ref = oracle.eval_dual(sub, lam_prev.cpu().numpy())
    xg = ev["x"].view(N, M)[torch.from_numpy(users).cuda()].cpu().numpy().reshape(-1)
    assert np.array_equal(xg, ref["x"])
    R = ev["R"].cpu().numpy()
    lp = lam_prev.cpu().numpy()
    ident = ev["g"].item() - ev["P"].item() - float(np.dot(lp, np.asarray(B) - R))
    assert abs(ident) <= 1e-9 * (abs(ev["g"].item()) + abs(ev["P"].item()))
    # coordinate optimality of lambda^{t+1}
    v = lam.cpu().numpy()
    for k in range(K):
        lo = lp.copy()
        hi = lp.copy()
        if v[k] > 0:
            hi[k] = v[k] * (1 + 1e-9)
            lo[k] = v[k] * (1 - 1e-9)
            R_hi = kp.kp_eval_dual(prob, _lamd(torch, hi), ctx=ctx)["R"][k].item()
            R_lo = kp.kp_eval_dual(prob, _lamd(torch, lo), ctx=ctx)["R"][k].item()
            assert R_hi <= B[k] < R_lo, (k, R_hi, B[k], R_lo)
        else:
            hi[k] = 0.0
            assert kp.kp_eval_dual(prob, _lamd(torch, hi), ctx=ctx)["R"][k].item() <= B[k]


@gpu
def test_config4_autograd_as_specified():
    """Configuration 4 at full size (N = 1e7, M = 20, K = 50, 41 GB) as
    specified.  The autograd dual (DualFn) at 64 multipliers drawn
    U(0, 0.5)^K, which price every item out (x = 0, R = 0, g = lambda.B and
    the gradient is B exactly), and at 64 drawn U(0, 1/K)^K (reading A21): the
    gradient is B - R of the same evaluation, sampled users' decisions equal
    the oracle's (so do their consumptions), and the finite-difference
    convexity bracket (reading A15) holds for the GPU's own g along a random
    direction d at h = 1e-4:
        grad(lam - h d).d <= (g(lam + h d) - g(lam - h d)) / 2h <= grad(lam + h d).d
    (up to the FP64 rounding of g).  Then 200 dual-descent steps (Eq.14, step
    per reading A14) driven by the autograd gradient equal kp_dd_step's
    iterates bit for bit."""
    kp, torch = _kp()
    from kpgen import device as kgd
    print("config 4 full size", flush=True)
    arrs, B, tree, meta, prob = _full_size_problem(kp, 4)
    N, M, K = meta["N"], meta["M"], meta["K"]
    Bv = np.asarray(B, np.float64)
    users = np.sort(np.random.default_rng(8).choice(N, 2048, replace=False))
    sub = kgd.host_users(meta, B, tree, users)
    uidx = torch.from_numpy(users).cuda()
    h = 1e-4
    rng = np.random.default_rng(44)

    def dual(lam_np):
        lam = torch.tensor(lam_np, dtype=torch.float64, device="cuda", requires_grad=True)
        g = kp.DualFn.apply(lam, prob)
        g.backward()
        return g.item(), lam.grad.cpu().numpy()

    pts = [("U(0,0.5)", l) for l in kpgen.random_lambdas(4100, 64, K, 0.5)] + \
          [("U(0,1/K)", l) for l in kpgen.random_lambdas(4101, 64, K, 1.0 / K)]
    for t, (kind, lam_np) in enumerate(pts):
        g, grad = dual(lam_np)
        ev = kp.kp_eval_dual(prob, _lamd(torch, lam_np), want_x=True)
        R = ev["R"].cpu().numpy()
        assert np.array_equal(grad, Bv - R), (kind, t)
        xg = ev["x"].view(N, M)[uidx].cpu().numpy().reshape(-1)
        assert np.array_equal(xg, oracle.eval_dual(sub, lam_np)["x"]), (kind, t)
        if kind == "U(0,0.5)":
            assert not R.any() and np.array_equal(grad, Bv) and ev["P"].item() == 0.0, t
        d = rng.uniform(-1.0, 1.0, K)
        d[lam_np < 2 * h] = 0.0
        gp, grp = dual(lam_np + h * d)
        gm, grm = dual(lam_np - h * d)
        fd = (gp - gm) / (2 * h)
        slack = 1e-12 * (abs(gp) + abs(gm)) / h + 1e-12 * float(np.abs(grad * d).sum())
        assert float(grm @ d) - slack <= fd <= float(grp @ d) + slack, (kind, t, float(grm @ d), fd, float(grp @ d))
    # 200 DD steps: autograd-driven and kp_dd_step from the same start
    alpha = 1e-3 * 1e4 / N
    lam0 = kpgen.random_lambdas(4102, 1, K, 1.0 / K)[0]
    a = torch.tensor(lam0, dtype=torch.float64, device="cuda")
    b = a.clone()
    for step in range(200):
        l = a.clone().requires_grad_(True)
        kp.DualFn.apply(l, prob).backward()
        with torch.no_grad():
            a = torch.clamp(l - alpha * l.grad, min=0.0)
        kp.kp_dd_step(prob, alpha, b)
        if step % 50 == 49:
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), step
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


@gpu
def test_full_size_batched_matches_plain():
    """The batched workload at full size (256 instances, 37M users) in the
    benchmark's launch configuration (graph-replayed plan, cost-ordered block
    layout, later passes re-split): every iteration's multipliers equal the
    plain per-instance sweeps' bit for bit, and sampled users of three
    instances take the oracle's decisions at the last multipliers."""
    kp, torch = _kp()
    from kpgen import device as kgd
    print("batched workload full size", flush=True)
    data = kgd.device_batched(0, 256)
    probs = [kp.Problem(a["p"], B, tree.parent, tree.cap, tree.leaf_of_item, b=a["b"], N=m["N"], M=m["M"],
                        K=m["K"]) for a, B, tree, m in data]
    plan = kp.BatchedSCD(probs)
    ctxs = [kp.Context() for _ in probs]
    lams = [torch.zeros(pr.K, dtype=torch.float64, device="cuda") for pr in probs]
    for t in range(5):
        outs, _ = plan.step()
        torch.cuda.synchronize()
        for s, pr in enumerate(probs):
            lams[s] = kp.kp_scd_sweep(pr, lams[s], ctx=ctxs[s])["lam"]
        torch.cuda.synchronize()
        for s in range(len(probs)):
            assert torch.equal(outs[s], lams[s]), (t, s)
        print("iteration", t, "equal", flush=True)
    plan.close()
    rng = np.random.default_rng(11)
    for s in (0, 39, 128):
        a, B, tree, m = data[s]
        ev = kp.kp_eval_dual(probs[s], lams[s], want_x=True, ctx=ctxs[s])
        users = np.sort(rng.choice(m["N"], min(2048, m["N"]), replace=False))
        sub = kgd.host_users(m, B, tree, users)
        ref = oracle.eval_dual(sub, lams[s].cpu().numpy())
        xg = ev["x"].view(m["N"], m["M"])[torch.from_numpy(users).cuda()].cpu().numpy().reshape(-1)
        assert np.array_equal(xg, ref["x"]), s


PRESOLVE_CASES = [
    ("c3-N20000-n2000", lambda: kpgen.config_instance(3, N=20000), 2000),
    ("c1-dense-n1000", lambda: kpgen.config_instance(1), 1000),
    ("csr-d1-M10K10-n3000", lambda: kpgen.make_instance(30000, 10, 10, seed=78, Q=3, csr_d=1,
                                                        budget_frac=0.1), 3000),
]


@gpu
@pytest.mark.parametrize("name,mk,n", PRESOLVE_CASES, ids=[c[0] for c in PRESOLVE_CASES])
def test_presolve_parity(name, mk, n):
    """Pre-solving by sampling (Sec. 5.3) on the device: the gathered
    sub-instance, the scaled budgets and every SCD sweep equal the oracle's,
    so the pre-solved multipliers and the sweep count match exactly; a
    solve started from them reaches the gap in fewer iterations."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    prob = kp.Problem.from_host(inst)
    users = kpgen.sample_users(21, inst.N, n)
    lam0 = np.ones(inst.K)
    want, it_want = oracle.presolve(inst, users, max_iter=30, lam0=lam0)
    lam = _lamd(torch, lam0)
    lam, it = kp.kp_presolve(prob, users, lam, max_iter=30)
    assert it == it_want
    assert np.array_equal(lam.cpu().numpy(), want)
    _, h0 = kp.solve(prob, "scd", lam0=lam0, tol=1e-3, max_iter=40)
    _, h1 = kp.solve(prob, "scd", lam0=lam0, tol=1e-3, max_iter=40, presolve_users=users)
    print("iterations without / with pre-solve", len(h0), len(h1), flush=True)
    assert len(h1) <= len(h0)


@gpu
def test_presolve_rejects_bad_samples():
    kp, torch = _kp()
    inst = kpgen.config_instance(1)
    prob = kp.Problem.from_host(inst)
    lam = _lamd(torch, np.zeros(inst.K))
    for bad in ([0, 0, 1], [-1, 2], [inst.N], []):
        with pytest.raises(kp.KPError):
            kp.kp_presolve(prob, np.asarray(bad, np.int64), lam)


@gpu
def test_batched_plan_window_trajectory():
    """Batched plans start each iteration's threshold search with a window
    around the previous multiplier (per knapsack, from its last step): every
    instance still follows the oracle's SCD trajectory bit for bit, with the
    window on and off (the pass counts are reported)."""
    kp, torch = _kp()
    insts = [kpgen.config_instance(3, N=4000), kpgen.config_instance(3, run=1, N=2500),
             kpgen.make_instance(3000, 12, 9, seed=45, Q=3, csr_d=1, budget_frac=0.1),
             kpgen.make_instance(2000, 8, 3, seed=46, Q=2, budget_frac=0.1),
             kpgen.config_instance(1)]
    probs = [kp.Problem.from_host(i) for i in insts]
    passes = {}
    for window in (True, False):
        ctx = kp.Context()
        ctx.set_window(window)
        ctx.set_timing(True)
        plan = kp.BatchedSCD(probs, ctx=ctx)
        lams = [np.zeros(i.K) for i in insts]
        for t in range(12):
            outs, _ = plan.step()
            torch.cuda.synchronize()
            for s, inst in enumerate(insts):
                want = oracle.scd_sweep(inst, lams[s])
                assert np.array_equal(outs[s].cpu().numpy(), want), (window, t, s)
                lams[s] = want
        passes[window] = ctx.timing()[1]
        plan.close()
    print("passes with / without the window", passes[True], passes[False], flush=True)


@gpu
@pytest.mark.parametrize("name,mk", [
    ("c2-dense-N3000", lambda: kpgen.config_instance(2, N=3000)),
    ("c5-inst-dense", lambda: kpgen.batched_instances(run=0, n=40, max_N=6000)[39]),
    ("c4-dense-K50-N2000", lambda: kpgen.config_instance(4, N=2000)),
], ids=["c2-dense-N3000", "c5-inst-dense", "c4-dense-K50-N2000"])
def test_scd_alternating_trajectory(name, mk):
    """Dense instances whose synchronous iterations alternate between two
    multiplier vectors: searches that start with a window around the
    multiplier of two iterations back (and the general kernel's window pass)
    keep every update equal to the oracle's, window on and off.  With K = 50
    the histogram bins limit the general kernel's tile (4 users of M = 20);
    its window passes run without them, on 8-user tiles."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    prob = kp.Problem.from_host(inst)
    win = kp.Context()
    full = kp.Context()
    full.set_window(False)
    lam = np.zeros(inst.K)
    for t in range(10):
        want = oracle.scd_sweep(inst, lam)
        for ctx in (win, full):
            got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
            assert np.array_equal(got, want), (t, np.flatnonzero(got != want), got, want)
        lam = want
    print("window searches", win.window_stats(), flush=True)


def _free_tree(M):
    """No local constraint: every item with a positive adjusted profit is taken."""
    return kpgen.Tree(np.zeros(0, np.int32), np.zeros(0, np.int32), np.full(M, -1, np.int32))


# (name, instance, iterations, the iteration after which lambda jumps,
# whether some pass must run the lane-per-user window pass, None: not
# checked): the first group converges (windows around lambda^t), the second
# alternates between two multiplier vectors (windows around lambda^{t-2}: the
# lane-per-user pass where the probe finds every sampled user's lines far
# below zero, as at c2's upper multipliers, else the general kernel)
DENSE_WINDOW_CASES = [
    ("c1-N10000", lambda: kpgen.config_instance(1, N=10000), 16, 12, True),
    ("M10-K2-hier-N8000", lambda: kpgen.make_instance(8000, 10, 2, seed=84, p_dist="exp1", budget_frac=0.05,
                                                      tree=kpgen.tree_hier_2_2_3(10)), 16, 12, True),
    ("M16-K2-laminar-N6000", lambda: kpgen.make_instance(6000, 16, 2, seed=85, budget_frac=0.08,
                                                         tree=random_laminar(16, np.random.default_rng(9))),
     16, 12, True),
    ("M5-K2-free-N5000", lambda: kpgen.make_instance(5000, 5, 2, seed=72, budget_frac=0.15, tree=_free_tree(5)),
     16, 12, True),
    ("M12-K2-top4-lognormal-N6001", lambda: kpgen.make_instance(6001, 12, 2, seed=77, Q=4, p_dist="lognormal",
                                                                budget_frac=0.1), 16, 12, True),
    ("M3-K2-top1-N9000", lambda: kpgen.make_instance(9000, 3, 2, seed=79, Q=1, budget_frac=0.2), 16, 12, True),
    ("M8-K1-top3-N37", lambda: kpgen.make_instance(37, 8, 1, seed=74, Q=3, budget_frac=0.2), 12, 8, None),
    ("c2-N6000", lambda: kpgen.config_instance(2, N=6000), 10, 6, True),
    ("M10-K6-hier-N4000", lambda: kpgen.make_instance(4000, 10, 6, seed=75, p_dist="exp1", budget_frac=0.08,
                                                      tree=kpgen.tree_hier_2_2_3(10)), 10, 6, None),
    ("M8-K2-top2-N5000", lambda: kpgen.make_instance(5000, 8, 2, seed=86, Q=2, budget_frac=0.1), 16, 12, None),
    ("M12-K10-top3-N4000", lambda: kpgen.make_instance(4000, 12, 10, seed=87, Q=3, budget_frac=0.08), 10, 6, None),
]


@gpu
@pytest.mark.parametrize("name,mk,iters,jump,lane_pass", DENSE_WINDOW_CASES, ids=[c[0] for c in DENSE_WINDOW_CASES])
def test_dense_window_pass_trajectory(name, mk, iters, jump, lane_pass):
    """The lane-per-user window pass of dense costs (M, K <= 16): windows
    around lambda^t decided per item by the distance to its rank neighbours
    and to zero, the rest walked exactly with the pairs dealt over the wave.
    Every update equals the oracle's, as do the general kernel's (kernel
    choice off) and the full search's, with a jump that puts the thresholds
    outside the windows; both window kernels try the same searches.
    Alternation windows (away from lambda^t) go to the lane-per-user pass
    only when a probe of the users finds (almost) every line far below
    zero."""
    kp, torch = _kp()
    print("case", name, flush=True)
    inst = mk()
    prob = kp.Problem.from_host(inst)
    lane = kp.Context()
    gen = kp.Context()
    gen.set_kernel_choice(False)
    full = kp.Context()
    full.set_window(False)
    lam = np.zeros(inst.K)
    kernels = []
    for t in range(iters):
        want = oracle.scd_sweep(inst, lam)
        for ctx in (lane, gen, full):
            got = kp.kp_scd_sweep(prob, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
            assert np.array_equal(got, want), (t, np.flatnonzero(got != want), got, want)
            if ctx is lane:
                kernels.append(ctx.launch_shape()[0])
        lam = want
        if t == jump:   # the next windows miss
            lam = lam * np.where(np.arange(inst.K) % 2 == 0, 1.5, 0.5)
    print("window searches lane", lane.window_stats(), "general", gen.window_stats(),
          "users walked", lane.window_listed(), "kernels", kernels, flush=True)
    if lane_pass is not None:
        assert (3 in kernels) == lane_pass
    assert lane.window_stats()[0] == gen.window_stats()[0] > 0


CATEGORICAL_CASES = [("csr-d2", 2), ("dense", 0)]


@gpu
@pytest.mark.parametrize("name,csr_d", CATEGORICAL_CASES, ids=[c[0] for c in CATEGORICAL_CASES])
def test_categorical_scd_trajectory(name, csr_d):
    """Categorical variables (Sec. 2): the library's copies of every item
    (paper_2002_00352_amd.categorical) give the oracle's counts x_ij,
    consumption and SCD trajectory (the oracle expands the instance with its
    own code)."""
    kp, torch = _kp()
    from paper_2002_00352_amd import categorical
    print("case categorical", name, flush=True)
    # root cap 5 over 6 items, a group of the first 3 with cap 3, item caps 1..3
    parent = np.array([-1, 0] + [1, 1, 1, 0, 0, 0], np.int32)
    cap = np.array([5, 3, 2, 1, 3, 2, 1, 3], np.int32)
    leaf = np.arange(2, 8, dtype=np.int32)
    tree = kpgen.Tree(parent, cap, leaf)
    inst = kpgen.make_instance(3001, 6, 5, seed=61, csr_d=csr_d, tree=tree, budget_frac=0.1)
    cp = categorical.expand(kp.Problem.from_host(inst))
    binst, ioc = oracle.categorical_binary(inst)
    assert np.array_equal(cp.item_of_copy, ioc) and cp.binary.M == binst.M == 12
    ctx = kp.Context()
    lam = np.zeros(inst.K)
    for t in range(6):
        ev = kp.kp_eval_dual(cp.binary, _lamd(torch, lam), want_x=True, ctx=ctx)
        ref = oracle.eval_dual(binst, lam)
        want_x = oracle.categorical_counts(ref["x"], inst.N, ioc, inst.M)
        assert np.array_equal(cp.counts(ev["x"]).cpu().numpy(), want_x)
        assert np.array_equal(ev["R"].cpu().numpy(), ref["R"])
        want = oracle.scd_sweep(binst, lam)
        got = kp.kp_scd_sweep(cp.binary, _lamd(torch, lam), ctx=ctx)["lam"].cpu().numpy()
        assert np.array_equal(got, want), (t, np.flatnonzero(got != want))
        lam = want
    assert want_x.max() >= 2   # some item is taken more than once


@gpu
@pytest.mark.parametrize("nbytes", [16, 16 * 7 + 5, 16 * (1 << 20) + 48, 64 << 20])
def test_stream_read_checksum(nbytes):
    """The streaming-read probe reads every whole 16-byte word once: its
    checksum equals the host's XOR of the same words (sizes below one load
    per thread, with a ragged tail past the unrolled loads, and 64 MB)."""
    kp, torch = _kp()
    print("case", nbytes, flush=True)
    rng = np.random.default_rng(nbytes)
    host = rng.integers(0, 256, nbytes, dtype=np.uint8)
    t = torch.from_numpy(host).cuda()
    got = int(kp.kp_stream_read(t).cpu().numpy().view(np.uint64)[0])
    n16 = nbytes // 16
    words = host[:n16 * 16].view("<u4").reshape(-1, 4)
    acc = np.bitwise_xor.reduce(words, axis=0).astype(np.uint64)
    want = int(((acc[0] ^ acc[2]) << np.uint64(32)) | (acc[1] ^ acc[3]))
    assert got == want
