#!/usr/bin/env python3
"""Benchmark of the per-user subproblem sweep on one MI355X.

A step is one synchronous coordinate-descent (SCD) iteration over the whole
instance: scoring, the local greedy, the consumption / dual reductions, every
user's breakpoint walk for every knapsack, the global threshold search and
the multiplier update, starting from lambda = 0 and feeding each step's
lambda to the next.  The timed steps follow the warm-up iterations (each of
which is timed on its own and reported: the cold start), and the full solve
from lambda = 0 to a 1e-3 duality gap is timed separately.  Inputs are
generated on the GPU and resident in HBM before the timed region.  Prints one
JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5, "c3cat": 3, "alg5": 0, "cdmodes": 0, "c1big": 1}
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2002_00352_amd/csrc/kp_kernels.hip", "paper_2002_00352_amd/csrc/kp_ell.hip",
                  "paper_2002_00352_amd/csrc/kp_ell_impl.h", "paper_2002_00352_amd/csrc/kp_device.h",
                  "paper_2002_00352_amd/csrc/kp_internal.h"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(workload, bytes_per_launch):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"sweep_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(cfg_id, seconds, lam, n_max=None):
    """The oracle's SCD sweep (the paper's candidates and map/reduce, as the
    oracle runs them) timed on a bounded prefix of the same workload
    (host-generated users) at the multipliers the GPU's timed steps reached,
    on all host threads and on one.  The prefix grows until one sweep on all
    threads takes about `seconds`; the one-thread figure uses a prefix 1/8 as
    long (n_max: the workload's users, default the configuration's)."""
    import numpy as np
    import kpgen
    import oracle
    threads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    lam = np.asarray(lam, np.float64)
    n_max = n_max or kpgen.CONFIGS[cfg_id]["N"]
    n, dt = 20_000, 0.0
    while True:
        inst = kpgen.config_instance(cfg_id, N=n)
        t0 = time.perf_counter()
        oracle.scd_sweep(inst, lam)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * seconds or n >= n_max:
            break
        n = int(min(n_max, n * min(16.0, max(1.5, seconds / max(dt, 1e-3)))))
    n1 = max(1000, n // 8)
    inst1 = kpgen.config_instance(cfg_id, N=n1)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.scd_sweep(inst1, lam)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    return {"value": n / dt, "unit": "user-solves/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} users of the same workload, one SCD sweep at the multipliers of the "
                      f"last timed GPU step ({dt:.1f} s on {threads} threads)",
            "single_thread": {"value": n1 / dt1, "cores": 1,
                              "sample": f"first {n1} users, same sweep ({dt1:.1f} s on 1 thread)"}}


def time_to_gap(tol=1e-3):
    """Wall time of the GPU drivers (sweeps + post-processing) on the small
    plain workload until the relative duality gap is <= tol: SCD, and DD with
    the paper's step 1e-3 (the best gap it reaches within its iteration cap);
    and the oracle's drivers on the same instance."""
    import numpy as np
    import torch
    import paper_2002_00352_amd as kp
    import kpgen
    import oracle
    inst = kpgen.config_instance(1)
    prob = kp.Problem.from_host(inst)
    out = {"workload": kpgen.CONFIGS[1]["name"], "tol": tol}
    for method, cap in (("scd", 100), ("dd", 400)):
        kp.solve(prob, method, tol=tol, max_iter=3, alpha=1e-3)          # warm the context
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, hist = kp.solve(prob, method, tol=tol, max_iter=cap, alpha=1e-3)
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - t0
        t0 = time.perf_counter()
        ref = oracle.solve(inst, method, tol=tol, max_iter=cap, alpha=1e-3)
        t_cpu = time.perf_counter() - t0
        out[method] = {"gpu_seconds": t_gpu, "iterations": len(hist), "gap_rel": hist[-1]["gap_rel"],
                       "reached": bool(hist[-1]["gap_rel"] <= tol), "oracle_seconds": t_cpu,
                       "oracle_iterations": len(ref), "oracle_gap_rel": ref[-1]["gap_rel"]}
    return out


def time_to_gap_full(prob, meta, tol=1e-3, max_iter=60, presolve_n=10_000):
    """Wall time of the SCD driver on the full instance from lambda^0 = 0 until
    the relative duality gap is <= tol (every pass of the cold iterations and
    the post-processing included; data resident), on a fresh context, without
    and with pre-solving by sampling (n users, Sec. 5.3; its sweeps
    included)."""
    import torch
    import paper_2002_00352_amd as kp
    import kpgen
    out = {"tol": tol, "lambda0": 0.0}
    for label, users in (("scd", None), ("scd_presolve", kpgen.sample_users(meta["seed"], meta["N"], presolve_n))):
        kp._default_ctx = None          # a fresh context: no window history
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, hist = kp.solve(prob, "scd", tol=tol, max_iter=max_iter, presolve_users=users)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[label] = {"seconds": dt, "iterations": len(hist), "gap_rel": hist[-1]["gap_rel"],
                      "reached": bool(hist[-1]["gap_rel"] <= tol)}
        if users is not None:
            out[label]["sample_users"] = int(len(users))
    return out


def config4_leg(prob, meta, steps=200):
    """The autograd workload as specified: the dual and its gradient (DualFn
    forward + backward) at 64 multipliers U(0, 0.5)^K and 64 U(0, 1/K)^K;
    then `steps` dual-descent steps (Eq.14, step 1e-3 scaled per reading A14)
    driven by the autograd gradient, timed against the same steps through
    kp_dd_step, with the best dual value along the path and the relative gap
    to the post-processed primal at the last iterate."""
    import numpy as np
    import torch
    import paper_2002_00352_amd as kp
    import kpgen
    N, K = meta["N"], meta["K"]
    out = {}
    for kind, scale, seed in (("U(0,0.5)", 0.5, 4100), ("U(0,1/K)", 1.0 / K, 4101)):
        pts = kpgen.random_lambdas(seed, 64, K, scale)
        lam = torch.tensor(pts[0], dtype=torch.float64, device="cuda", requires_grad=True)
        kp.DualFn.apply(lam, prob).backward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gs = []
        for l_np in pts:
            lam = torch.tensor(l_np, dtype=torch.float64, device="cuda", requires_grad=True)
            g = kp.DualFn.apply(lam, prob)
            g.backward()
            gs.append(g)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[kind] = {"points": len(pts), "ms_per_forward_backward": dt * 1e3 / len(pts),
                     "g_min": min(float(g.item()) for g in gs)}
    alpha = 1e-3 * 1e4 / N
    lam0 = kpgen.random_lambdas(4102, 1, K, 1.0 / K)[0]
    a = torch.tensor(lam0, dtype=torch.float64, device="cuda")
    best = (float("inf"), a.clone())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gvals = []
    for _ in range(steps):
        l = a.clone().requires_grad_(True)
        g = kp.DualFn.apply(l, prob)
        g.backward()
        gvals.append(g.detach())
        with torch.no_grad():
            a = torch.clamp(l - alpha * l.grad, min=0.0)
    torch.cuda.synchronize()
    t_ag = time.perf_counter() - t0
    b = torch.tensor(lam0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        kp.kp_dd_step(prob, alpha, b)
    torch.cuda.synchronize()
    t_dd = time.perf_counter() - t0
    g_best = min(float(x.item()) for x in gvals)
    fx = kp.kp_primal_fixup(prob, a)
    P_hat = float(fx["P"].item())
    out["dd_steps"] = {"steps": steps, "alpha": alpha, "autograd_ms_per_step": t_ag * 1e3 / steps,
                       "kp_dd_step_ms_per_step": t_dd * 1e3 / steps, "autograd_over_plain": t_ag / t_dd,
                       "same_iterates": bool(torch.equal(a, b)), "best_dual": g_best,
                       "primal_fixed_up_last": P_hat,
                       "gap_rel_best": (g_best - P_hat) / abs(P_hat) if P_hat else None}
    return out


def stream_ceiling(tensors, reps=3):
    """Measured streaming-read rate (GB/s) of the probe kernel over the given
    device arrays (HIP events on the current stream, the probe's own)."""
    import torch
    import paper_2002_00352_amd as kp
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    nbytes = sum(t.numel() * t.element_size() for t in tensors)
    for t in tensors:
        kp.kp_stream_read(t, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        for t in tensors:
            kp.kp_stream_read(t, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"kernel": "k_stream_read", "bytes": nbytes, "ms": ms, "GBs": nbytes / (ms * 1e-3) / 1e9}


def copy_probe(nbytes):
    """A plain device copy of known size (the scale reference for the HBM
    byte counters)."""
    import torch
    torch.cuda.set_device(0)
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "calls": 3}))


def _csv_rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def summarize_trace(trace_dir, bench_log, kernel_subs):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run of bench.py:
    the per-kernel statistics and the average duration of the timed sweep
    passes (the last `launches` dispatches of each kernel of a pass;
    kernel_subs: "|"-separated name fragments of the kernels of one pass; a
    fragment "a/b" takes the dispatches of either kernel (passes that run
    one or the other); a trailing "#n" sets the number of dispatches taken,
    e.g. every dispatch of the timed iterations of a graph-captured batched
    plan)."""
    rec = next(json.loads(l) for l in open(bench_log) if l.startswith("{"))
    stats = _csv_rows(os.path.join(trace_dir, "run_kernel_stats.csv"))
    trace = _csv_rows(os.path.join(trace_dir, "run_kernel_trace.csv"))
    # the batched line times whole iterations: its timed passes are the last
    # steps * passes_per_step dispatches of the batched kernel
    batched = rec["roofline"]["kernel"].startswith("k_sweep_batched")
    n = round(rec["steps"] * rec["passes_per_step"]) if batched else rec["roofline"]["launches"]
    if "#" in kernel_subs:
        kernel_subs, cnt = kernel_subs.rsplit("#", 1)
        n = int(cnt)
    subs = kernel_subs.split("|")
    # the timed passes end where the streaming ceiling's first read starts
    # (the benchmark measures it right after them)
    marks = [int(r["Start_Timestamp"]) for r in trace if "k_stream_read" in r["Kernel_Name"]]
    end = min(marks) if marks else None
    per = []
    for sub in subs:
        disp = sorted((r for r in trace if any(x in r["Kernel_Name"] for x in sub.split("/"))
                       and (end is None or int(r["Start_Timestamp"]) < end)),
                      key=lambda r: int(r["Start_Timestamp"]))
        per.append([(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6 for r in disp[-n:]])
    durs = [sum(x) for x in zip(*per)]
    avg = sum(durs) / len(durs)
    out = [f"| kernel | calls | avg ms | total ms | % |", "|---|---|---|---|---|"]
    for r in stats[:12]:
        out.append(f"| `{r['Name'][:60]}` | {r['Calls']} | {float(r['AverageNs']) * 1e-6:.3f} | "
                   f"{float(r['TotalDurationNs']) * 1e-6:.1f} | {float(r['Percentage']):.2f} |")
    out.append("")
    if batched:
        it_ms = sum(durs) / rec["steps"]
        out.append(f"Timed iterations (the last {n} dispatches of " + " + ".join(f"`{x}`" for x in subs) +
                   f", {rec['steps']} iterations): {it_ms:.3f} ms of sweep kernels per iteration; passes "
                   f"{min(durs):.3f} to {max(durs):.3f} ms.")
        out.append(f"bench.py's own HIP-event time per iteration (every pass and the search kernels): "
                   f"{rec['roofline']['avg_launch_ms']:.3f} ms; "
                   f"{rec['roofline']['algo_bytes_per_launch'] / 1e9:.2f} GB algorithmic bytes per iteration "
                   f"-> {rec['roofline']['algo_bytes_per_launch'] / (it_ms * 1e-3) / 1e9:.1f} GB/s from the trace.")
    else:
        out.append(f"Timed sweep passes (the last {n} dispatches of " + " + ".join(f"`{x}`" for x in subs) +
                   " before the streaming-ceiling probe" +
                   f"): average {avg:.3f} ms per pass (kernels only), min {min(durs):.3f}, max {max(durs):.3f}; "
                   + ", ".join(f"`{x}` {sum(p) / len(p):.3f} ms" for x, p in zip(subs, per)) + ".")
        out.append(f"bench.py's own HIP-event average per pass (both launches and the list reset "
                   f"between the events): {rec['roofline']['avg_launch_ms']:.3f} ms; "
                   f"{rec['roofline']['algo_bytes_per_launch'] / 1e9:.2f} GB algorithmic bytes per pass "
                   f"-> {rec['roofline']['algo_bytes_per_launch'] / (avg * 1e-3) / 1e9:.1f} GB/s from the trace.")
    out.append(f"bench line: value {rec['value']:.4g} {rec['unit']}, ms_per_step {rec['ms_per_step']:.2f}, "
               f"passes_per_step {rec['passes_per_step']}.")
    print("\n".join(out))


def summarize_pmc(fetch_dir, write_dir, cfetch_dir, cwrite_dir, kernel_subs, launches, workload,
                  copy_bytes):
    """HBM bytes per sweep pass from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch) of the pass's kernels ("|"-separated name fragments), each
    scaled by what the same counter reads for a plain copy of known size;
    written with the hash of the kernel sources they were taken on."""
    def per_dispatch(d, counter, sub):
        allrows = _csv_rows(os.path.join(d, "run_counter_collection.csv"))
        # the timed passes end where the streaming ceiling's first read starts
        marks = [int(r["Dispatch_Id"]) for r in allrows if "k_stream_read" in r["Kernel_Name"]]
        end = min(marks) if (marks and sub) else None
        rows = [r for r in allrows if sub in r["Kernel_Name"] and r["Counter_Name"] == counter
                and (end is None or int(r["Dispatch_Id"]) < end)]
        vals = {}
        for r in rows:
            vals[r["Dispatch_Id"]] = vals.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        return [vals[k] for k in sorted(vals, key=int)]
    subs = kernel_subs.split("|")
    f = [sum(x) for x in zip(*[per_dispatch(fetch_dir, "FETCH_SIZE", s)[-launches:] for s in subs])]
    w = [sum(x) for x in zip(*[per_dispatch(write_dir, "WRITE_SIZE", s)[-launches:] for s in subs])]
    cf_k = max(per_dispatch(cfetch_dir, "FETCH_SIZE", ""))    # the copy dispatches (KiB)
    cw_k = max(per_dispatch(cwrite_dir, "WRITE_SIZE", ""))
    sf = copy_bytes / (cf_k * 1024.0)
    sw = copy_bytes / (cw_k * 1024.0)
    fb = sum(f) / len(f) * 1024.0 * sf
    wb = sum(w) / len(w) * 1024.0 * sw
    rec = {"workload": workload, "kernels": subs, "kernel_hash": kernel_hash(),
           "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
           "hbm_bytes_per_launch": fb + wb, "fetch_scale": sf, "write_scale": sw,
           "launches_averaged": len(f), "copy_probe_bytes": copy_bytes,
           "copy_fetch_kib": cf_k, "copy_write_kib": cw_k}
    print(json.dumps(rec, indent=1))


def bench_batched(args):
    """The batched ragged workload (256 instances, device-generated): SCD
    iterations of the whole batch through one persistent launch per pass with
    the first pass of each iteration replayed from a HIP graph, and the same
    iterations as 256 sequential plain sweeps for comparison."""
    import numpy as np
    import torch
    import paper_2002_00352_amd as kp
    from kpgen import device as kgd

    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    data = kgd.device_batched(0, 256)
    probs = [kp.Problem(a["p"], B, tree.parent, tree.cap, tree.leaf_of_item, b=a["b"],
                        N=m["N"], M=m["M"], K=m["K"]) for a, B, tree, m in data]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    users = sum(m["N"] for _, _, _, m in data)
    # the plan's LDS budget and block split, tuned on this batch (whole
    # iterations from lambda = 0 per candidate)
    from paper_2002_00352_amd import autotune
    t_tune = time.perf_counter()
    choice, table = autotune.tune_batched(probs, steps=2, warmup=1)
    t_tune = time.perf_counter() - t_tune
    tctx = kp.Context()
    tctx.set_batched_tuning(*choice)
    bs = kp.BatchedSCD(probs, ctx=tctx)
    for _ in range(args.warmup):
        bs.step()
    torch.cuda.synchronize()
    ctx = bs.ctx
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bs.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_k, iters, bytes_k = ctx.timing()
    passes = ctx.batched_passes()
    ctx.set_timing(False)
    lam_batched = [t.cpu().numpy().copy() for t in bs.lam]
    # the same iterations as sequential plain sweeps (one call per instance)
    seq_steps = min(args.steps, 3)
    lams = [torch.zeros(pr.K, dtype=torch.float64, device="cuda") for pr in probs]
    outs = [torch.zeros(pr.K, dtype=torch.float64, device="cuda") for pr in probs]
    # one context per instance, as a caller running them one by one would
    # keep (each context carries its instance's window history)
    sctxs = [kp.Context() for _ in probs]
    for _ in range(args.warmup):
        for i, pr in enumerate(probs):
            kp.kp_scd_sweep(pr, lams[i], outs[i], ctx=sctxs[i])
        lams, outs = outs, lams
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(seq_steps):
        for i, pr in enumerate(probs):
            kp.kp_scd_sweep(pr, lams[i], outs[i], ctx=sctxs[i])
        lams, outs = outs, lams
    torch.cuda.synchronize()
    seq_dt = (time.perf_counter() - t0) / seq_steps
    per_iter_bytes = bytes_k / max(iters, 1)
    avg_iter_ms = ms_k / max(iters, 1)
    achieved = per_iter_bytes / (avg_iter_ms * 1e-3) / 1e9
    rec = {
        "metric": "user-subproblem solves/s per SCD sweep",
        "value": users * args.steps / dt,
        "unit": "user-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded counter-based generator, generated on the GPU)",
        "config": {"workload": "c5 batched ragged: 256 instances, N log-uniform [1e3,1e6), M 4..32, "
                               "K 1..16, Q 1..4, dense U(0,1)", "instances": len(probs), "users": users,
                   "graph": True},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_sweep_batched (whole iterations: every pass and the search kernels)",
                     "launches": iters, "avg_launch_ms": avg_iter_ms,
                     "algo_bytes_per_launch": per_iter_bytes,
                     "algo_bytes_rule": "every input byte of every instance once per iteration"},
        "passes_per_step": passes / args.steps,
        "tuning": {"choice": {"lds_bytes": choice[0], "block_mult": choice[1]},
                   "plan_shape": dict(zip(("blocks", "lds_bytes", "min_users_per_tile", "max_users_per_tile"),
                                          bs.shape())),
                   "tried": [{"lds_bytes": c[0], "block_mult": c[1], "ms_per_iteration": ms,
                              "blocks": sh[0]} for c, ms, sh in table],
                   "seconds": t_tune},
        "sequential_plain_ms_per_step": seq_dt * 1e3,
        "batched_speedup_vs_sequential": seq_dt / (dt / args.steps),
        "lambda_head": [float(v) for v in lam_batched[0][:4]],
        "gen_s": t_gen,
    }
    print(json.dumps(rec), flush=True)


def bench_alg5(args, N=100_000_000, M=10, Q=3):
    """Alg.5's setting (Sec. 5.1) at scale: N users, M = K items, item j
    consuming only knapsack j (per-item CSR, one entry per row), one top-Q
    cap, U(0,1) profits and costs, B_k = 0.1 D_k.  The same SCD iterations
    with Alg.5's map and with the general map (the event walk's
    threshold-element path), each on its own context from lambda = 0."""
    import numpy as np
    import torch
    import paper_2002_00352_amd as kp
    import kpgen
    from kpgen import device as kgd

    torch.cuda.set_device(0)
    N = args.users or N
    K = M
    seed = 7000
    L = kgd.lib()
    st = kgd._stream()
    t_gen = time.perf_counter()
    p = torch.empty(N * M, dtype=torch.float32, device="cuda")
    val = torch.empty(N * M, dtype=torch.float32, device="cuda")
    kgd._ok(L.kpgen_values(seed, kpgen.S_P, 0, N * M, None, p.data_ptr(), st))
    kgd._ok(L.kpgen_values(seed, kpgen.S_VAL, 0, N * M, None, val.data_ptr(), st))
    col = (torch.arange(N * M, device="cuda", dtype=torch.int64) % M).to(torch.int32)
    rowptr = torch.arange(N * M + 1, device="cuda", dtype=torch.int64)
    sums = torch.zeros(K, dtype=torch.int64, device="cuda")
    kgd._ok(L.kpgen_colsum_csr(col.data_ptr(), val.data_ptr(), N * M, K, sums.data_ptr(), st))
    B = kpgen.budgets(sums.cpu().numpy().astype(np.float64) * 2.0 ** -24, 0.1, 1)
    tree = kpgen.tree_topq(M, Q)
    prob = kp.Problem(p, B, tree.parent, tree.cap, tree.leaf_of_item, rowptr=rowptr, col=col, val=val,
                      N=N, M=M, K=K, row_nnz=1)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    res = {}
    lams = {}
    for label, on in (("alg5", True), ("general", False)):
        ctx = kp.Context()
        ctx.set_alg5(on)
        lam = torch.zeros(K, dtype=torch.float64, device="cuda")
        out = torch.zeros(K, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            kp.kp_scd_sweep(prob, lam, out, ctx=ctx)
            lam, out = out, lam
        torch.cuda.synchronize()
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            kp.kp_scd_sweep(prob, lam, out, ctx=ctx)
            lam, out = out, lam
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms_k, launches, bytes_k = ctx.timing()
        ctx.set_timing(False)
        res[label] = {"ms_per_step": dt * 1e3 / args.steps, "value": N * args.steps / dt,
                      "passes_per_step": launches / args.steps, "kernel_ms_per_pass": ms_k / max(launches, 1),
                      "achieved_GBs": bytes_k / max(launches, 1) / (ms_k / max(launches, 1) * 1e-3) / 1e9}
        lams[label] = lam.cpu().numpy()
        ctx.close()
    ulp = np.abs(lams["alg5"].view(np.int64) - lams["general"].view(np.int64))
    a = res["alg5"]
    rec = {
        "metric": "user-subproblem solves/s per SCD sweep",
        "value": a["value"], "unit": "user-solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": a["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded counter-based generator, generated on the GPU)",
        "config": {"workload": f"Alg.5 setting: N={N} M=K={M} diagonal per-item CSR, top-{Q}, U(0,1)",
                   "N": N, "M": M, "K": K, "Q": Q},
        "roofline": {"bound": "hbm", "achieved": a["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": a["achieved_GBs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_ell SCD passes with Alg.5's map", "avg_launch_ms": a["kernel_ms_per_pass"]},
        "alg5_map": a, "general_map": res["general"],
        "alg5_over_general_time": a["ms_per_step"] / res["general"]["ms_per_step"],
        "final_lambda_max_ulp_apart": int(ulp.max()), "gen_s": t_gen,
    }
    print(json.dumps(rec), flush=True)


def bench_cd_modes(args, tol=1e-3):
    """Iterations and time to a relative duality gap <= tol (or the best gap
    within the cap) of the coordinate-descent variants (Sec. 4.3.2: SCD,
    cyclic, block), SCD with Sec. 5.2's interpolated reduce, and DD with the
    paper's steps 1e-3 and 2e-3 (scaled per reading A14), from lambda = 0 on
    the small plain workload and reduced copies of the dense and hierarchical
    sparse ones.  The GPU iterates equal the oracle's bit for bit (tested), so
    the counts are the method's, not the hardware's."""
    import numpy as np
    import torch
    import paper_2002_00352_amd as kp
    import kpgen
    torch.cuda.set_device(0)
    out = []
    for cfg, N in ((1, None), (2, 200_000), (3, 1_000_000)):
        inst = kpgen.config_instance(cfg, N=N) if N else kpgen.config_instance(cfg)
        prob = kp.Problem.from_host(inst)
        K = inst.K
        runs = [("scd", {}), ("cyclic", {}), ("block", {"block": max(1, K // 2)}), ("interp", {}),
                ("dd", {"alpha": 1e-3 * 1e4 / inst.N}), ("dd", {"alpha": 2e-3 * 1e4 / inst.N})]
        for method, kw in runs:
            cap = 300 if method in ("cyclic", "block", "dd") else 100
            kp._default_ctx = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam, hist = kp.solve(prob, method, tol=tol, max_iter=cap, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            gaps = [h["gap_rel"] for h in hist]
            out.append({"workload": inst.name, "N": inst.N, "K": K, "method": method,
                        **{k: v for k, v in kw.items()}, "iterations": len(hist),
                        "reached": bool(gaps[-1] <= tol), "gap_rel": gaps[-1], "best_gap_rel": min(gaps),
                        "max_viol_last": hist[-1]["max_viol"], "seconds": dt})
            print(json.dumps(out[-1]), flush=True)
    print(json.dumps({"metric": "iterations to duality gap", "tol": tol, "runs": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dd-steps", type=int, default=10, help="DD sweeps timed after the SCD steps")
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--users", type=int, default=None, help="override N (testing only)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gap", action="store_true", help="skip the time-to-gap runs on the full instance")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="run a plain device copy of BYTES (counter calibration) and exit")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE_DIR", "BENCH_LOG", "KERNELS"),
                    help="print a markdown summary of a rocprofv3 kernel trace of bench.py and exit")
    ap.add_argument("--summarize-pmc", nargs=8,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR", "KERNELS",
                             "LAUNCHES", "WORKLOAD", "COPY_BYTES"),
                    help="print the HBM traffic record from rocprofv3 counter runs and exit")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_pmc:
        a = args.summarize_pmc
        summarize_pmc(a[0], a[1], a[2], a[3], a[4], int(a[5]), a[6], int(a[7]))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sweep shards by users; see the design notes). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "c5":
        bench_batched(args)
        return
    if args.workload == "alg5":
        bench_alg5(args)
        return
    if args.workload == "cdmodes":
        bench_cd_modes(args)
        return
    import numpy as np
    import torch
    import paper_2002_00352_amd as kp
    import kpgen
    from kpgen import device as kgd

    torch.cuda.set_device(0)
    cfg_id = WORKLOADS[args.workload]
    if args.workload == "c3cat" and args.users is None:
        args.users = 20_000_000   # the copies' index arrays of the expansion stay a few GB
    if args.workload == "c1big" and args.users is None:
        args.users = 10_000_000   # c1's recipe (dense, M = 10, K = 2, top-1) at c2's size: it converges
    t_gen = time.perf_counter()
    arrs, B, tree, meta = kgd.device_instance(cfg_id, 0, N=args.users)
    cap = tree.cap
    if args.workload == "c3cat":
        # categorical variables (Sec. 2): every item may be taken twice (the
        # per-item caps of the hierarchy raised to 2), run as binary copies
        cap = tree.cap.copy()
        cap[np.asarray(tree.leaf_of_item)] = 2
    prob = kp.Problem(arrs["p"], B, tree.parent, cap, tree.leaf_of_item, b=arrs.get("b"),
                      rowptr=arrs.get("rowptr"), col=arrs.get("col"), val=arrs.get("val"),
                      N=meta["N"], M=meta["M"], K=meta["K"],
                      row_nnz=meta["csr_d"] if meta["csr_d"] else None)
    if args.workload == "c1big":
        meta = dict(meta, name="c1 recipe at scale: plain SCD N=%d M=10 K=2 top-1 dense, U(0,1)" % meta["N"])
    if args.workload == "c3cat":
        from paper_2002_00352_amd import categorical
        prob = categorical.expand(prob).binary
        meta = dict(meta, M=prob.M, name="c3 categorical (item caps 2, %d binary copies per user) N=%d"
                    % (prob.M, meta["N"]))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    ctx = kp.default_context()
    K = meta["K"]
    lam = torch.zeros(K, dtype=torch.float64, device="cuda")
    out = torch.zeros(K, dtype=torch.float64, device="cuda")
    warm_ms = []
    for _ in range(args.warmup):
        t0 = time.perf_counter()
        kp.kp_scd_sweep(prob, lam, out, ctx=ctx)
        torch.cuda.synchronize()
        warm_ms.append((time.perf_counter() - t0) * 1e3)
        lam, out = out, lam
    torch.cuda.synchronize()
    ctx.set_timing(True)
    win0 = ctx.window_stats()
    listed0 = ctx.window_listed()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        kp.kp_scd_sweep(prob, lam, out, ctx=ctx)
        lam, out = out, lam
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_k, launches, bytes_k = ctx.timing()
    ctx.set_timing(False)
    win = [b - a for a, b in zip(win0, ctx.window_stats())]
    listed = ctx.window_listed() - listed0
    dt = t1 - t0
    N = meta["N"]
    value = N * args.steps / dt
    per_launch_bytes = bytes_k / max(launches, 1)
    avg_ms = ms_k / max(launches, 1)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    traffic = traffic_for(args.workload, per_launch_bytes)
    lean = bool(meta["csr_d"]) and meta["M"] <= 16
    # the ceiling streams the arrays the pass reads (the lean kernel never
    # reads rowptr)
    ceiling = stream_ceiling([t for t in (prob.p, prob.b, None if lean else prob.rowptr, prob.col, prob.val)
                              if t is not None])
    physical = traffic / (avg_ms * 1e-3) / 1e9 if traffic else None
    kernel_name = {1: "k_ell window pass (all users, then the listed ones)",
                   3: "k_dense window pass (lane per user)"}.get(ctx.launch_shape()[0], "k_sweep (scd)")
    rec = {
        "metric": "user-subproblem solves/s per SCD sweep",
        "value": value,
        "unit": "user-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded counter-based generator, generated on the GPU)",
        "config": {"workload": meta["name"], "N": N, "M": meta["M"], "K": meta["K"],
                   "b_format": "csr" if meta["csr_d"] else "dense", "seed": meta["seed"],
                   "lambda0": 0.0},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel_name, "launches": launches,
                     "avg_launch_ms": avg_ms, "algo_bytes_per_launch": per_launch_bytes,
                     "algo_bytes_rule": "every input byte of the ABI layout once per pass (p, and b dense, "
                                        "or CSR rowptr + col + val)",
                     "physical_GBs": physical,
                     "frac_physical": physical / HBM_PEAK_GBS if physical else None,
                     # frac: streaming the same arrays once takes this share of
                     # the pass's time; frac_physical: counted HBM bytes of the
                     # pass per second against the streaming rate
                     "ceiling": dict(ceiling, frac=ceiling["ms"] / avg_ms,
                                     frac_physical=physical / ceiling["GBs"] if physical else None)},
        "passes_per_step": launches / args.steps,
        "warmup_ms_per_step": warm_ms,
        "threshold_search": {"window_tried": win[0], "window_missed_above": win[1],
                             "window_missed_below": win[2], "window_events": win[3],
                             "knapsack_searches": K * args.steps,
                             "users_listed_per_sweep": listed / args.steps},
        "pct_hbm_peak": 100.0 * achieved / HBM_PEAK_GBS,
        "lambda_final_head": [float(v) for v in lam[:4].cpu().numpy()],
        "gen_s": t_gen,
    }
    lam_warm = lam.cpu().numpy().copy()
    # the DD sweep (Eq. 14) on the same instance: evaluation kernel + update
    lam_dd = lam.clone()
    kp.kp_dd_step(prob, 1e-12, lam_dd, ctx=ctx)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.dd_steps):
        kp.kp_dd_step(prob, 1e-12, lam_dd, ctx=ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_d, n_d, bytes_d = ctx.timing()
    ctx.set_timing(False)
    if n_d:
        dd_ms = ms_d / n_d
        dd_gbs = bytes_d / n_d / (dd_ms * 1e-3) / 1e9
        # frac counts the ABI's bytes (the rule above); read_GBs / frac_read
        # count the bytes the kernel reads (the lean kernel skips rowptr),
        # ceiling_frac: the streaming probe's time over the same arrays
        # against the sweep's
        rec["dd_sweep"] = {"steps": args.dd_steps, "ms_per_step": (t1 - t0) * 1e3 / args.dd_steps,
                           "user_solves_per_s": N * args.dd_steps / (t1 - t0),
                           "kernel_avg_ms": dd_ms, "achieved_GBs": dd_gbs,
                           "frac": dd_gbs / HBM_PEAK_GBS,
                           "read_bytes": ceiling["bytes"],
                           "read_GBs": ceiling["bytes"] / (dd_ms * 1e-3) / 1e9,
                           "frac_read": ceiling["bytes"] / (dd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "ceiling_frac": ceiling["ms"] / dd_ms}
    # the same DD steps through the autograd form (forward: evaluation kernel,
    # backward: the gradient kernel from the saved consumption)
    lam_ag = [lam.clone()]

    def ag_step():
        l = lam_ag[0].clone().requires_grad_(True)
        kp.DualFn.apply(l, prob).backward()
        with torch.no_grad():
            lam_ag[0] = torch.clamp(l - 1e-12 * l.grad, min=0.0)
    ag_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.dd_steps):
        ag_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if "dd_sweep" in rec:
        ag_ms = (t1 - t0) * 1e3 / args.dd_steps
        rec["dd_sweep"]["autograd_ms_per_step"] = ag_ms
        rec["dd_sweep"]["autograd_over_plain"] = ag_ms / rec["dd_sweep"]["ms_per_step"]
    if args.workload == "c3" and args.users is None and not args.no_gap:
        rec["time_to_gap_full"] = time_to_gap_full(prob, meta)
    if args.workload == "c4":
        rec["config4_autograd"] = config4_leg(prob, meta)
    del prob, arrs
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        if args.workload != "c3cat":
            rec["cpu_baseline"] = cpu_baseline(cfg_id, args.cpu_seconds, lam_warm, n_max=N)
        rec["time_to_gap"] = time_to_gap()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
