"""Benchmark: time to relative residual 1e-4 of the greedy ALS + Galerkin
solver (plain FP64, Jacobi-PCG) on the 3D-grid workload, plus the mixed
precision solve, the HBM bandwidth of the factored operator application on
the cortex-shell workload, and the FP64 CPU oracle on a bounded sample.

One JSON line on stdout.  Usage:
    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_1808_05510_amd import connreg, synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
METRIC = "secs to rel. residual 1e-4 & op-apply HBM GB/s: plain FP64 vs mixed+learned-PC"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def op_apply_bytes(n_y, n_x, n_inj, r, s):
    """Algorithmic bytes of one factored operator application: read U, V, X,
    the Omega bits and the neighbour tables, write L_y U, L_y^2 U, L_x V,
    L_x^2 V and Omega o (U Z H)."""
    return (s * ((n_y + n_x) * r + n_x * n_inj + 2 * (n_y + n_x) * r + n_y * n_inj)
            + n_y * n_inj / 8 + 24 * (n_y + n_x))


# Inner ALS solve tolerances: plain FP64 solves its u- and v-systems to a
# relative residual of 1e-8; mixed precision to 1e-4, because the ALS stage
# only sketches the bases on which the Galerkin step (FP64) solves (Section 4,
# after Algorithm 1).  Measured on the 3-D grid workload: relres at rank 60 is
# 3.80e-3 with 1e-4 inner solves against 3.82e-3 with 1e-8.
FP64_RTOL = 1e-8
MIXED_RTOL = 1e-4


def op_traffic():
    """HBM bytes of one op_apply call from the committed counter summary, or
    None when the kernel sources changed since the counters were taken."""
    from paper_1808_05510_amd import traffic
    path = os.path.join(ROOT, "profiles", "op_apply_shells_r100_fp64_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except OSError:
        return None
    return t["traffic_bytes"] if t.get("sources_sha") == traffic.sources_hash() else None


def sig(x, n=4):
    """x rounded to n significant digits (compact JSON)."""
    if x is None or not np.isfinite(x) or x == 0:
        return x
    return float(f"{x:.{n}g}")


def w_rel_diff(a, b):
    """||W_a - W_b||_F / ||W_b||_F for two results W = U Z V^T (torch, FP64,
    through thin QR of the stacked factors; measurement only)."""
    def fro(F, G):
        rf = torch.linalg.qr(F, mode="r")[1]
        rg = torch.linalg.qr(G, mode="r")[1]
        return float(torch.linalg.norm(rf @ rg.T))
    Ua, Za, Va = (a[k].to(torch.float64) for k in ("U", "Z", "V"))
    Ub, Zb, Vb = (b[k].to(torch.float64) for k in ("U", "Z", "V"))
    d = fro(torch.cat([Ua @ Za, -(Ub @ Zb)], 1), torch.cat([Va, Vb], 1))
    return d / fro(Ub @ Zb, Vb)


def write_detail(path, detail):
    """Curves, per-problem arrays and every figure behind the summary line."""
    if not path:
        return
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    with open(path, "w") as f:
        json.dump(detail, f, indent=1, default=float)
    log(f"[bench] details written to {path}")


def compact_cpu(cpu):
    if cpu is None:
        return None
    keep = ("value", "unit", "cores", "kind", "sample")
    out = {k: cpu[k] for k in keep}
    out["value"] = sig(out["value"])
    return out


def summarize(mixed, learned, shells, batch, op, highrank=None):
    """Scalar figures of every leg for the one-line result (seconds, relres,
    W error against the FP64 GPU solve, bandwidths)."""
    s = {}
    if mixed:
        s["mixed"] = dict(s=sig(mixed["seconds"]), relres=sig(mixed["relres"]),
                          w_err_vs_fp64=sig(mixed.get("w_err_vs_fp64")),
                          fp64_same_rtol_s=sig(mixed["fp64_same_rtol"]["seconds"]))
    if learned:
        s["mixed_learned_pc"] = dict(
            s=sig(learned["learned"]["seconds"]), relres=sig(learned["learned"]["relres"]),
            w_err_vs_fp64=sig(learned["learned"].get("w_err_vs_fp64")),
            base_step_s=sig(learned["base"]["seconds"]),
            train_s=sig(learned["train_s"]), pairs=learned["pairs"],
            inner_iters={k: sig(v["mean_iters"], 3) for k, v in learned["inner_u_solves"].items()},
            inner_ms={k: sig(v["mean_ms"], 3) for k, v in learned["inner_u_solves"].items()})
    if shells:
        s["shells"] = {k: dict(s=sig(v["seconds"]), rank=v["rank"], relres=sig(v["relres"]))
                       for k, v in shells.items() if isinstance(v, dict) and "seconds" in v}
        if "w_err_mixed_vs_fp64" in shells:
            s["shells"]["w_err_mixed_vs_fp64"] = sig(shells["w_err_mixed_vs_fp64"])
    if highrank:
        s["highrank_2d"] = {k: dict(s=sig(v["seconds"]), rank=v["rank"], relres=sig(v["relres"]),
                                    at=v["seconds_at_rank"])
                            for k, v in highrank.items() if isinstance(v, dict) and "seconds" in v}
        if "w_err_mixed_vs_fp64" in highrank:
            s["highrank_2d"]["w_err_mixed_vs_fp64"] = sig(highrank["w_err_mixed_vs_fp64"])
    if batch:
        s["batch"] = dict(seq_s=sig(batch["sequential_s"]), batched_s=sig(batch["batched_s"]),
                          speedup=sig(batch["speedup"], 3))
        if batch.get("with_base_step"):
            bb = batch["with_base_step"]
            s["batch"]["base_step"] = dict(seq_s=sig(bb["sequential_s"]),
                                           batched_s=sig(bb["batched_s"]),
                                           speedup=sig(bb["speedup"], 3))
    if op:
        s["op_apply_GBps"] = {k: round(v["GBps_mean"]) for k, v in op.items() if "GBps_mean" in v}
        if "gram" in op:
            s["gram_bf16_TFLOPs"] = {k: round(v["TFLOPs"]) for k, v in op["gram"].items()}
    return s


def time_solves(prob, steps, warmup, opts):
    res = None
    for _ in range(warmup):
        res = prob.greedy_solve(**opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times = []
    for _ in range(steps):
        t1 = time.perf_counter()
        res = prob.greedy_solve(**opts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return total, times, res


def bench_op_apply(d, r, reps, warm, fp32):
    """Median time of cr_op_apply with a 512 MiB cache flush before each call,
    timed with events on the library's stream (torch's current stream)."""
    prob = connreg.Problem(d, "mixed" if fp32 else "fp64", "cuda:0")
    dt = torch.float32 if fp32 else torch.float64
    g = torch.Generator(device="cuda:0").manual_seed(1)
    U = torch.randn((r, prob.n_y), device="cuda:0", dtype=dt, generator=g).T
    V = torch.randn((r, prob.n_x), device="cuda:0", dtype=dt, generator=g).T
    Z = torch.randn((r, r), device="cuda:0", dtype=dt, generator=g).T
    flush = torch.empty(512 * 1024 * 1024 // 4, device="cuda:0", dtype=torch.float32)
    ts = []
    for k in range(warm + reps):
        flush.fill_(float(k))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        prob.op_apply(U, Z, V, fp32=fp32)
        e1.record()
        e1.synchronize()
        if k >= warm:
            ts.append(e0.elapsed_time(e1) * 1e-3)
    s = 4 if fp32 else 8
    nbytes = op_apply_bytes(prob.n_y, prob.n_x, prob.n_inj, r, s)
    med = float(np.median(ts))
    mean = float(np.mean(ts))
    prob.close()
    return dict(r=r, dtype="f32" if fp32 else "f64", seconds=med, mean_seconds=mean,
                GBps_mean=nbytes / mean / 1e9,
                iqr=[float(np.percentile(ts, 25)), float(np.percentile(ts, 75))],
                bytes=nbytes, GBps=nbytes / med / 1e9, frac=nbytes / med / 1e9 / HBM_PEAK_GBS)


def bench_gram(d, r, reps, warm):
    """Batched masked Gram U^T diag(Omega_a) U, all a, in Khatri-Rao form on the
    BF16 matrix cores: r (r + 1) n_inj n_y flops per call."""
    prob = connreg.Problem(d, "fp64", "cuda:0")
    g = torch.Generator(device="cuda:0").manual_seed(2)
    U = torch.randn((r, prob.n_y), device="cuda:0", dtype=torch.float64, generator=g).T
    U = U / U.norm(dim=0, keepdim=True)
    ts = []
    for k in range(warm + reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        prob.masked_gram(U, "bf16")
        e1.record()
        e1.synchronize()
        if k >= warm:
            ts.append(e0.elapsed_time(e1) * 1e-3)
    flops = float(r) * (r + 1) * prob.n_inj * prob.n_y
    med = float(np.median(ts))
    prob.close()
    return dict(r=r, seconds=med, flops=flops, TFLOPs=flops / med / 1e12,
                frac=flops / med / 1e12 / BF16_PEAK_TFLOPS)


def bench_batch(count=16, max_rank=40, tau=1e-4, prec="mixed", precond="jacobi"):
    """The uneven 16-problem batch: each problem solved on its own (full
    device), then all at once through cr_greedy_solve_batch.  precond "base"
    declares both grids boxes (spectral u-steps, SMW v-solves)."""
    specs = synth.config4_specs(0, count)
    t0 = time.perf_counter()
    datas = [synth.box_problem(box_y=s.box_y, box_x=s.box_x,
                               offset=tuple((np.array(s.box_y) - np.array(s.box_x)) // 2),
                               n_inj=s.n_inj, lam=s.lam, max_rank=max_rank, seed=s.seed)
             for s in specs]
    gen = time.perf_counter() - t0
    streams = [torch.cuda.Stream() for _ in datas]
    probs = [connreg.Problem(d, prec, "cuda:0", stream=st) for d, st in zip(datas, streams)]
    if precond != "jacobi":
        for d, p in zip(datas, probs):
            p.set_box(d["box_y"])
            p.set_box(d["box_x"], which="source")
            p.set_precond(precond)
    opts = dict(max_rank=max_rank, tau_res=tau, seed=0,
                pcg_rtol=MIXED_RTOL if prec == "mixed" else FP64_RTOL)
    # PCG grid shapes from the tuning table (one autotune per size bucket)
    t0 = time.perf_counter()
    table = connreg.TuningTable()
    shapes = [table.apply(p) for p in probs]
    tune_s = time.perf_counter() - t0
    # warm-up (workspace allocation) then sequential timing
    connreg.greedy_solve_batch(probs[:1], [dict(opts, max_rank=2)])
    for p in probs:
        p.greedy_solve(**dict(opts, max_rank=2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [p.greedy_solve(**opts) for p in probs]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    bat = connreg.greedy_solve_batch(probs, [opts] * len(probs))
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    out = dict(problems=count, precision=prec, precond=precond, generation_s=gen,
               tuning=dict(buckets=len(table.table), seconds=tune_s,
                           vpt=[[e["vpt_u"], e["vpt_v"]] for e in shapes]),
               sequential_s=t_seq, batched_s=t_bat, speedup=t_seq / t_bat,
               sizes=[[p.n_y, p.n_x, p.n_inj] for p in probs],
               ranks_seq=[r["rank"] for r in seq], ranks_batch=[r["rank"] for r in bat],
               relres_seq=[r["stats"]["relres"] for r in seq],
               relres_batch=[r["stats"]["relres"] for r in bat])
    for p in probs:
        p.close()
    return out


def bench_learned(d2, lam, opts, steps, warmup, train_seeds=(100, 101), train_steps=300,
                  ref=None):
    """Mixed precision with the learned u-system preconditioner on the same
    workload: the network (spectral base step + 3-D conv refinement) is
    trained on u-systems dumped from FP64 greedy runs of other seeds (same
    grids and lambda); collection and training are timed separately.  The
    same mixed solve with the spectral base step alone is timed beside it.
    Both declare the source box too, so the v-systems take the SMW direct
    solve."""
    from paper_1808_05510_amd import lpc_train
    t0 = time.perf_counter()
    parts = []
    handles = []
    for s in train_seeds:
        dtr = synth.config2(lam=lam, seed=s)
        ptr = connreg.Problem(dtr, "fp64", "cuda:0")
        ptr.set_box(dtr["box_y"])
        parts.append(lpc_train.collect_pairs(ptr, max_rank=20, every=2, perturb=0.3, seed=s))
        handles.append(ptr)
    data = lpc_train.concat(parts)
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    pc = connreg.Pc(tuple(int(v) for v in d2["box_y"]), channels=8, seed=0)
    t0 = time.perf_counter()
    hist = lpc_train.train(pc, handles[-1], data, steps=train_steps, batch=8, lr=3e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    out = dict(pairs=len(data), collect_s=t_collect, train_s=t_train, train_steps=train_steps,
               loss_first=hist[0], loss_last=float(np.mean(hist[-20:])))
    # inner u-solves of the timed workload (a seed unseen in training) to
    # relres 1e-4, checked in FP64 by the solver's own residual
    pe = connreg.Problem(d2, "fp64", "cuda:0")
    pe.set_box(d2["box_y"])
    ev = lpc_train.collect_pairs(pe, max_rank=20, every=4, perturb=0.3, seed=0)
    inner = {}
    for kind in ("jacobi", "base", "learned"):
        rows = lpc_train.evaluate(pe, ev, pc if kind == "learned" else None, rtol=1e-4,
                                  precond=kind)
        inner[kind] = dict(systems=len(rows), mean_iters=float(np.mean([r["iters"] for r in rows])),
                           mean_ms=1e3 * float(np.mean([r["seconds"] for r in rows])),
                           max_relres=float(max(r["relres"] for r in rows)))
    out["inner_u_solves"] = inner
    pe.close()
    for kind in ("learned", "base"):
        pm = connreg.Problem(d2, "mixed", "cuda:0")
        pm.set_box(d2["box_y"])
        pm.set_box(d2["box_x"], which="source")
        if kind == "learned":
            pm.set_pc(pc)
        else:
            pm.set_precond("base")
        _, mtimes, mres = time_solves(pm, steps, warmup, opts)
        out[kind] = dict(seconds=float(np.mean(mtimes)), rank=mres["rank"],
                         relres=mres["stats"]["relres"], pcg_iters=mres["stats"]["pcg_iters"],
                         reached_tau=bool(mres["stats"]["relres"] <= opts["tau_res"]),
                         curve=[[h["rank"], h["relres"], h["seconds"]] for h in mres["history"]])
        if ref is not None:
            out[kind]["w_err_vs_fp64"] = w_rel_diff(mres, ref)
        pm.set_pc(None)
        pm.close()
    for h in handles:
        h.close()
    pc.close()
    return out


def bench_shells(steps=1):
    """Greedy solve on the cortex-shell workload, to relres 1e-4 or the rank
    cap of 100: plain FP64 (inner rtol 1e-8 and, for comparison at equal
    tolerance, 1e-4) and mixed (1e-4); one timed solve each after a short
    warm-up that allocates the workspace.  The mixed W error is taken
    against the plain FP64 solve."""
    d3 = synth.config3(seed=0)
    out = {}
    results = {}
    for key, prec, rtol in (("fp64", "fp64", FP64_RTOL), ("fp64_rtol1e-4", "fp64", MIXED_RTOL),
                            ("mixed", "mixed", MIXED_RTOL)):
        p = connreg.Problem(d3, prec, "cuda:0")
        p.greedy_solve(max_rank=2, tau_res=1e-4, seed=0, pcg_rtol=rtol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = p.greedy_solve(max_rank=int(d3["max_rank"]), tau_res=1e-4, seed=0, pcg_rtol=rtol)
        torch.cuda.synchronize()
        out[key] = dict(seconds=time.perf_counter() - t0, rank=res["rank"], pcg_rtol=rtol,
                        relres=res["stats"]["relres"], pcg_iters=res["stats"]["pcg_iters"],
                        reached_tau=bool(res["stats"]["relres"] <= 1e-4),
                        curve=[[h["rank"], h["relres"], h["seconds"]] for h in res["history"]])
        results[key] = res
        p.close()
    out["w_err_mixed_vs_fp64"] = w_rel_diff(results["mixed"], results["fp64"])
    return out


def bench_highrank(max_rank=250, kind="topview", precs=("fp64", "mixed"), verbose=0):
    """The paper's operating point: high rank on a 2-D cortical map (top-view
    size, n_inj 126), Galerkin tolerance tau(r)/2 from the paper's schedule
    for the target rank, no delta W stop (so the target rank is reached).
    Seconds to each of the paper's reported ranks (125, 200, 250, 400, 500)
    that the run passes."""
    d = synth.cortex_2d(kind, seed=0)
    gtol = 0.5 * synth.tau_schedule(max_rank)
    out = dict(kind=kind, n_y=int(d["Ly_rowptr"].size - 1), n_x=int(d["Lx_rowptr"].size - 1),
               n_inj=int(d["X"].shape[1]), lam=float(d["lam"]), max_rank=max_rank,
               galerkin_rtol=gtol)
    for prec in precs:
        p = connreg.Problem(d, prec, "cuda:0")
        rtol = MIXED_RTOL if prec == "mixed" else FP64_RTOL
        p.greedy_solve(max_rank=2, tau_dW=0.0, galerkin_rtol=gtol, seed=0, pcg_rtol=rtol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = p.greedy_solve(max_rank=max_rank, tau_dW=0.0, galerkin_rtol=gtol, seed=0,
                             pcg_rtol=rtol, verbose=verbose)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        hist = res["history"]
        at = {str(h["rank"]): round(h["seconds"], 3) for h in hist
              if h["rank"] in (125, 200, 250, 400, 500)}
        out[prec] = dict(seconds=secs, rank=res["rank"], relres=res["stats"]["relres"],
                         pcg_iters=res["stats"]["pcg_iters"],
                         galerkin_iters=res["stats"]["galerkin_iters"], seconds_at_rank=at,
                         J=hist[-1]["J"] if hist else None,
                         curve=[[h["rank"], h["relres"], h["seconds"], h["J"]] for h in hist])
        out.setdefault("_res", {})[prec] = res
        p.close()
    if "fp64" in precs and "mixed" in precs:
        out["w_err_mixed_vs_fp64"] = w_rel_diff(out["_res"]["mixed"], out["_res"]["fp64"])
    out.pop("_res", None)
    return out


def blas_threads():
    from threadpoolctl import threadpool_info
    n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
    return max(n) if n else 1


def cpu_baseline(d, lam, ranks_needed, sample_ranks):
    """FP64 oracle (NumPy/SciPy, Jacobi-CG inner solves to 1e-8, dense
    projected solve) on the first ``sample_ranks`` greedy steps of the same
    workload, on the host's BLAS threads, scaled to the ranks the GPU solve
    needed by the sample's mean seconds per rank (a lower estimate: a rank
    costs more as the basis grows and the residual shrinks); with
    sample_ranks >= ranks_needed the value is the measured time itself.
    Also: the first rank on one host thread, and the full 1-D toy solve
    (rank 20, dense inner solves)."""
    from threadpoolctl import threadpool_limits

    from oracle import greedy as ogreedy
    from oracle import operator as oop
    P = oop.problem_from_arrays(d, lam=lam)
    opts = dict(u_method="cg", v_method="cg", inner_rtol=1e-8, galerkin="dense", tau_res=1e-4)
    threads = blas_threads()
    t0 = time.perf_counter()
    res = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=sample_ranks, **opts))
    dt = time.perf_counter() - t0
    done = len(res.history)
    ends = np.array([h["seconds"] for h in res.history])
    per = np.diff(np.concatenate([[0.0], ends]))
    if done >= ranks_needed:
        value = float(ends[ranks_needed - 1])
        how = f"measured over all {ranks_needed} ranks"
    else:
        value = float(ends[-1] / done * ranks_needed)
        how = (f"first {done} ranks measured ({dt:.1f} s, {ends[-1] / done:.2f} s/rank), "
               f"scaled by {ranks_needed}/{done} (lower estimate: later ranks cost more)")
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=1, **opts))
        one_thread_rank = time.perf_counter() - t0
    d1 = synth.config1()
    P1 = oop.problem_from_arrays(d1)
    t0 = time.perf_counter()
    r1 = ogreedy.greedy_solve(P1, ogreedy.GreedyOptions(
        max_rank=int(d1["max_rank"]), tau_res=float(d1["tau_res"]), u_method="dense",
        v_method="dense", galerkin="dense"))
    toy_s = time.perf_counter() - t0
    return dict(value=value, unit="s", cores=threads, kind="oracle",
                sample=f"FP64 oracle greedy solve of the same 40^3/30^3 workload to rank "
                       f"{ranks_needed} on {threads} host threads: {how}",
                seconds_per_rank=[float(x) for x in per], one_thread_first_rank_s=one_thread_rank,
                toy_1d_full_solve_s=toy_s, toy_1d_rank=len(r1.history))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lam", type=float, default=1e3)
    ap.add_argument("--max-rank", type=int, default=60)
    ap.add_argument("--tau", type=float, default=1e-4)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-op", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-ranks", type=int, default=12,
                    help="oracle ranks timed for cpu_baseline (the rest extrapolated)")
    ap.add_argument("--op-reps", type=int, default=100)
    ap.add_argument("--op-warm", type=int, default=20)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--op-only", action="store_true", help="only the op_apply bandwidth part")
    ap.add_argument("--batch-only", action="store_true", help="only the 16-problem batch")
    ap.add_argument("--learned-only", action="store_true",
                    help="only the mixed solves with the learned preconditioner and the base step")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-shells", action="store_true")
    ap.add_argument("--no-highrank", action="store_true")
    ap.add_argument("--highrank-rank", type=int, default=250,
                    help="target rank of the 2-D high-rank leg (the paper goes to 1000)")
    ap.add_argument("--highrank-only", action="store_true")
    ap.add_argument("--detail", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file for curves and per-problem arrays ('' = none)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); the solver is a "
              "single-device library", file=sys.stderr)
        sys.exit(2)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    connreg.load()

    if a.learned_only:
        d2 = synth.config2(lam=a.lam, seed=0)
        mopts = dict(max_rank=a.max_rank, tau_res=a.tau, seed=0, pcg_rtol=MIXED_RTOL)
        lr = bench_learned(d2, a.lam, mopts, a.steps, a.warmup)
        log(f"[bench] mixed+learned: {lr['learned']['seconds']:.3f} s/solve (base step alone "
            f"{lr['base']['seconds']:.3f} s)")
        for kind in ("learned", "base"):
            e = lr[kind]
            log(f"[bench] {kind}: rank {e['rank']}, relres {e['relres']:.4e}, "
                f"pcg iterations {e['pcg_iters']}")
        log(f"[bench] pair collection {lr['collect_s']:.1f} s, training {lr['train_s']:.2f} s "
            f"({lr['train_steps']} steps, {lr['pairs']} pairs, loss {lr['loss_first']:.3e} -> "
            f"{lr['loss_last']:.3e})")
        for kind, e in lr["inner_u_solves"].items():
            log(f"[bench] inner u-solves {kind}: {e['mean_iters']:.1f} iterations, "
                f"{e['mean_ms']:.2f} ms")
        return
    if a.highrank_only:
        hr = bench_highrank(a.highrank_rank, verbose=1)
        write_detail(a.detail, {"highrank_2d": hr})
        for k in ("fp64", "mixed"):
            log(f"[bench] highrank {k}: {hr[k]['seconds']:.1f} s to rank {hr[k]['rank']} "
                f"(at ranks {hr[k]['seconds_at_rank']}), relres {hr[k]['relres']:.3e}, "
                f"galerkin iterations {hr[k]['galerkin_iters']}, pcg {hr[k]['pcg_iters']}")
        log(f"[bench] highrank mixed W error vs fp64 {hr['w_err_mixed_vs_fp64']:.2e}")
        return
    if a.batch_only:
        for pre in ("jacobi", "base"):
            b = bench_batch(precond=pre)
            log(json.dumps(b))
        return
    if a.op_only:
        d3 = synth.config3(seed=0)
        for fp32 in (False, True):
            o = bench_op_apply(d3, 100, a.op_reps, a.op_warm, fp32)
            log(f"[bench] op_apply {o['dtype']} r=100: {o['seconds']*1e6:.1f} us, {o['GBps']:.0f} GB/s")
        for r in (60, 100):
            o = bench_gram(d3, r, 10, 3)
            log(f"[bench] BF16 KR Gram r={r}: {o['seconds']*1e3:.3f} ms, {o['TFLOPs']:.0f} TFLOP/s "
                f"({100*o['frac']:.1f}% of BF16 dense peak)")
        return
    d2 = synth.config2(lam=a.lam, seed=0)
    opts = dict(max_rank=a.max_rank, tau_res=a.tau, seed=0, verbose=1 if a.verbose else 0,
                pcg_rtol=FP64_RTOL)
    mopts = dict(opts, pcg_rtol=MIXED_RTOL)
    op = None
    roof = None
    if not a.no_op:
        # first, in a fresh process: after minutes of large allocations by the
        # solves the same calls measure about 10% slower (allocator and page
        # state; the MFMA-bound Gram below runs at the same speed either way)
        log("[bench] op_apply bandwidth on the cortex-shell workload (n_y ~ 262k, n_x ~ 131k)")
        d3 = synth.config3(seed=0)
        op = {}
        for fp32 in (False, True):
            for r in (20, 60, 100):
                o = bench_op_apply(d3, r, a.op_reps, a.op_warm, fp32)
                op[f"{o['dtype']}_r{r}"] = o
                log(f"[bench] op_apply {o['dtype']} r={r}: {o['seconds']*1e6:.1f} us, "
                    f"{o['GBps']:.0f} GB/s ({100*o['frac']:.1f}% of HBM peak)")
        gram = {}
        for r in (60, 100):
            o = bench_gram(d3, r, 10, 3)
            gram[f"bf16_r{r}"] = o
            log(f"[bench] BF16 KR Gram r={r}: {o['seconds']*1e3:.3f} ms, {o['TFLOPs']:.0f} TFLOP/s")
        op["gram"] = gram
        o = op["f64_r100"]
        # achieved: algorithmic bytes over the mean event-timed call
        tr = op_traffic()
        roof = dict(bound="hbm", achieved=round(o["GBps_mean"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(o["GBps_mean"] / HBM_PEAK_GBS, 4),
                    traffic=None if tr is None else int(tr),
                    kernel="cr_op_apply (FP64, r=100, shells)")
        del d3

    log("[bench] FP64 solves on 40^3 / 30^3, n_inj 64")
    p64 = connreg.Problem(d2, "fp64", "cuda:0")
    total, times, res = time_solves(p64, a.steps, a.warmup, opts)
    hist = res["history"]
    ranks = res["rank"]
    reached = res["stats"]["relres"] <= a.tau
    log(f"[bench] fp64: {np.mean(times):.3f} s/solve, rank {ranks}, relres {res['stats']['relres']:.3e}")
    p64.close()

    mixed = None
    if not a.no_mixed:
        log("[bench] mixed-precision solves")
        pm = connreg.Problem(d2, "mixed", "cuda:0")
        mt, mtimes, mres = time_solves(pm, a.steps, a.warmup, mopts)
        mixed = dict(seconds=float(np.mean(mtimes)), rank=mres["rank"],
                     relres=mres["stats"]["relres"], pcg_iters=mres["stats"]["pcg_iters"],
                     galerkin_iters=mres["stats"]["galerkin_iters"], pcg_rtol=MIXED_RTOL,
                     w_err_vs_fp64=w_rel_diff(mres, res))
        log(f"[bench] mixed: {mixed['seconds']:.3f} s/solve, rank {mixed['rank']}")
        pm.close()
        # context: plain FP64 at the mixed runs' inner tolerance, which shows
        # how much of their gain is the tolerance rather than the precision
        pf = connreg.Problem(d2, "fp64", "cuda:0")
        _, ftimes, fres = time_solves(pf, a.steps, a.warmup, mopts)
        mixed["fp64_same_rtol"] = dict(seconds=float(np.mean(ftimes)), relres=fres["stats"]["relres"],
                                       pcg_iters=fres["stats"]["pcg_iters"], pcg_rtol=MIXED_RTOL)
        log(f"[bench] fp64 at inner rtol {MIXED_RTOL:g}: {mixed['fp64_same_rtol']['seconds']:.3f} s/solve")
        pf.close()

    learned = None
    if not a.no_learned:
        log("[bench] mixed precision + learned u-system preconditioner")
        learned = bench_learned(d2, a.lam, mopts, a.steps, a.warmup, ref=res)
        log(f"[bench] mixed+learned: {learned['learned']['seconds']:.3f} s/solve "
            f"(base step alone {learned['base']['seconds']:.3f} s; training "
            f"{learned['train_s']:.1f} s on {learned['pairs']} pairs)")

    shells = None
    if not a.no_shells:
        log("[bench] greedy solve on the cortex-shell workload (n_y 262,136, n_x 131,068)")
        shells = bench_shells()
        log(f"[bench] shells: fp64 {shells['fp64']['seconds']:.2f} s (rank {shells['fp64']['rank']}, "
            f"relres {shells['fp64']['relres']:.2e}); mixed {shells['mixed']['seconds']:.2f} s")

    highrank = None
    if not a.no_highrank:
        log(f"[bench] high-rank 2-D top-view map to rank {a.highrank_rank}")
        highrank = bench_highrank(a.highrank_rank)
        for k in ("fp64", "mixed"):
            log(f"[bench] highrank {k}: {highrank[k]['seconds']:.1f} s to rank {highrank[k]['rank']}"
                f" (at ranks {highrank[k]['seconds_at_rank']}), relres {highrank[k]['relres']:.3e}")

    batch = None
    if not a.no_batch:
        log("[bench] 16-problem batch (sequential vs one batched call)")
        batch = bench_batch()
        log(f"[bench] batch: sequential {batch['sequential_s']:.2f} s, batched "
            f"{batch['batched_s']:.2f} s, speedup {batch['speedup']:.2f}")
        bb = bench_batch(precond="base")
        batch["with_base_step"] = bb
        log(f"[bench] batch with spectral/SMW solves: sequential {bb['sequential_s']:.2f} s, "
            f"batched {bb['batched_s']:.2f} s, speedup {bb['speedup']:.2f}")

    cpu = None
    if not a.no_cpu:
        log("[bench] CPU oracle sample")
        cpu = cpu_baseline(d2, a.lam, ranks, a.cpu_ranks)

    secs = float(np.mean(times))
    curve = [[h["rank"], h["relres"], h["seconds"]] for h in hist]
    detail = {
        "fp64": dict(seconds=times, rank=ranks, relres=res["stats"]["relres"],
                     pcg_iters=res["stats"]["pcg_iters"],
                     galerkin_iters=res["stats"]["galerkin_iters"], relres_curve=curve),
        "mixed": mixed, "mixed_learned_pc": learned, "shells": shells, "op_apply": op,
        "batch": batch, "roofline": roof, "cpu_baseline": cpu, "highrank_2d": highrank,
    }
    write_detail(a.detail, detail)
    line = {
        "metric": METRIC,
        "value": round(secs, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(secs * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D grids 40^3 target / 30^3 source, n_inj 64, lambda 1e3, "
                               "rank cap 60, plain FP64 Jacobi-PCG (inner rtol 1e-8)",
                   "tau_res": a.tau, "seed": 0},
        "reached_tau": bool(reached),
        "rank": ranks,
        "relres": sig(res["stats"]["relres"]),
        "pcg_iters": res["stats"]["pcg_iters"],
        "roofline": roof,
        "cpu_baseline": compact_cpu(cpu),
        "summary": summarize(mixed, learned, shells, batch, op, highrank),
        "detail_file": a.detail,
    }
    print(json.dumps(line, separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
