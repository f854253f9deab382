"""bench.py's contract that holds without a GPU: more than one GPU is refused
with a message, and the one-line result's summary of every leg stays compact
(the full line must fit in about 2 KB for a reader that keeps only the tail
of the output)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_summary_of_all_legs_is_compact():
    sys.path.insert(0, ROOT)
    import bench
    mixed = dict(seconds=1.4549, relres=0.0038113, w_err_vs_fp64=3.125e-4,
                 fp64_same_rtol=dict(seconds=1.2634))
    inner = {k: dict(mean_iters=2.4, mean_ms=0.571) for k in ("jacobi", "base", "learned")}
    learned = dict(learned=dict(seconds=0.2163, relres=0.003783, w_err_vs_fp64=3.2e-4),
                   base=dict(seconds=0.1806), train_s=0.945, pairs=40, inner_u_solves=inner)
    leg = dict(seconds=9.59, rank=100, relres=0.005899)
    shells = {"fp64": leg, "fp64_rtol1e-4": leg, "mixed": leg, "w_err_mixed_vs_fp64": 1.1e-3}
    hr = dict(seconds=18.85, rank=250, relres=5.8e-4,
              seconds_at_rank={"125": 7.498, "200": 13.151, "250": 18.851})
    highrank = {"fp64": hr, "mixed": hr, "w_err_mixed_vs_fp64": 2.3e-4}
    bb = dict(sequential_s=2.263, batched_s=1.17, speedup=1.934)
    batch = dict(sequential_s=15.06, batched_s=14.91, speedup=1.01, with_base_step=bb)
    op = {f"f{s}_r{r}": dict(GBps_mean=1771.0) for s in (32, 64) for r in (20, 60, 100)}
    op["gram"] = {"bf16_r60": dict(TFLOPs=299.0), "bf16_r100": dict(TFLOPs=361.0)}
    s = bench.summarize(mixed, learned, shells, batch, op, highrank)
    assert set(s) == {"mixed", "mixed_learned_pc", "shells", "highrank_2d", "batch",
                      "op_apply_GBps", "gram_bf16_TFLOPs"}
    text = json.dumps(s, separators=(",", ":"))
    # the rest of the line (metric, value, config, roofline, cpu_baseline)
    # takes about 970 bytes; the whole line about 2,010
    assert len(text) <= 1060, len(text)
