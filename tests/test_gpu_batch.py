"""Batched greedy solves (several problems at once, one handle and stream
each, persistent kernels sharing the device) and the PCG autotuner.

Each batched result must match the FP64 oracle in lockstep (relative W
error <= 1e-6), and a batch too large to run all at once (the scheduler then
runs fewer problems concurrently) must give the same answers as the same
problems solved one at a time (1e-8 at tight tolerances: only the grid
shapes, hence the rounding order, differ)."""
import numpy as np
import pytest
import torch

from oracle import greedy as ogreedy
from oracle import metrics as omet
from oracle import operator as oop
from paper_1808_05510_amd import connreg, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def small_boxes(count):
    out = []
    for k in range(count):
        by = (7 + k % 3, 6 + k % 2, 5 + k % 4)
        bx = (5 + k % 2, 4 + k % 3, 4)
        out.append(synth.box_problem(box_y=by, box_x=bx, offset=(1, 1, 0), n_inj=4 + 3 * k,
                                     sigma=1.2, hole_r=1.0, wt_rank=3, wt_w=(1.5, 3.0),
                                     lam=10.0 ** (1 + k % 3), seed=1000 + k))
    return out


def _np(t):
    return t.detach().cpu().numpy()


def test_batch_matches_oracle_lockstep():
    ds = small_boxes(5)
    streams = [torch.cuda.Stream() for _ in ds]
    probs = []
    for d, s in zip(ds, streams):
        with torch.cuda.stream(s):
            probs.append(connreg.Problem(d, "fp64", DEV, stream=s))
    o = dict(max_rank=5, als_fixed_sweeps=2, pcg_rtol=1e-13, pcg_maxit=20000,
             galerkin_rtol=1e-13, galerkin_maxit=20000, seed=3)
    res = connreg.greedy_solve_batch(probs, [o] * len(probs))
    for d, r in zip(ds, res):
        P = oop.problem_from_arrays(d)
        ref = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=5, als_fixed_sweeps=2,
                                                            u_method="dense", v_method="dense",
                                                            galerkin="dense", seed=3))
        U, V, Z = _np(r["U"]), _np(r["V"]), _np(r["Z"])
        err = omet.diff_norm(U, Z, V, ref.U, ref.Z, ref.V) / omet.low_rank_norm(ref.U, ref.Z, ref.V)
        assert r["rank"] == 5 and r["status"] == "ok" and err < 1e-6
    for p in probs:
        p.close()


def test_batch_with_large_problems_matches_sequential():
    ds = small_boxes(6)
    for k in range(2):
        ds.append(synth.box_problem(box_y=(48, 44, 40), box_x=(20, 18, 16), offset=(4, 4, 4),
                                    n_inj=20, sigma=2.0, hole_r=2.0, wt_rank=4, wt_w=(2.0, 6.0),
                                    lam=300.0, seed=77 + k))
    streams = [torch.cuda.Stream() for _ in ds]
    probs = [connreg.Problem(d, "fp64", DEV, stream=s) for d, s in zip(ds, streams)]
    o = dict(max_rank=3, als_fixed_sweeps=2, pcg_rtol=1e-12, pcg_maxit=20000,
             galerkin_rtol=1e-12, galerkin_maxit=20000, seed=5)
    seq = [p.greedy_solve(**o) for p in probs]
    bat = connreg.greedy_solve_batch(probs, [o] * len(probs))
    for a, b in zip(seq, bat):
        x = [_np(a[k]) for k in ("U", "Z", "V")]
        y = [_np(b[k]) for k in ("U", "Z", "V")]
        err = omet.diff_norm(y[0], y[1], y[2], x[0], x[1], x[2]) / omet.low_rank_norm(*x)
        assert b["status"] == "ok" and b["rank"] == a["rank"] == 3 and err < 1e-8
    for p in probs:
        p.close()


def test_batch_rejects_shared_stream():
    ds = small_boxes(2)
    probs = [connreg.Problem(d, "fp64", DEV) for d in ds]  # both on the current stream
    with pytest.raises(connreg.ConnRegError):
        connreg.greedy_solve_batch(probs, [dict(max_rank=2)] * 2)


def test_autotune_picks_a_valid_shape_and_keeps_results():
    d = synth.box_problem(box_y=(20, 18, 16), box_x=(14, 12, 10), offset=(2, 2, 2), n_inj=12,
                          sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 5.0), lam=100.0, seed=8)
    g = connreg.Problem(d, "fp64", DEV)
    o = dict(max_rank=4, als_fixed_sweeps=2, pcg_rtol=1e-12, galerkin_rtol=1e-12, seed=1)
    base = g.greedy_solve(**o)
    vu, vv, tu, tv = g.autotune()
    assert vu in (1, 2, 4, 8) and vv in (1, 2, 4, 8) and tu > 0 and tv > 0
    tuned = g.greedy_solve(**o)
    a = [_np(base[k]) for k in ("U", "Z", "V")]
    b = [_np(tuned[k]) for k in ("U", "Z", "V")]
    err = omet.diff_norm(b[0], b[1], b[2], a[0], a[1], a[2]) / omet.low_rank_norm(a[0], a[1], a[2])
    assert err < 1e-8
    g.set_tuning(0, 0)


def test_mixed_autotune_through_the_tuning_table(tmp_path):
    """cr_autotune_pcg on a mixed handle (its FP32 PCG), applied and reused
    through the JSON tuning table; the tuned solve keeps its accuracy."""
    d = synth.box_problem(box_y=(20, 18, 16), box_x=(14, 12, 10), offset=(2, 2, 2), n_inj=12,
                          sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 5.0), lam=100.0, seed=9)
    o = dict(max_rank=4, als_fixed_sweeps=2, pcg_rtol=1e-6, galerkin_rtol=1e-10, seed=1)
    g = connreg.Problem(d, "mixed", DEV)
    base = g.greedy_solve(**o)
    path = str(tmp_path / "tuning.json")
    e = connreg.TuningTable(path).apply(g)
    assert e["vpt_u"] in (1, 2, 4, 8) and e["vpt_v"] in (1, 2, 4, 8)
    assert e["us_per_iter_u"] > 0 and e["us_per_iter_v"] > 0
    tuned = g.greedy_solve(**o)
    a = [_np(base[k]) for k in ("U", "Z", "V")]
    b = [_np(tuned[k]) for k in ("U", "Z", "V")]
    err = omet.diff_norm(b[0], b[1], b[2], a[0], a[1], a[2]) / omet.low_rank_norm(a[0], a[1], a[2])
    assert err < 1e-4
    # a second handle of the same bucket takes the stored shape
    g2 = connreg.Problem(d, "mixed", DEV)
    e2 = connreg.TuningTable(path).apply(g2, tune_missing=False)
    assert e2 == e
    g.close()
    g2.close()
