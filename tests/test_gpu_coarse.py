"""The two-level preconditioner of the v-systems (cr_problem_set_coarse):
it must never change the answer (same stopping test), only the iteration
count.  Checked through the C ABI:

* greedy lockstep with the oracle on a ragged 3-D box (FP64 1e-6, mixed 1e-4)
  and on the 40^3/30^3 grids (FP64) with the coarse level on;
* the same solves with and without it agree to the inner tolerance, and the
  v-system PCG iterations drop;
* invalid set-ups are rejected.
"""
import numpy as np
import pytest
import torch

from oracle import greedy as ogreedy
from oracle import metrics as omet
from oracle import operator as oop
from paper_1808_05510_amd import connreg, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def np_(t):
    return t.detach().to("cpu", torch.float64).numpy()


def mid_box(n_inj=37, seed=4):
    return synth.box_problem(box_y=(11, 10, 9), box_x=(8, 7, 9), offset=(1, 2, 0), n_inj=n_inj,
                             sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 4.0), lam=30.0, seed=seed)


def werr(res, ref):
    U, V, Z = np_(res["U"]), np_(res["V"]), np_(res["Z"])
    Ur, Zr, Vr = ref
    return omet.diff_norm(U, Z, V, Ur, Zr, Vr) / omet.low_rank_norm(Ur, Zr, Vr)


@pytest.mark.parametrize("prec,tol,n_inj", [("fp64", 1e-6, 37), ("mixed", 1e-4, 37),
                                            ("fp64", 1e-6, 100), ("mixed", 1e-4, 100)])
def test_greedy_lockstep_with_coarse(prec, tol, n_inj):
    d = mid_box(n_inj=n_inj)
    P = oop.problem_from_arrays(d)
    ores = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=6, als_fixed_sweeps=2,
                                                         u_method="dense", v_method="dense",
                                                         galerkin="dense", seed=3))
    g = connreg.Problem(d, prec, DEV)
    g.set_coarse(d["coords_x"], 3)
    res = g.greedy_solve(max_rank=6, als_fixed_sweeps=2, pcg_rtol=1e-13, pcg_maxit=20000,
                         galerkin_rtol=1e-13, galerkin_maxit=20000, seed=3)
    g.close()
    assert res["rank"] == 6
    err = werr(res, (ores.U, ores.Z, ores.V))
    print(f"[coarse] {prec} n_inj {n_inj}: W error vs oracle {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_coarse_keeps_answer_and_cuts_v_iterations(prec):
    d = synth.config2(lam=1e3, seed=0)
    o = dict(max_rank=4, als_fixed_sweeps=2, pcg_rtol=1e-10, pcg_maxit=200000, seed=0,
             galerkin_rtol=1e-12, galerkin_maxit=20000)
    g = connreg.Problem(d, prec, DEV)
    r0 = g.greedy_solve(**o)
    g.set_coarse(d["coords_x"], 5)
    r1 = g.greedy_solve(**o)
    g.close()
    err = werr(r1, tuple(np_(r0[k]) for k in ("U", "Z", "V")))
    it0, it1 = r0["stats"]["pcg_iters"], r1["stats"]["pcg_iters"]
    print(f"[coarse] {prec} 40^3/30^3: PCG iterations {it0} -> {it1}, W difference {err:.2e}")
    assert err <= (1e-7 if prec == "fp64" else 1e-4)
    assert it1 < 0.8 * it0


def test_set_coarse_rejects_bad_input():
    d = mid_box()
    g = connreg.Problem(d, "fp64", DEV)
    with pytest.raises(connreg.ConnRegError):
        g.set_coarse(d["coords_x"], 7)  # 7^3 > 256 voxels per aggregate
    with pytest.raises(connreg.ConnRegError):
        connreg._check(connreg.load().cr_problem_set_coarse(g.h, 0, None, 3, 3))
    g.set_coarse(d["coords_x"], 0)  # off
    g.close()
