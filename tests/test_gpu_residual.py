"""The residual norm of Algorithm 1's stopping test (||D - A(W)||_F /
||D||_F, FP64) in its two forms, through the C ABI against the oracle
(which takes thin QR factors of the stacked residual factors):

* the Gram form trace((F^T F)(G^T G)), whose absolute error is near
  sqrt(eps) ||F|| ||G||, used while relres is above 1e-6;
* CholQR2 factors R_F, R_G with ||R||_F = ||R_F Cm R_G^T||_F (error near
  eps ||F|| ||G||), used below it (CONNREG_RESID_QR=2: always);
* the greedy loop's incrementally updated residual Grams, which must give
  the relres of the factors it returns at every rank.
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


def mid_box():
    return synth.box_problem(box_y=(11, 10, 9), box_x=(8, 7, 9), offset=(1, 2, 0), n_inj=37,
                             sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 4.0), lam=30.0, seed=4)


def small_target_box():
    """mid_box with the two grids swapped in size: 504 target, 990 source voxels."""
    return synth.box_problem(box_y=(8, 7, 9), box_x=(11, 10, 9), offset=(0, 0, 0), n_inj=37,
                             sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 4.0), lam=30.0, seed=4)


# r = 160 (k = 37 + 3 r = 517 columns): on mid_box the source-side factor has
# more columns than its 504 rows, so only the target side has a CholQR2
# factor; on small_target_box the other way round
@pytest.mark.parametrize("maker,r", [(synth.config1, 5), (mid_box, 12), (mid_box, 40),
                                     (mid_box, 160), (small_target_box, 160)])
def test_residual_norm_cholqr2_matches_oracle(monkeypatch, maker, r):
    monkeypatch.setenv("CONNREG_RESID_QR", "2")
    d = maker()
    P = oop.problem_from_arrays(d)
    rng = np.random.default_rng(r)
    U = np.linalg.qr(rng.standard_normal((P.n_y, r)))[0]
    V = np.linalg.qr(rng.standard_normal((P.n_x, r)))[0]
    Z = rng.standard_normal((r, r))
    g = connreg.Problem(d, "fp64", DEV)
    a, b = g.residual_norm(U, Z, V)
    g.close()
    ao, bo = omet.residual_norm(P, U, Z, V)
    assert abs(a - ao) <= 1e-12 * ao
    assert abs(b - bo) <= 1e-12 * bo


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_greedy_tiny_relres_at_full_rank(prec):
    """The 40-voxel toy to its full rank 40, where W = W*.  In FP64 the
    relative residual falls to rounding level and the solve stops on
    tau_res = 1e-10; in mixed precision the FP32 storage of the bases sets a
    floor near 1e-6, which the library's relres must report faithfully.
    Near full rank both residual factors have more columns than rows, so the
    library forms the residual's entries."""
    d = synth.config1_small(seed=0)
    P = oop.problem_from_arrays(d)
    g = connreg.Problem(d, prec, DEV)
    res = g.greedy_solve(max_rank=40, tau_res=1e-10, als_fixed_sweeps=2, pcg_rtol=1e-13,
                         pcg_maxit=50000, galerkin_rtol=1e-14, galerkin_maxit=50000, seed=0)
    g.close()
    U, V, Z = np_(res["U"]), np_(res["V"]), np_(res["Z"])
    ro = omet.residual_norm(P, U, Z, V)[1]
    rg = res["stats"]["relres"]
    print(f"[resid] {prec}: rank {res['rank']}, library relres {rg:.3e}, oracle {ro:.3e}")
    if prec == "fp64":
        assert rg <= 1e-10 and ro <= 1e-10
        assert abs(rg - ro) <= 1e-13
    else:
        assert ro <= 1e-5 and abs(rg - ro) <= 1e-5


@pytest.mark.parametrize("r", [35, 45])
def test_residual_norm_small_relres_from_cholqr2(r):
    """A near-exact low-rank W (the exact solution with Omega = 1, whose
    right-hand side has rank n_inj, truncated by its SVD) has a relative
    residual far below 1e-6 (1e-7 and 1e-10 at ranks 35 and 45): the
    library's automatic switch to CholQR2 factors must reproduce the
    oracle's QR value."""
    from oracle import dense as odense
    d = synth.config1(seed=1)
    d["Omega"] = np.ones_like(d["Omega"])
    P = oop.problem_from_arrays(d)
    Ws = odense.solve_full_mask(P, (200,), (200,))
    Uf, s, Vt = np.linalg.svd(Ws)
    U, Z, V = Uf[:, :r], np.diag(s[:r]), Vt[:r].T
    ao, bo = omet.residual_norm(P, U, Z, V)
    g = connreg.Problem(d, "fp64", DEV)
    a, b = g.residual_norm(U, Z, V)
    g.close()
    print(f"[resid] truncated exact solution: oracle relres {bo:.3e}, library {b:.3e}")
    assert bo < 1e-6
    if r == 35:
        assert abs(b - bo) <= 1e-3 * bo + 1e-14
    else:
        # at rank 45 the columns of [N | U | L_y U | L_y^2 U] (140 of them in
        # 200 rows) are numerically dependent, CholQR2's Cholesky fails and
        # the Gram form is kept: its value is then only as accurate as its
        # floor, sqrt(eps k) ||F_R|| ||G_R|| / ||D||
        F, G = oop.residual_factors(P, U, Z, V)
        floor = np.sqrt(2.2e-16 * F.shape[1]) * np.linalg.norm(F) * np.linalg.norm(G) / omet.d_norm(P)
        assert abs(b - bo) <= floor, (b, bo, floor)


def test_greedy_incremental_grams_give_each_ranks_relres():
    """Per-rank relres of a lockstep greedy run (incremental residual Grams)
    against the oracle's lockstep run, at every rank."""
    d = mid_box()
    P = oop.problem_from_arrays(d)
    ores = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=10, als_fixed_sweeps=2,
                                                         u_method="dense", v_method="dense",
                                                         galerkin="dense", seed=2))
    g = connreg.Problem(d, "fp64", DEV)
    res = g.greedy_solve(max_rank=10, als_fixed_sweeps=2, pcg_rtol=1e-13, pcg_maxit=20000,
                         galerkin_rtol=1e-13, galerkin_maxit=20000, seed=2)
    g.close()
    for hg, ho in zip(res["history"], ores.history):
        assert abs(hg["relres"] - ho["relres"]) <= 1e-7 * ho["relres"], (hg["rank"], hg["relres"],
                                                                          ho["relres"])


def test_barrier_timeout_surfaces_through_deferred_reads(monkeypatch):
    """A grid barrier that gives up (forced from the host: a poll bound of
    one, so waiting workgroups time out at once; every kernel still runs to
    its end) must turn into an error even where the PCG scalars are read
    after the next launch has cleared the barrier words (the FP64 u-solve's
    deferred read)."""
    monkeypatch.setenv("CONNREG_BAR_SPIN", "1")
    d = synth.config2(lam=1e3, seed=0)  # 63 u-system and 106 v-system workgroups
    g = connreg.Problem(d, "fp64", DEV)
    with pytest.raises(connreg.ConnRegError, match="timed out"):
        g.greedy_solve(max_rank=2, seed=0)
    g.close()
