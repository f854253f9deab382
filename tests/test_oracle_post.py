"""Pins of the oracle's post-processing (SVD of the solution, the objective
in factored form, entry statistics) against dense definitions, a library
SVD of the dense matrix and brute-force loops.  CPU only."""
import numpy as np
import pytest

from paper_1808_05510_amd import synth
from oracle import operator as oop
from oracle import post as opost
from tests.helpers import rand_orth, rel


@pytest.fixture(scope="module")
def p3d():
    return oop.problem_from_arrays(synth.config2_tiny(seed=1))


def test_core_svd_is_the_svd_of_W():
    rng = np.random.default_rng(1)
    U = rand_orth(rng, 40, 6)
    V = rand_orth(rng, 25, 6)
    Z = rng.standard_normal((6, 6))
    Uh, s, Vh = opost.core_svd(U, Z, V)
    W = U @ Z @ V.T
    assert rel(Uh @ np.diag(s) @ Vh.T, W) < 1e-13
    assert np.allclose(Uh.T @ Uh, np.eye(6), atol=1e-13)
    assert np.allclose(Vh.T @ Vh, np.eye(6), atol=1e-13)
    sv = np.linalg.svd(W, compute_uv=False)[:6]
    assert np.allclose(s, sv, rtol=1e-12, atol=0)
    assert np.all(np.diff(s) <= 0)


def test_objective_factored_matches_dense(p3d):
    rng = np.random.default_rng(2)
    U = rng.standard_normal((p3d.n_y, 4))
    V = rng.standard_normal((p3d.n_x, 4))
    Z = rng.standard_normal((4, 4))
    W = U @ Z @ V.T
    J, mis, reg = opost.objective_factored(p3d, U, Z, V)
    assert abs(J - oop.objective(p3d, W)) <= 1e-12 * J
    assert abs(mis - 0.5 * np.sum((p3d.Omega * (W @ p3d.X - p3d.Y)) ** 2)) <= 1e-12 * mis
    Ly, Lx = p3d.Ly.toarray(), p3d.Lx.toarray()
    assert abs(reg - 0.5 * p3d.lam * np.sum((Ly @ W + W @ Lx.T) ** 2)) <= 1e-12 * reg


def test_entry_stats_brute_force():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((13, 3))
    B = rng.standard_normal((7, 3))
    st = opost.entry_stats(A, B, block=5)
    cnt, mn, mx, ma, ss, ssn = 0, np.inf, -np.inf, 0.0, 0.0, 0.0
    for i in range(13):
        for j in range(7):
            w = sum(A[i, k] * B[j, k] for k in range(3))
            cnt += w < 0
            mn, mx, ma = min(mn, w), max(mx, w), max(ma, abs(w))
            ss += w * w
            ssn += w * w if w < 0 else 0.0
    assert st["count_neg"] == cnt and 0 < cnt < 91
    assert st["min"] == pytest.approx(mn, rel=1e-14) and st["max"] == pytest.approx(mx, rel=1e-14)
    assert st["max_abs"] == pytest.approx(ma, rel=1e-14)
    assert st["sum_sq"] == pytest.approx(ss, rel=1e-13)
    assert st["sum_sq_neg"] == pytest.approx(ssn, rel=1e-13)


def test_oracle_paper_toy_trends_and_mask_ablation():
    """The oracle on the paper's toy brain: the distance to W_true falls
    with the rank and levels off, and dropping the mask (Omega = 1) fits the
    truth worse (section "Test problem: a toy brain"; values unpinned)."""
    from oracle import greedy as ogreedy
    kw = dict(u_method="dense", v_method="dense", galerkin="dense", tau_dW=1e-7)
    d = synth.paper_toy()
    Wt = d["Wt_dense"]
    P = oop.problem_from_arrays(d)
    err = {}
    for r in (10, 30, 40):
        res = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=r, **kw))
        err[r] = np.linalg.norm(res.U @ res.Z @ res.V.T - Wt) / np.linalg.norm(Wt)
    assert err[40] < err[10] and abs(err[40] - err[30]) <= 0.1 * err[30]
    P1 = oop.problem_from_arrays(synth.paper_toy(omega_ones=True))
    res1 = ogreedy.greedy_solve(P1, ogreedy.GreedyOptions(max_rank=40, **kw))
    assert np.linalg.norm(res1.U @ res1.Z @ res1.V.T - Wt) / np.linalg.norm(Wt) > err[40]
