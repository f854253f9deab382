"""Projected CG (eq. Proj_Sylv) on the GPU against the FP64 oracle, in both
tile sizes of the MFMA kernel and in the BF16-Gram form with FP64 correction
steps.

  * r <= 40: against the oracle's dense solve of the r^2 x r^2 system, 1e-9
    relative (both solves run to 1e-13);
  * r = 150: against the oracle's matrix CG run to 1e-13, 1e-9 relative;
  * r = 300 (several Gram row blocks, 19 x 19 tiles): the returned core
    satisfies the projected equation as the oracle applies it, to the
    requested 1e-12 plus rounding (1e-11 relative).
"""
import numpy as np
import pytest

from paper_1808_05510_amd import connreg
from oracle import galerkin as ogal
from oracle import operator as oop
from tests.helpers import max_rel, rand_orth, rel
from tests.test_gpu_parity import mid_box

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def np_(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def boxes():
    return {"mid3d": mid_box(), "manyinj": mid_box(seed=6, n_inj=150)}


def _problem(monkeypatch, d, tile, low, prec="fp64"):
    monkeypatch.setenv("CONNREG_GAL_TILE", str(tile))
    monkeypatch.setenv("CONNREG_GAL_LOW", str(low))
    return connreg.Problem(d, prec, DEV)


@pytest.mark.parametrize("low", [0, 1])
@pytest.mark.parametrize("tile", [16, 32])
@pytest.mark.parametrize("r", [1, 9, 40])
@pytest.mark.parametrize("name", ["mid3d", "manyinj"])
def test_projected_cg_dense(monkeypatch, boxes, name, r, tile, low):
    d = boxes[name]
    P = oop.problem_from_arrays(d)
    rng = np.random.default_rng(100 + r)
    U = rand_orth(rng, P.n_y, r)
    V = rand_orth(rng, P.n_x, r)
    g = _problem(monkeypatch, d, tile, low)
    try:
        Z, it, status = g.galerkin_project(U, V, rtol=1e-13, maxit=20000)
    finally:
        g.close()
    Zo = ogal.solve_dense(ogal.project(P, U, V))
    assert status == "ok" and it > 0
    assert max_rel(np_(Z), Zo) < 1e-9


@pytest.mark.parametrize("low", [0, 1])
@pytest.mark.parametrize("tile", [16, 32])
def test_projected_cg_r150_oracle_cg(monkeypatch, boxes, tile, low):
    d = boxes["manyinj"]
    P = oop.problem_from_arrays(d)
    r = 150
    rng = np.random.default_rng(7)
    U = rand_orth(rng, P.n_y, r)
    V = rand_orth(rng, P.n_x, r)
    pr = ogal.project(P, U, V)
    Zo, _ = ogal.solve_cg(pr, np.zeros((r, r)), rtol=1e-13, maxit=20000)
    g = _problem(monkeypatch, d, tile, low)
    try:
        Z, it, status = g.galerkin_project(U, V, rtol=1e-13, maxit=20000)
    finally:
        g.close()
    assert status == "ok"
    assert rel(np_(Z), Zo) < 1e-9
    assert max_rel(np_(Z), Zo) < 1e-9


@pytest.mark.parametrize("low", [0, 1])
@pytest.mark.parametrize("tile", [16, 32])
def test_projected_cg_r300_residual(monkeypatch, boxes, tile, low):
    d = boxes["mid3d"]
    P = oop.problem_from_arrays(d)
    r = 300
    rng = np.random.default_rng(8)
    U = rand_orth(rng, P.n_y, r)
    V = rand_orth(rng, P.n_x, r)
    pr = ogal.project(P, U, V)
    g = _problem(monkeypatch, d, tile, low)
    try:
        Z, it, status = g.galerkin_project(U, V, rtol=1e-12, maxit=40000)
    finally:
        g.close()
    assert status == "ok" and it > 0
    B = ogal.rhs(pr)
    res = np.linalg.norm(B - ogal.apply_Ap(pr, np_(Z))) / np.linalg.norm(B)
    assert res < 1e-11, res


def test_projected_cg_warm_start_and_mixed_problem(monkeypatch, boxes):
    """A mixed-precision problem takes the BF16-Gram form by default and
    reaches the solution of its projected system (assembled from its FP32
    data) that the FP64-Gram form reaches, to the solver tolerance; a warm
    start from that solution takes no iteration."""
    d = boxes["mid3d"]
    P = oop.problem_from_arrays(d)
    r = 40
    rng = np.random.default_rng(9)
    U = rand_orth(rng, P.n_y, r)
    V = rand_orth(rng, P.n_x, r)
    Zo = ogal.solve_dense(ogal.project(P, U, V))
    monkeypatch.setenv("CONNREG_GAL_LOW", "0")
    g0 = connreg.Problem(d, "mixed", DEV)
    monkeypatch.delenv("CONNREG_GAL_LOW")
    monkeypatch.delenv("CONNREG_GAL_TILE", raising=False)
    g = connreg.Problem(d, "mixed", DEV)
    try:
        Z0, _, status0 = g0.galerkin_project(U, V, rtol=1e-13, maxit=20000)
        Z, it, status = g.galerkin_project(U, V, rtol=1e-13, maxit=20000)
        assert status0 == "ok" and status == "ok" and it > 0
        assert max_rel(np_(Z), np_(Z0)) < 1e-9
        assert max_rel(np_(Z), Zo) < 1e-4  # FP32 data against the FP64 oracle
        Z2, it2, status2 = g.galerkin_project(U, V, Z0=Z, rtol=1e-6, maxit=20000)
        assert status2 == "ok" and it2 == 0
        assert max_rel(np_(Z2), np_(Z)) == 0.0
    finally:
        g.close()
        g0.close()
