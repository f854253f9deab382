"""Parity at the benchmark's full sizes, in the launch configurations that
bench.py times.

* op_apply on the cortex-shell workload (n_y 262,136, n_x 131,068, n_inj 128)
  at r = 100, FP64 and FP32 handles: every output element against the FP64
  oracle (sparse products and one dense product, under a second each at this
  size), at the bars of the small cases (1e-13 / 1e-12 FP64, 2e-6 FP32).
* The greedy solve on the 40^3 / 30^3 grids (n_y 64,000, n_x 27,000, n_inj
  64): three ranks in lockstep with the oracle (same initial vectors, two ALS
  sweeps per rank, inner solves to 1e-12 on both sides), W within 1e-6 (FP64)
  and 1e-4 (mixed precision).
* A u-system of that grid (eq. ALS_linsys, n_y 64,000) solved by Jacobi-PCG,
  by flexible CG with the spectral base step and with the (untrained)
  network, against the oracle's Jacobi-CG solution at 1e-13.
* An ALS step of that grid with both boxes declared (flexible CG with the
  spectral base step for u, the SMW direct solve for v: the solvers of the
  mixed + learned-preconditioner benchmark) in lockstep with the oracle's ALS.
* The benchmark's 16-problem batch (n_y 20k-120k, n_inj 16-128): one batched
  call against the same problems solved one at a time (a property at any
  size: the same factors to the inner tolerance), three ranks in FP64.
"""
import numpy as np
import pytest
import torch

from oracle import als as oals
from oracle import greedy as ogreedy
from oracle import metrics as omet
from oracle import operator as oop
from paper_1808_05510_amd import connreg, synth
from tests.helpers import max_rel, rand_orth, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def np_(t):
    return t.detach().to("cpu", torch.float64).numpy()


@pytest.fixture(scope="module")
def shells():
    d = synth.config3(seed=0)
    return d, oop.problem_from_arrays(d)


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("fp32", [False, True])
def test_op_apply_full_shells_r100(shells, fp32, fused, monkeypatch):
    """Default path, and the fused ring-2 window sweeps (CONNREG_OP_FUSED=2)."""
    monkeypatch.setenv("CONNREG_OP_FUSED", "2" if fused else "0")
    d, P = shells
    r = 100
    rng = np.random.default_rng(21)
    U = rng.standard_normal((P.n_y, r))
    V = rng.standard_normal((P.n_x, r))
    Z = rng.standard_normal((r, r))
    if fp32:  # the FP32 path takes FP32 inputs: compare on the rounded values
        U, V, Z = (a.astype(np.float32).astype(np.float64) for a in (U, V, Z))
    g = connreg.Problem(d, "mixed" if fp32 else "fp64", DEV)
    F, G = g.op_apply(U, Z, V, fp32=fp32)
    F, G = np_(F), np_(G)
    g.close()
    f = oop.op_apply(P, U, Z, V)
    assert F.shape == (P.n_y, 2 * r + P.n_inj) and G.shape == (P.n_x, 2 * r)
    tol, tol_m = (2e-6, 2e-6) if fp32 else (1e-13, 1e-12)
    assert rel(F[:, :r], f.LyU) < tol
    assert rel(F[:, r:2 * r], f.Ly2U) < tol
    assert rel(G[:, :r], f.LxV) < tol
    assert rel(G[:, r:], f.Lx2V) < tol
    assert rel(F[:, 2 * r:], f.M) < tol_m
    # every element, relative to its block's largest entry
    for a, b in ((F[:, :r], f.LyU), (F[:, r:2 * r], f.Ly2U), (G[:, :r], f.LxV),
                 (G[:, r:], f.Lx2V)):
        assert max_rel(a, b) < tol
    assert max_rel(F[:, 2 * r:], f.M) < tol_m


def test_op_apply_factors_full_shells_r100(shells):
    """The factor pair F G^T = A(U Z V^T) at full size: sampled entries of
    A(W) from the oracle's factors, and ||A(W)||_F by thin QR of both pairs."""
    d, P = shells
    r = 100
    rng = np.random.default_rng(22)
    U = rng.standard_normal((P.n_y, r))
    V = rng.standard_normal((P.n_x, r))
    Z = rng.standard_normal((r, r))
    g = connreg.Problem(d, "fp64", DEV)
    F, G = g.op_apply_factors(U, Z, V)
    F, G = np_(F), np_(G)
    g.close()
    f = oop.op_apply(P, U, Z, V)
    rows = rng.choice(P.n_y, 400, replace=False)
    cols = rng.choice(P.n_x, 300, replace=False)
    # oracle entries A(W)[i, k] of eq. multitermSylv, term by term
    want = (P.lam * (U[rows] @ Z @ f.Lx2V[cols].T + 2.0 * f.LyU[rows] @ Z @ f.LxV[cols].T
                     + f.Ly2U[rows] @ Z @ V[cols].T) + f.M[rows] @ P.X[cols].T)
    got = F[rows] @ G[cols].T
    assert max_rel(got, want) < 1e-12
    Fo = np.hstack([P.lam * U, 2.0 * P.lam * f.LyU, P.lam * f.Ly2U, f.M])
    Go = np.hstack([f.Lx2V @ Z.T, f.LxV @ Z.T, V @ Z.T, P.X])
    n_or = omet.fro_factored(Fo, Go)
    assert abs(omet.fro_factored(F, G) - n_or) <= 1e-11 * n_or


@pytest.fixture(scope="module")
def grid_oracle():
    d = synth.config2(lam=1e3, seed=0)
    P = oop.problem_from_arrays(d)
    ores = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(
        max_rank=3, als_fixed_sweeps=2, galerkin="dense", seed=0, u_method="cg", v_method="cg",
        inner_rtol=1e-12))
    return d, ores


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_greedy_full_grid_lockstep(grid_oracle, prec, tol):
    d, ores = grid_oracle
    R = 3
    g = connreg.Problem(d, prec, DEV)
    res = g.greedy_solve(max_rank=R, als_fixed_sweeps=2, pcg_rtol=1e-12, pcg_maxit=200000,
                         galerkin_rtol=1e-13, galerkin_maxit=20000, seed=0)
    g.close()
    assert res["rank"] == R
    U, V, Z = np_(res["U"]), np_(res["V"]), np_(res["Z"])
    err = (omet.diff_norm(U, Z, V, ores.U, ores.Z, ores.V)
           / omet.low_rank_norm(ores.U, ores.Z, ores.V))
    assert err <= tol, err
    for hg, ho in zip(res["history"], ores.history):
        assert abs(hg["relres"] - ho["relres"]) <= (1e-6 if prec == "fp64" else 1e-3) * ho["relres"]


def test_u_solves_full_grid():
    d = synth.config2(lam=1e3, seed=0)
    P = oop.problem_from_arrays(d)
    rng = np.random.default_rng(31)
    r = 3
    U = rand_orth(rng, P.n_y, r)
    V = rand_orth(rng, P.n_x, r)
    Z = rng.standard_normal((r, r))
    v = rng.standard_normal(P.n_x)
    v /= np.linalg.norm(v)
    g = connreg.Problem(d, "fp64", DEV)
    g.set_box(d["box_y"])
    rhs, dd, coef = g.u_system(U, Z, V, v)
    xref = oals.solve_u(P, v, rhs.cpu().numpy(), method="cg", rtol=1e-13, maxit=200000)
    xs = {}
    for kind in ("jacobi", "base"):
        x, it, rr, fb, st = g.u_solve(dd, coef, rhs, rtol=1e-13, maxit=200000, precond=kind)
        assert st == "ok", (kind, st)
        xs[kind] = x.cpu().numpy()
        assert rel(xs[kind], xref) < 1e-7, kind
    pc = connreg.Pc(d["box_y"], channels=8, seed=7)
    x, it, rr, fb, st = g.u_solve(dd, coef, rhs, rtol=1e-13, maxit=200000, pc=pc)
    assert st in ("ok", "pc_fallback") and rel(x.cpu().numpy(), xref) < 1e-7
    assert rel(xs["base"], xs["jacobi"]) < 1e-7
    pc.close()
    g.close()


def test_als_step_full_grid_spectral_and_smw():
    d = synth.config2(lam=1e3, seed=0)
    P = oop.problem_from_arrays(d)
    rng = np.random.default_rng(41)
    r = 3
    U = rand_orth(rng, P.n_y, r)
    V = rand_orth(rng, P.n_x, r)
    Z = rng.standard_normal((r, r))
    F, G = oop.residual_factors(P, U, Z, V)
    v0 = ogreedy.init_v(P, F, G, 7, r)
    a = oals.als(P, F, G, v0, fixed_sweeps=2, u_method="cg", v_method="cg", rtol=1e-13)
    g = connreg.Problem(d, "fp64", DEV)
    g.set_box(d["box_y"])
    g.set_box(d["box_x"], which="source")
    g.set_precond("base")
    u, v, st = g.als_step(U, Z, V, v0, als_fixed_sweeps=2, pcg_rtol=1e-13, pcg_maxit=200000)
    g.close()
    assert st["sweeps"] == 2 and st["status"] == "ok"
    assert abs(abs(float(np_(u) @ a.u)) - 1.0) < 1e-9
    assert abs(abs(float(np_(v) @ a.v)) - 1.0) < 1e-9
    # (solutions to 1e-13 of systems with condition numbers up to about 1e6)
    assert abs(st["unorm"] - a.unorm) <= 1e-7 * a.unorm
    assert abs(st["vnorm"] - a.vnorm) <= 1e-7 * a.vnorm


def test_batch_full_size_matches_one_at_a_time():
    specs = synth.config4_specs(0, 16)
    ds = [synth.box_problem(box_y=sp.box_y, box_x=sp.box_x,
                            offset=tuple((np.array(sp.box_y) - np.array(sp.box_x)) // 2),
                            n_inj=sp.n_inj, lam=sp.lam, max_rank=3, seed=sp.seed) for sp in specs]
    streams = [torch.cuda.Stream() for _ in ds]
    probs = [connreg.Problem(d, "fp64", DEV, stream=st) for d, st in zip(ds, streams)]
    o = dict(max_rank=3, als_fixed_sweeps=2, pcg_rtol=1e-12, pcg_maxit=200000,
             galerkin_rtol=1e-12, galerkin_maxit=20000, seed=5)
    seq = [p.greedy_solve(**o) for p in probs]
    bat = connreg.greedy_solve_batch(probs, [o] * len(probs))
    for a, b in zip(seq, bat):
        x = [np_(a[k]) for k in ("U", "Z", "V")]
        y = [np_(b[k]) for k in ("U", "Z", "V")]
        err = omet.diff_norm(y[0], y[1], y[2], x[0], x[1], x[2]) / omet.low_rank_norm(*x)
        assert b["status"] == "ok" and b["rank"] == a["rank"] == 3 and err < 1e-8, err
    for p in probs:
        p.close()
