"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Tolerances:
  * stencils / factored products in FP64: 1e-12 relative (summation order);
  * FP32 storage: 2e-6 relative (about 16 unit roundoffs of float32);
  * residual norm: its Gram form loses half the digits, bound
    1e-15 * k * (||F_R|| ||G_R|| / ||R||)^2 relative (k = factor width);
  * projected CG / PCG solves run to 1e-13 and are compared at 1e-9;
  * greedy solve, lockstep (same initial vectors, fixed ALS sweeps, tight
    inner solves): relative W difference <= 1e-6 in FP64 and <= 1e-4 in
    mixed precision, the two targets the solver is specified to meet.
"""
import numpy as np
import pytest
import torch

from paper_1808_05510_amd import connreg, synth
from oracle import als as oals
from oracle import dense as odense
from oracle import galerkin as ogal
from oracle import greedy as ogreedy
from oracle import metrics as omet
from oracle import operator as oop
from tests.helpers import max_rel, rand_orth, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def np_(t):
    return t.detach().cpu().numpy()


def mid_box(seed=4, n_inj=37):
    """Ragged sizes: 990 / 504 voxels, 37 injections (not multiples of any tile)."""
    return synth.box_problem(box_y=(11, 10, 9), box_x=(8, 7, 9), offset=(1, 2, 0), n_inj=n_inj,
                             sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 4.0), lam=30.0,
                             seed=seed)


def dense_mask_box(seed=5):
    """Omega with ~40% unobserved entries, so the library takes its dense-mask path."""
    d = mid_box(seed=seed, n_inj=19)
    rng = np.random.default_rng(seed)
    d["Omega"] = (rng.random(d["Omega"].shape) > 0.4).astype(np.uint8)
    return d


def scrambled_box(seed=7):
    """mid_box with the target voxels renumbered at random: the Laplacian is
    the same graph, but neighbours lie anywhere in the index range, so the
    library has no LDS-window tables and every stencil takes the gather form."""
    import scipy.sparse as sp
    # 2,688 target voxels: a tile's scattered neighbours then span more than
    # the 2,048-voxel window
    d = synth.box_problem(box_y=(16, 14, 12), box_x=(8, 7, 9), offset=(1, 2, 0), n_inj=21,
                          sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 4.0), lam=30.0, seed=seed)
    n = len(d["Ly_rowptr"]) - 1
    perm = np.random.default_rng(seed).permutation(n)
    L = sp.csr_matrix((d["Ly_val"], d["Ly_colidx"], d["Ly_rowptr"]), shape=(n, n))
    Lp = L[perm][:, perm].tocsr()
    Lp.sort_indices()
    d["Ly_rowptr"] = Lp.indptr.astype(np.int32)
    d["Ly_colidx"] = Lp.indices.astype(np.int32)
    d["Ly_val"] = Lp.data.astype(np.float64)
    for k in ("Y", "Omega", "coords_y", "Wt_g"):
        d[k] = np.ascontiguousarray(d[k][perm])
    d.pop("box_y", None)
    return d


CASES = {
    "toy1d": lambda: synth.config1(),
    "tiny3d": lambda: synth.config2_tiny(),
    "mid3d": mid_box,
    "densemask": dense_mask_box,
    # more than one 128-injection block of the masked products
    "manyinj": lambda: mid_box(seed=6, n_inj=150),
    "scrambled": scrambled_box,
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    d = CASES[request.param]()
    return request.param, d, oop.problem_from_arrays(d)


# ------------------------------------------------------------------ op_apply
# 112 is the largest rank of the register-resident masked product, 120 takes
# the LDS-chunked one; 64 is the last padded k-step count, 67 and 100 take
# exact ones (67 with a partial last step); 150 makes T = Z H loop over two
# 128-row chunks
@pytest.mark.parametrize("r", [0, 1, 7, 64, 67, 100, 112, 120, 150])
def test_op_apply_fp64(case, r):
    name, d, P = case
    r = min(r, P.n_x)
    rng = np.random.default_rng(r + 11)
    U = rng.standard_normal((P.n_y, r))
    V = rng.standard_normal((P.n_x, r))
    Z = rng.standard_normal((r, r))
    g = connreg.Problem(d, "fp64", DEV)
    F, G = g.op_apply(U, Z, V)
    f = oop.op_apply(P, U, Z, V)
    F, G = np_(F), np_(G)
    assert F.shape == (P.n_y, 2 * r + P.n_inj)
    if r:
        assert rel(F[:, :r], f.LyU) < 1e-13
        assert rel(F[:, r:2 * r], f.Ly2U) < 1e-13
        assert rel(G[:, :r], f.LxV) < 1e-13
        assert rel(G[:, r:], f.Lx2V) < 1e-13
        assert rel(F[:, 2 * r:], f.M) < 1e-12
        # element by element (relative to the block's largest entry)
        for a, b in ((F[:, :r], f.LyU), (F[:, r:2 * r], f.Ly2U), (G[:, :r], f.LxV),
                     (G[:, r:], f.Lx2V)):
            assert max_rel(a, b) < 1e-13
        assert max_rel(F[:, 2 * r:], f.M) < 1e-12
    else:
        assert np.abs(F).max() == 0.0
    if name == "tiny3d" and r:
        # the factored form reassembles to the dense operator
        Wd = U @ Z @ V.T
        A = (P.lam * (U @ Z @ G[:, r:].T + 2 * F[:, :r] @ Z @ G[:, :r].T + F[:, r:2 * r] @ Z @ V.T)
             + F[:, 2 * r:] @ P.X.T)
        assert rel(A, oop.apply_A(P, Wd)) < 1e-12


@pytest.mark.parametrize("r", [0, 1, 7, 40, 100])
def test_op_apply_factors(case, r):
    """cr_op_apply_factors: F G^T is A(U Z V^T) with no lambda or Z
    arithmetic left to the caller (k = 3r + n_inj columns)."""
    name, d, P = case
    r = min(r, P.n_x)
    rng = np.random.default_rng(r + 31)
    U = rng.standard_normal((P.n_y, r))
    V = rng.standard_normal((P.n_x, r))
    Z = rng.standard_normal((r, r))
    g = connreg.Problem(d, "fp64", DEV)
    F, G = g.op_apply_factors(U, Z, V)
    F, G = np_(F), np_(G)
    g.close()
    k = 3 * r + P.n_inj
    assert F.shape == (P.n_y, k) and G.shape == (P.n_x, k)
    A = oop.apply_A(P, U @ Z @ V.T)
    assert rel(F @ G.T, A) < 1e-12
    assert max_rel(F @ G.T, A) < 1e-12


# FP32 sweeps of 8 or more columns take the LDS-window stencil where the
# geometry has window tables (all cases but "scrambled")
@pytest.mark.parametrize("r", [1, 8, 67, 100, 120])
def test_op_apply_fp32(case, r):
    name, d, P = case
    r = min(r, P.n_x)
    rng = np.random.default_rng(r + 12)
    U = rng.standard_normal((P.n_y, r)).astype(np.float32).astype(np.float64)
    V = rng.standard_normal((P.n_x, r)).astype(np.float32).astype(np.float64)
    Z = rng.standard_normal((r, r)).astype(np.float32).astype(np.float64)
    g = connreg.Problem(d, "mixed", DEV)
    F, G = g.op_apply(U, Z, V, fp32=True)
    f = oop.op_apply(P, U, Z, V)
    F, G = np_(F).astype(np.float64), np_(G).astype(np.float64)
    assert rel(F[:, :r], f.LyU) < 2e-6
    assert rel(F[:, r:2 * r], f.Ly2U) < 2e-6
    assert rel(G[:, r:], f.Lx2V) < 2e-6
    assert rel(F[:, 2 * r:], f.M) < 2e-6


@pytest.mark.parametrize("r", [1, 7, 67, 100, 150])
@pytest.mark.parametrize("fp32", [False, True])
def test_op_apply_fused_sweep(case, r, fp32, monkeypatch):
    """The fused ring-2 window sweeps (CONNREG_OP_FUSED=2: L w and L^2 w in
    one pass per side, the masked product from the target pass's staged
    values) against the oracle at the same bars as the default path.  The
    scrambled geometry has no ring-2 tables and 150 injections exceed the
    fused product's 128: both take the default path."""
    monkeypatch.setenv("CONNREG_OP_FUSED", "2")
    name, d, P = case
    r = min(r, P.n_x)
    rng = np.random.default_rng(r + 31)
    U = rng.standard_normal((P.n_y, r))
    V = rng.standard_normal((P.n_x, r))
    Z = rng.standard_normal((r, r))
    if fp32:
        U, V, Z = (a.astype(np.float32).astype(np.float64) for a in (U, V, Z))
    g = connreg.Problem(d, "mixed" if fp32 else "fp64", DEV)
    F, G = g.op_apply(U, Z, V, fp32=fp32)
    g.close()
    f = oop.op_apply(P, U, Z, V)
    F, G = np_(F).astype(np.float64), np_(G).astype(np.float64)
    tol, tol_m = (2e-6, 2e-6) if fp32 else (1e-13, 1e-12)
    for a, b in ((F[:, :r], f.LyU), (F[:, r:2 * r], f.Ly2U), (G[:, :r], f.LxV),
                 (G[:, r:], f.Lx2V)):
        assert rel(a, b) < tol
        assert max_rel(a, b) < tol
    assert rel(F[:, 2 * r:], f.M) < tol_m
    assert max_rel(F[:, 2 * r:], f.M) < tol_m


# ------------------------------------------------------------------ residual norm
def test_residual_norm(case):
    name, d, P = case
    rng = np.random.default_rng(13)
    for r in (0, 3, 9):
        U = rand_orth(rng, P.n_y, r) if r else np.zeros((P.n_y, 0))
        V = rand_orth(rng, P.n_x, r) if r else np.zeros((P.n_x, 0))
        Z = rng.standard_normal((r, r)) * 0.1
        g = connreg.Problem(d, "fp64", DEV)
        a, b = g.residual_norm(U, Z, V)
        Fr, Gr = oop.residual_factors(P, U, Z, V)
        ref = omet.fro_factored(Fr, Gr)
        k = Fr.shape[1]
        bound = 1e-15 * k * (np.linalg.norm(Fr) * np.linalg.norm(Gr) / ref) ** 2 + 1e-13
        assert abs(a - ref) <= bound * ref, (r, a, ref, bound)
        assert abs(b - ref / omet.d_norm(P)) <= bound * ref / omet.d_norm(P)
    assert abs(g.rhs_norm() - omet.d_norm(P)) <= 1e-12 * omet.d_norm(P)


# ------------------------------------------------------------------ Galerkin
@pytest.mark.parametrize("r", [1, 9, 40])
def test_galerkin_project(case, r):
    name, d, P = case
    r = min(r, P.n_x)
    rng = np.random.default_rng(14 + r)
    U = rand_orth(rng, P.n_y, r)
    V = rand_orth(rng, P.n_x, r)
    g = connreg.Problem(d, "fp64", DEV)
    Z, it, status = g.galerkin_project(U, V, rtol=1e-13, maxit=20000)
    Zo = ogal.solve_dense(ogal.project(P, U, V))
    assert status == "ok" and it > 0
    assert rel(np_(Z), Zo) < 1e-9


# ------------------------------------------------------------------ ALS
def test_als_step_lockstep(case):
    name, d, P = case
    ores = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=3, u_method="dense" if P.n_y < 3000 else "direct",
                                                         v_method="dense" if P.n_x < 3000 else "smw",
                                                         galerkin="dense", als_fixed_sweeps=2))
    U, V, Z = ores.U, ores.V, ores.Z
    F, G = oop.residual_factors(P, U, Z, V)
    v0 = ogreedy.init_v(P, F, G, 7, 3)
    a = oals.als(P, F, G, v0, fixed_sweeps=2, u_method="direct", v_method="smw")
    g = connreg.Problem(d, "fp64", DEV)
    u, v, st = g.als_step(U, Z, V, v0, als_fixed_sweeps=2, pcg_rtol=1e-13, pcg_maxit=20000)
    assert st["sweeps"] == 2 and st["status"] == "ok"
    assert abs(abs(float(np_(u) @ a.u)) - 1.0) < 1e-9
    assert abs(abs(float(np_(v) @ a.v)) - 1.0) < 1e-9
    assert abs(st["unorm"] - a.unorm) <= 1e-9 * a.unorm
    assert abs(st["vnorm"] - a.vnorm) <= 1e-9 * a.vnorm


# ------------------------------------------------------------------ greedy
def _wdiff(U1, Z1, V1, U2, Z2, V2):
    return omet.diff_norm(U1, Z1, V1, U2, Z2, V2) / omet.low_rank_norm(U2, Z2, V2)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_greedy_lockstep(case, prec, tol):
    name, d, P = case
    R = min(8, P.n_x)
    ores = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(
        max_rank=R, als_fixed_sweeps=3, galerkin="dense", seed=5,
        u_method="dense" if P.n_y < 3000 else "direct",
        v_method="dense" if P.n_x < 3000 else "smw"))
    g = connreg.Problem(d, prec, DEV)
    res = g.greedy_solve(max_rank=R, als_fixed_sweeps=3, pcg_rtol=1e-13, pcg_maxit=20000,
                         galerkin_rtol=1e-13, galerkin_maxit=20000, seed=5)
    assert res["rank"] == R
    U, V, Z = np_(res["U"]), np_(res["V"]), np_(res["Z"])
    assert np.allclose(U.T @ U, np.eye(R), atol=1e-12 if prec == "fp64" else 1e-5)
    err = _wdiff(U, Z, V, ores.U, ores.Z, ores.V)
    assert err <= tol, err
    # per-rank relative residual as reported by the library vs the oracle's
    for hg, ho in zip(res["history"], ores.history):
        assert abs(hg["relres"] - ho["relres"]) <= (1e-5 if prec == "fp64" else 1e-3) * ho["relres"]


@pytest.mark.parametrize("r2", ["0", "1"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_greedy_lockstep_pcg_barrier_forms(monkeypatch, r2, prec, tol):
    """The PCG with three grid barriers per iteration everywhere
    (CONNREG_PCG_R2=0) and with two in every eligible system, the v-systems'
    low-rank term included (=1; the default takes two in the u-systems only),
    in lockstep with the oracle on the ragged box at the default bars."""
    monkeypatch.setenv("CONNREG_PCG_R2", r2)
    d = mid_box()
    P = oop.problem_from_arrays(d)
    R = 8
    ores = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(
        max_rank=R, als_fixed_sweeps=3, galerkin="dense", seed=5, u_method="dense",
        v_method="dense"))
    g = connreg.Problem(d, prec, DEV)
    res = g.greedy_solve(max_rank=R, als_fixed_sweeps=3, pcg_rtol=1e-13, pcg_maxit=20000,
                         galerkin_rtol=1e-13, galerkin_maxit=20000, seed=5)
    g.close()
    assert res["rank"] == R
    U, V, Z = np_(res["U"]), np_(res["V"]), np_(res["Z"])
    err = _wdiff(U, Z, V, ores.U, ores.Z, ores.V)
    assert err <= tol, err
    for hg, ho in zip(res["history"], ores.history):
        assert abs(hg["relres"] - ho["relres"]) <= (1e-5 if prec == "fp64" else 1e-3) * ho["relres"]


def test_greedy_full_rank_exact():
    d = synth.box_problem(box_y=(4, 3, 3), box_x=(4, 3, 3), offset=(0, 0, 0), n_inj=5, sigma=1.0,
                          hole_r=1.0, wt_rank=3, wt_w=(1.5, 3.0), lam=5.0, seed=2)
    P = oop.problem_from_arrays(d)
    Wstar = odense.solve_kron(P)
    g = connreg.Problem(d, "fp64", DEV)
    res = g.greedy_solve(max_rank=36, pcg_rtol=1e-14, pcg_maxit=20000, galerkin_rtol=1e-14,
                         galerkin_maxit=100000)
    W = np_(res["U"]) @ np_(res["Z"]) @ np_(res["V"]).T
    assert res["rank"] == 36
    assert rel(W, Wstar) < 1e-8


def test_greedy_resume_matches_uninterrupted():
    d = synth.config1()
    g = connreg.Problem(d, "fp64", DEV)
    o = dict(als_fixed_sweeps=2, pcg_rtol=1e-13, galerkin_rtol=1e-13, seed=1)
    full = g.greedy_solve(max_rank=6, **o)
    half = g.greedy_solve(max_rank=3, **o)
    rest = g.greedy_solve(max_rank=6, resume=(half["U"], half["Z"], half["V"]), **o)
    a = [np_(full[k]) for k in ("U", "Z", "V")]
    b = [np_(rest[k]) for k in ("U", "Z", "V")]
    assert rest["rank"] == 6
    assert _wdiff(b[0], b[1], b[2], a[0], a[1], a[2]) < 1e-8


def test_greedy_stops_on_residual():
    d = synth.config1()
    g = connreg.Problem(d, "fp64", DEV)
    res = g.greedy_solve(max_rank=20, tau_res=3e-2)
    assert res["status"] == "ok"
    assert res["history"][-1]["relres"] <= 3e-2
    assert all(h["relres"] > 3e-2 for h in res["history"][:-1])


def test_invalid_arguments_are_rejected():
    d = synth.config1()
    g = connreg.Problem(d, "fp64", DEV)
    with pytest.raises(connreg.ConnRegError):
        g.greedy_solve(max_rank=0)
    bad = dict(d)
    bad["Ly_val"] = d["Ly_val"] * 2.0  # not a graph Laplacian
    with pytest.raises(connreg.ConnRegError):
        connreg.Problem(bad, "fp64", DEV)


# ------------------------------------------------------------------ masked Grams
@pytest.mark.parametrize("r", [1, 17, 70])
def test_masked_gram_fp64_and_bf16(case, r):
    name, d, P = case
    r = min(r, P.n_x)
    rng = np.random.default_rng(31 + r)
    U = rand_orth(rng, P.n_y, r)
    g = connreg.Problem(d, "fp64", DEV)
    ref = np.stack([U.T @ (P.Omega[:, a][:, None] * U) for a in range(P.n_inj)])
    G64 = np_(g.masked_gram(U, "fp64"))
    assert rel(G64, ref) < 1e-13
    Gbf = np_(g.masked_gram(U, "bf16"))
    # entry bound: 2^-8 ||U_a|| ||U_b|| (orthonormal columns: 2^-8) + FP32 accumulation
    assert np.abs(Gbf - ref).max() <= 2.0 ** -8 + 1e-5


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-7), ("mixed", 1e-4)])
def test_warm_started_sweeps_match_cold_starts(monkeypatch, prec, tol):
    """ALS sweeps after the first start each PCG from the previous sweep's
    solution; the tolerance stays relative to the original right-hand side, so
    the factors agree with cold starts to the inner tolerance, in fewer
    iterations."""
    d = mid_box()
    out = {}
    for warm in ("0", "1"):
        monkeypatch.setenv("CONNREG_PCG_WARM", warm)
        g = connreg.Problem(d, prec, DEV)
        out[warm] = g.greedy_solve(max_rank=6, als_fixed_sweeps=3, pcg_rtol=1e-10,
                                   pcg_maxit=20000, galerkin_rtol=1e-13, seed=3)
        g.close()
    c, w = out["0"], out["1"]
    assert c["rank"] == w["rank"] == 6
    err = _wdiff(np_(w["U"]), np_(w["Z"]), np_(w["V"]), np_(c["U"]), np_(c["Z"]), np_(c["V"]))
    assert err <= tol, err
    assert w["stats"]["pcg_iters"] < c["stats"]["pcg_iters"]


@pytest.mark.parametrize("xbs", ["256", "512"])
def test_fp32_register_rows_up_to_128_injections(monkeypatch, xbs):
    """Mixed precision with 64 < n_inj <= 128: the v-system PCG keeps 128 FP32
    rows of X in registers (256- or 512-thread groups); lockstep with the
    oracle at the mixed-precision bar."""
    d = mid_box(seed=8, n_inj=100)
    P = oop.problem_from_arrays(d)
    R = 6
    ores = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(
        max_rank=R, als_fixed_sweeps=3, galerkin="dense", seed=5, u_method="dense",
        v_method="dense"))
    monkeypatch.setenv("CONNREG_PCG_XBS", xbs)
    g = connreg.Problem(d, "mixed", DEV)
    res = g.greedy_solve(max_rank=R, als_fixed_sweeps=3, pcg_rtol=1e-13, pcg_maxit=20000,
                         galerkin_rtol=1e-13, galerkin_maxit=20000, seed=5)
    g.close()
    assert res["rank"] == R
    err = _wdiff(np_(res["U"]), np_(res["Z"]), np_(res["V"]), ores.U, ores.Z, ores.V)
    assert err <= 1e-4, err
