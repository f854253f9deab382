"""Pins of the FP64 oracle against facts fixed outside it: published test
vectors, closed forms, the objective it must differentiate, brute force on
tiny inputs, and invariants the paper states.  CPU only."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from paper_1808_05510_amd import synth
from oracle import als as oals
from oracle import dense as odense
from oracle import galerkin as ogal
from oracle import greedy as ogreedy
from oracle import metrics as omet
from oracle import operator as oop
from oracle import rng as orng
from tests.helpers import rand_orth, rel


# ---------------------------------------------------------------- fixtures
@pytest.fixture(scope="module")
def p1d():
    return oop.problem_from_arrays(synth.config1_small(seed=3))


@pytest.fixture(scope="module")
def p3d_arrays():
    return synth.config2_tiny(seed=1)


@pytest.fixture(scope="module")
def p3d(p3d_arrays):
    return oop.problem_from_arrays(p3d_arrays)


def torch_objective(P, W):
    """J(W) of eq. obj_fun written in torch (differentiated by autograd)."""
    X = torch.tensor(P.X)
    Y = torch.tensor(P.Y)
    Om = torch.tensor(P.Omega)
    Ly = torch.tensor(P.Ly.toarray())
    Lx = torch.tensor(P.Lx.toarray())
    loss = 0.5 * ((Om * (W @ X - Y)) ** 2).sum()
    reg = 0.5 * P.lam * ((Ly @ W + W @ Lx.T) ** 2).sum()
    return loss + reg


def grad_J(P, W):
    Wt = torch.tensor(W, requires_grad=True)
    torch_objective(P, Wt).backward()
    return Wt.grad.numpy()


# ---------------------------------------------------------------- SplitMix64
def test_splitmix64_published_vector(root):
    lines = [l.split() for l in open(os.path.join(root, "tests/golden/splitmix64.txt"))
             if l.strip() and not l.startswith("#")]
    seed = int(lines[0][1])
    want = [int(l[0]) for l in lines[1:]]
    assert orng.splitmix64_sequence(seed, len(want)) == want


def test_uniform_stream_mapping():
    n = 17
    seed, stream = 42, 5
    x = orng.uniform_pm1(seed, stream, n)
    st = (seed ^ ((stream * orng.STREAM_MUL) % (1 << 64))) % (1 << 64)
    ints = orng.splitmix64_sequence(st, n)
    ref = np.array([(z >> 11) * 2.0 ** -52 - 1.0 for z in ints])
    assert np.array_equal(x, ref)
    assert x.min() >= -1.0 and x.max() < 1.0


# ---------------------------------------------------------------- Laplacians
@pytest.mark.parametrize("maker", [synth.config1_small, synth.config2_tiny])
def test_graph_laplacian_properties(maker):
    d = maker()
    for k in ("Ly", "Lx"):
        n = d[k + "_rowptr"].size - 1
        L = sp.csr_matrix((d[k + "_val"], d[k + "_colidx"], d[k + "_rowptr"]), shape=(n, n))
        Ld = L.toarray()
        assert np.array_equal(Ld, Ld.T)
        assert np.allclose(Ld @ np.ones(n), 0.0)
        off = Ld - np.diag(np.diag(Ld))
        assert set(np.unique(off)) <= {0.0, -1.0}
        assert np.array_equal(np.diag(Ld), -off.sum(1))
        # (L^2)_ii = deg_i^2 + deg_i for a unit-weight graph Laplacian
        assert np.allclose(np.diag(Ld @ Ld), np.diag(Ld) ** 2 + np.diag(Ld))


@pytest.mark.parametrize("dims", [(7,), (5, 4), (4, 3, 3)])
def test_box_laplacian_dct_eigenpairs(dims):
    """Path-graph Laplacian eigenpairs are DCT-II (closed form)."""
    coords = synth.box_coords(dims + (1,) * (3 - len(dims)))[:, : len(dims)]
    rp, ci, v = synth.graph_laplacian_csr(coords)
    n = rp.size - 1
    L = sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()
    Q, mu = odense.box_eigen(dims)
    assert np.allclose(Q.T @ Q, np.eye(n), atol=1e-13)
    assert np.allclose(L @ Q, Q * mu[None, :], atol=1e-12)
    assert np.allclose(np.sort(mu), np.linalg.eigvalsh(L), atol=1e-12)


# ---------------------------------------------------------------- operator
def test_gradient_of_objective_is_A_minus_D(p3d):
    """dJ/dW = A(W) - D: pins operator and RHS against eq. obj_fun."""
    rng = np.random.default_rng(0)
    W = rng.standard_normal((p3d.n_y, p3d.n_x))
    g = grad_J(p3d, W)
    assert rel(oop.apply_A(p3d, W) - oop.rhs_D(p3d), g) < 1e-12


def test_gradient_central_difference_1d(p1d):
    rng = np.random.default_rng(1)
    W = rng.standard_normal((p1d.n_y, p1d.n_x))
    E = rng.standard_normal(W.shape)
    h = 1e-4
    fd = (oop.objective(p1d, W + h * E) - oop.objective(p1d, W - h * E)) / (2 * h)
    an = float(np.sum(E * (oop.apply_A(p1d, W) - oop.rhs_D(p1d))))
    assert abs(fd - an) <= 1e-7 * abs(an)


def test_kron_form_equals_operator_form(p3d):
    rng = np.random.default_rng(2)
    W = rng.standard_normal((p3d.n_y, p3d.n_x))
    K = oop.kron_matrix(p3d)
    assert rel(oop.unvec(K @ oop.vec(W), p3d.n_y, p3d.n_x), oop.apply_A(p3d, W)) < 1e-13


def test_operator_symmetric_positive(p3d):
    rng = np.random.default_rng(3)
    P_ = rng.standard_normal((p3d.n_y, 3)) @ rng.standard_normal((3, p3d.n_x))
    Q_ = rng.standard_normal((p3d.n_y, 2)) @ rng.standard_normal((2, p3d.n_x))
    a = np.sum(oop.apply_A(p3d, P_) * Q_)
    b = np.sum(P_ * oop.apply_A(p3d, Q_))
    assert abs(a - b) <= 1e-12 * abs(a)
    assert np.sum(oop.apply_A(p3d, P_) * P_) > 0
    assert np.linalg.eigvalsh(oop.kron_matrix(p3d)).min() > 0


def test_full_mask_compresses_data_term(p3d):
    P1 = oop.Problem(p3d.Ly, p3d.Lx, p3d.X, p3d.Y, np.ones_like(p3d.Omega), p3d.lam)
    rng = np.random.default_rng(4)
    W = rng.standard_normal((p3d.n_y, p3d.n_x))
    assert rel(oop.apply_C(P1, W), W @ p3d.X @ p3d.X.T) < 1e-13


def test_B_is_L_of_L(p3d):
    rng = np.random.default_rng(5)
    W = rng.standard_normal((p3d.n_y, p3d.n_x))
    Ly, Lx = p3d.Ly.toarray(), p3d.Lx.toarray()
    Lop = lambda M: Ly @ M + M @ Lx
    assert rel(oop.apply_B(p3d, W), Lop(Lop(W))) < 1e-13


def test_factored_apply_and_residual(p3d):
    rng = np.random.default_rng(6)
    r = 4
    U = rng.standard_normal((p3d.n_y, r))
    V = rng.standard_normal((p3d.n_x, r))
    Z = rng.standard_normal((r, r))
    W = U @ Z @ V.T
    f = oop.op_apply(p3d, U, Z, V)
    assert rel(oop.op_assemble(p3d, U, Z, V, f), oop.apply_A(p3d, W)) < 1e-13
    F, G = oop.residual_factors(p3d, U, Z, V)
    R = oop.rhs_D(p3d) - oop.apply_A(p3d, W)
    assert rel(F @ G.T, R) < 1e-13
    assert abs(omet.fro_factored(F, G) - np.linalg.norm(R)) <= 1e-12 * np.linalg.norm(R)
    assert abs(omet.d_norm(p3d) - np.linalg.norm(oop.rhs_D(p3d))) <= 1e-13 * omet.d_norm(p3d)


# ---------------------------------------------------------------- exact solves
def test_kron_solution_zeroes_gradient(p3d):
    W = odense.solve_kron(p3d)
    g = grad_J(p3d, W)
    assert np.linalg.norm(g) <= 1e-9 * np.linalg.norm(oop.rhs_D(p3d))


@pytest.mark.parametrize("which", ["1d", "3d"])
def test_full_mask_dct_closed_form_matches_kron(which, p1d, p3d, p3d_arrays):
    if which == "1d":
        P, by, bx = p1d, (40,), (40,)
    else:
        P, by, bx = p3d, tuple(p3d_arrays["box_y"]), tuple(p3d_arrays["box_x"])
    P1 = oop.Problem(P.Ly, P.Lx, P.X, P.Y, np.ones_like(P.Omega), P.lam)
    assert rel(odense.solve_full_mask(P1, by, bx), odense.solve_kron(P1)) < 1e-10


# ---------------------------------------------------------------- ALS systems
def test_als_matrices_are_operator_slices(p3d):
    """A_hat u = A(u v^T) v for unit v; B_hat v = A(u v^T)^T u for unit u."""
    rng = np.random.default_rng(7)
    u = rng.standard_normal(p3d.n_y)
    v = rng.standard_normal(p3d.n_x)
    v /= np.linalg.norm(v)
    Ah = oals.u_matrix(p3d, v)
    assert rel(Ah @ u, oop.apply_A(p3d, np.outer(u, v)) @ v) < 1e-13
    u /= np.linalg.norm(u)
    v = rng.standard_normal(p3d.n_x)
    Bh = oals.v_matrix_dense(p3d, u)
    assert rel(Bh @ v, oop.apply_A(p3d, np.outer(u, v)).T @ u) < 1e-13


def test_u_solution_minimises_rank1_functional(p3d):
    """u_hat is the stationary point of <uv^T, A(uv^T)> - 2 u^T R v."""
    rng = np.random.default_rng(8)
    v = rng.standard_normal(p3d.n_x)
    v /= np.linalg.norm(v)
    R = oop.rhs_D(p3d)
    uh = oals.solve_u(p3d, v, R @ v, method="dense")
    Kt = torch.tensor(oop.kron_matrix(p3d))
    vt = torch.tensor(v)
    ut = torch.tensor(uh, requires_grad=True)
    W = torch.outer(ut, vt)
    w = W.T.reshape(-1)  # column stacking
    f = w @ (Kt @ w) - 2.0 * ut @ (torch.tensor(R) @ vt)
    f.backward()
    assert ut.grad.norm().item() <= 1e-9 * np.linalg.norm(R @ v)


@pytest.mark.parametrize("method", ["direct", "cg"])
def test_u_solvers_agree(p3d, method):
    rng = np.random.default_rng(9)
    v = rng.standard_normal(p3d.n_x)
    v /= np.linalg.norm(v)
    b = rng.standard_normal(p3d.n_y)
    ref = oals.solve_u(p3d, v, b, method="dense")
    assert rel(oals.solve_u(p3d, v, b, method=method), ref) < 1e-9


@pytest.mark.parametrize("method", ["smw", "cg"])
def test_v_solvers_agree(p3d, method):
    rng = np.random.default_rng(10)
    u = rng.standard_normal(p3d.n_y)
    u /= np.linalg.norm(u)
    b = rng.standard_normal(p3d.n_x)
    ref = oals.solve_v(p3d, u, b, method="dense")
    assert rel(oals.solve_v(p3d, u, b, method=method), ref) < 1e-9


def test_als_fixed_point_norms(p1d):
    """At an ALS fixed point ||u_hat|| = ||v_hat||."""
    F, G = oop.residual_factors(p1d, np.zeros((p1d.n_y, 0)), np.zeros((0, 0)),
                                np.zeros((p1d.n_x, 0)))
    v0 = ogreedy.init_v(p1d, F, G, 0, 0)
    a = oals.als(p1d, F, G, v0, fixed_sweeps=60, u_method="dense", v_method="dense")
    assert abs(a.unorm / a.vnorm - 1.0) < 1e-6


# ---------------------------------------------------------------- Galerkin
def test_projected_operator_is_projection(p3d):
    rng = np.random.default_rng(11)
    r = 5
    U = rand_orth(rng, p3d.n_y, r)
    V = rand_orth(rng, p3d.n_x, r)
    Z = rng.standard_normal((r, r))
    pr = ogal.project(p3d, U, V)
    assert rel(ogal.apply_Ap(pr, Z), U.T @ oop.apply_A(p3d, U @ Z @ V.T) @ V) < 1e-13
    assert rel(ogal.rhs(pr), U.T @ oop.rhs_D(p3d) @ V) < 1e-13
    K = ogal.kron_projected(pr)
    assert rel(K @ Z.reshape(-1, order="F"), ogal.apply_Ap(pr, Z).reshape(-1, order="F")) < 1e-13


def test_galerkin_orthogonality_and_cg(p3d):
    rng = np.random.default_rng(12)
    r = 6
    U = rand_orth(rng, p3d.n_y, r)
    V = rand_orth(rng, p3d.n_x, r)
    pr = ogal.project(p3d, U, V)
    Z = ogal.solve_dense(pr)
    R = oop.rhs_D(p3d) - oop.apply_A(p3d, U @ Z @ V.T)
    assert np.linalg.norm(U.T @ R @ V) <= 1e-10 * np.linalg.norm(oop.rhs_D(p3d))
    Zc, it = ogal.solve_cg(pr, np.zeros((r, r)), rtol=1e-13)
    assert rel(Zc, Z) < 1e-9 and it > 0


# ---------------------------------------------------------------- Algorithm 1
@pytest.fixture(scope="module")
def p3d_square():
    """Source box = target box, so rank n spans both spaces completely."""
    return oop.problem_from_arrays(synth.box_problem(
        box_y=(4, 3, 3), box_x=(4, 3, 3), offset=(0, 0, 0), n_inj=5, sigma=1.0,
        hole_r=1.0, wt_rank=3, wt_w=(1.5, 3.0), lam=5.0, seed=2))


@pytest.mark.parametrize("which", ["1d", "3d"])
def test_greedy_full_rank_reaches_exact_solution(which, p1d, p3d_square):
    """With r = n_x = n_y the Galerkin space is the whole space, so the
    Galerkin solution is W* itself."""
    P = p1d if which == "1d" else p3d_square
    Wstar = odense.solve_kron(P)
    r = min(P.n_x, P.n_y)
    res = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=r, u_method="dense",
                                                        v_method="dense", galerkin="dense"))
    assert res.status == "ok" and res.U.shape[1] == r
    assert rel(res.U @ res.Z @ res.V.T, Wstar) < 1e-9
    assert res.history[-1]["relres"] < 1e-9


def test_greedy_energy_monotone_and_consistent(p3d):
    res = ogreedy.greedy_solve(p3d, ogreedy.GreedyOptions(max_rank=12, u_method="dense",
                                                          v_method="dense", galerkin="dense"))
    E = [h["energy"] for h in res.history]
    assert all(E[k + 1] <= E[k] + 1e-12 * abs(E[k]) for k in range(len(E) - 1))
    W = res.U @ res.Z @ res.V.T
    # energy = J(W) - 1/2 ||Omega o Y||^2 (expansion of the quadratic objective)
    J = oop.objective(p3d, W)
    assert abs(E[-1] - (J - 0.5 * np.sum(p3d.OY ** 2))) <= 1e-10 * abs(J)
    # relres and delta W against dense evaluations
    Rd = oop.rhs_D(p3d) - oop.apply_A(p3d, W)
    assert abs(res.history[-1]["relres"] - np.linalg.norm(Rd) / np.linalg.norm(oop.rhs_D(p3d))) < 1e-12
    assert np.allclose(res.U.T @ res.U, np.eye(12), atol=1e-13)


def test_greedy_cg_galerkin_matches_dense(p1d):
    o = dict(max_rank=10, u_method="dense", v_method="dense", als_fixed_sweeps=3)
    a = ogreedy.greedy_solve(p1d, ogreedy.GreedyOptions(galerkin="dense", **o))
    b = ogreedy.greedy_solve(p1d, ogreedy.GreedyOptions(galerkin="cg", galerkin_rtol=1e-13, **o))
    Wa = a.U @ a.Z @ a.V.T
    Wb = b.U @ b.Z @ b.V.T
    assert rel(Wb, Wa) < 1e-8


def test_greedy_direct_paths_match_dense(p3d):
    o = dict(max_rank=6, als_fixed_sweeps=2, galerkin="dense")
    a = ogreedy.greedy_solve(p3d, ogreedy.GreedyOptions(u_method="dense", v_method="dense", **o))
    b = ogreedy.greedy_solve(p3d, ogreedy.GreedyOptions(u_method="direct", v_method="smw", **o))
    assert rel(b.U @ b.Z @ b.V.T, a.U @ a.Z @ a.V.T) < 1e-9


def test_toy_relres_decreases_with_rank():
    P = oop.problem_from_arrays(synth.config1())
    res = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=12, galerkin="dense"))
    rr = [h["relres"] for h in res.history]
    assert rr[-1] < 0.1 * rr[0]
