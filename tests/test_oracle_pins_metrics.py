"""Pins of the oracle's factored norms, error measures and stopping rules
against dense evaluations of their definitions and against a brute-force
ALS written from the operator itself.  CPU only.

Each pin is chosen so that a sign, transpose or off-by-one mistake in the
pinned function fails it: non-symmetric cores, unequal ranks, factors that
are not orthonormal, and stopping indices that are neither the first nor
the last step."""
import numpy as np
import pytest

from paper_1808_05510_amd import synth
from oracle import als as oals
from oracle import greedy as ogreedy
from oracle import metrics as omet
from oracle import operator as oop


@pytest.fixture(scope="module")
def p3d():
    return oop.problem_from_arrays(synth.config2_tiny(seed=1))


@pytest.fixture(scope="module")
def p1d():
    return oop.problem_from_arrays(synth.config1_small(seed=3))


def _factors(rng, n_y, n_x, r):
    return (rng.standard_normal((n_y, r)), rng.standard_normal((r, r)),
            rng.standard_normal((n_x, r)))


@pytest.mark.parametrize("r1,r2", [(3, 5), (4, 0), (0, 2), (6, 6)])
def test_diff_norm_is_dense_frobenius_difference(r1, r2):
    """||U1 Z1 V1^T - U2 Z2 V2^T||_F (non-orthonormal factors, non-symmetric
    cores, unequal ranks)."""
    rng = np.random.default_rng(100 + r1 * 7 + r2)
    U1, Z1, V1 = _factors(rng, 23, 17, r1)
    U2, Z2, V2 = _factors(rng, 23, 17, r2)
    want = np.linalg.norm(U1 @ Z1 @ V1.T - U2 @ Z2 @ V2.T)
    got = omet.diff_norm(U1, Z1, V1, U2, Z2, V2)
    assert abs(got - want) <= 1e-13 * want
    # the pin separates the mistakes it is meant to catch
    if r1 and r2:
        assert abs(np.linalg.norm(U1 @ Z1 @ V1.T + U2 @ Z2 @ V2.T) - want) > 1e-6 * want
        assert abs(np.linalg.norm(U1 @ Z1.T @ V1.T - U2 @ Z2 @ V2.T) - want) > 1e-6 * want


@pytest.mark.parametrize("r", [0, 1, 5])
def test_low_rank_norm_is_dense_frobenius(r):
    rng = np.random.default_rng(200 + r)
    U, Z, V = _factors(rng, 19, 31, r)
    want = np.linalg.norm(U @ Z @ V.T)
    assert abs(omet.low_rank_norm(U, Z, V) - want) <= 1e-13 * max(want, 1e-300)
    assert omet.fro_factored(np.zeros((4, 0)), np.zeros((3, 0))) == 0.0


def test_rms_error_is_dense_E_and_Erel():
    """E(W_r, W_*) = ||W_r - W_*||_F / sqrt(n_y n_x) and
    E_rel = ||W_r - W_*||_F / ||W_*||_F (section on the test problems), with
    W_* given as a factor pair of its own rank."""
    rng = np.random.default_rng(300)
    n_y, n_x = 27, 14
    U, Z, V = _factors(rng, n_y, n_x, 4)
    Fs = rng.standard_normal((n_y, 3))
    Gs = rng.standard_normal((n_x, 3))
    Wr = U @ Z @ V.T
    Ws = Fs @ Gs.T
    E, Erel = omet.rms_error(U, Z, V, Fs, Gs, n_y, n_x)
    d = np.linalg.norm(Wr - Ws)
    assert abs(E - d / np.sqrt(n_y * n_x)) <= 1e-13 * E
    assert abs(Erel - d / np.linalg.norm(Ws)) <= 1e-13 * Erel
    # W_r = W_* gives zero error
    E0, Erel0 = omet.rms_error(Fs, np.eye(3), Gs, Fs, Gs, n_y, n_x)
    assert E0 <= 1e-13 * np.linalg.norm(Ws) and Erel0 <= 1e-13


def test_residual_norm_is_dense(p3d):
    rng = np.random.default_rng(301)
    U, Z, V = _factors(rng, p3d.n_y, p3d.n_x, 3)
    R = oop.rhs_D(p3d) - oop.apply_A(p3d, U @ Z @ V.T)
    a, b = omet.residual_norm(p3d, U, Z, V)
    assert abs(a - np.linalg.norm(R)) <= 1e-12 * a
    assert abs(b - np.linalg.norm(R) / np.linalg.norm(oop.rhs_D(p3d))) <= 1e-12 * b


def _prefix_runs(P, J, **kw):
    """W_j for j = 1..J from runs capped at rank j (Algorithm 1 is
    deterministic, so run j is the first j steps of run J)."""
    out = []
    for j in range(1, J + 1):
        r = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(max_rank=j, **kw))
        out.append(r.U @ r.Z @ r.V.T)
    return out


def test_greedy_dW_is_dense_difference_of_iterates(p3d):
    """delta W_j = ||W_j - W_{j-1}||_F / ||W_j||_F (Algorithm 1), with W_0 = 0."""
    kw = dict(u_method="dense", v_method="dense", galerkin="dense", als_fixed_sweeps=2)
    J = 5
    res = ogreedy.greedy_solve(p3d, ogreedy.GreedyOptions(max_rank=J, **kw))
    Ws = _prefix_runs(p3d, J, **kw)
    assert np.allclose(Ws[-1], res.U @ res.Z @ res.V.T, rtol=0, atol=1e-12 * np.abs(Ws[-1]).max())
    prev = np.zeros_like(Ws[0])
    for j, W in enumerate(Ws):
        want = np.linalg.norm(W - prev) / np.linalg.norm(W)
        assert abs(res.history[j]["dW"] - want) <= 1e-9 * want, j
        prev = W
    assert res.history[0]["dW"] == pytest.approx(1.0, abs=1e-12)


def test_greedy_stops_at_first_rank_with_small_dW(p3d):
    """The tau stop of Algorithm 1: the run ends at the first rank whose
    delta W is at most tau (here a threshold between two later ranks)."""
    kw = dict(u_method="dense", v_method="dense", galerkin="dense", als_fixed_sweeps=2)
    full = ogreedy.greedy_solve(p3d, ogreedy.GreedyOptions(max_rank=10, **kw))
    dW = np.array([h["dW"] for h in full.history])
    # a tau that the sequence first meets at rank j0 >= 3 (not the first or last rank)
    j0 = next(j for j in range(2, len(dW) - 1) if dW[j] < dW[:j].min())
    tau = 0.5 * (dW[j0] + dW[:j0].min())
    res = ogreedy.greedy_solve(p3d, ogreedy.GreedyOptions(max_rank=10, tau_dW=tau, **kw))
    assert len(res.history) == j0 + 1
    assert res.history[-1]["dW"] <= tau < min(h["dW"] for h in res.history[:-1])


def test_greedy_stops_at_first_rank_with_small_relres(p1d):
    kw = dict(u_method="dense", v_method="dense", galerkin="dense", als_fixed_sweeps=2)
    full = ogreedy.greedy_solve(p1d, ogreedy.GreedyOptions(max_rank=8, **kw))
    rr = np.array([h["relres"] for h in full.history])
    tau = 0.5 * (rr[4] + rr[5]) if rr[5] < rr[4] else None
    assert tau is not None and np.all(rr[:5] > tau)
    res = ogreedy.greedy_solve(p1d, ogreedy.GreedyOptions(max_rank=8, tau_res=tau, **kw))
    assert len(res.history) == 6


def _brute_force_als(P, F, G, v0, delta_tol, max_sweeps):
    """The ALS loop written from the Kronecker matrix: A_hat and B_hat are
    (v kron I)^T K (v kron I) and (I kron u)^T K (I kron u), the right-hand
    sides R v and R^T u with R = F G^T formed densely.  Returns the sequence
    of | ||u_hat|| / ||v_hat|| - 1 |."""
    K = oop.kron_matrix(P)
    R = F @ G.T
    Iy, Ix = np.eye(P.n_y), np.eye(P.n_x)
    v = v0 / np.linalg.norm(v0)
    deltas = []
    for _ in range(max_sweeps):
        Mv = np.kron(v[:, None], Iy)        # vec(u v^T) = (v kron I) u
        uh = np.linalg.solve(Mv.T @ K @ Mv, R @ v)
        u = uh / np.linalg.norm(uh)
        Mu = np.kron(Ix, u[:, None])        # vec(u v^T) = (I kron u) v
        vh = np.linalg.solve(Mu.T @ K @ Mu, R.T @ u)
        v = vh / np.linalg.norm(vh)
        deltas.append(abs(np.linalg.norm(uh) / np.linalg.norm(vh) - 1.0))
        if deltas[-1] <= delta_tol:
            break
    return deltas


@pytest.mark.parametrize("j,delta_tol", [(0, 0.1), (2, 0.1), (1, 0.02)])
def test_adaptive_als_stops_at_first_small_delta(p3d, j, delta_tol):
    """Algorithm 1's ALS stop: sweeps continue while delta > tol and end at
    the first sweep whose delta is at most tol (at least one sweep)."""
    kw = dict(u_method="dense", v_method="dense", galerkin="dense", als_fixed_sweeps=2)
    base = ogreedy.greedy_solve(p3d, ogreedy.GreedyOptions(max_rank=j, **kw)) if j else None
    U = base.U if base else np.zeros((p3d.n_y, 0))
    V = base.V if base else np.zeros((p3d.n_x, 0))
    Z = base.Z if base else np.zeros((0, 0))
    F, G = oop.residual_factors(p3d, U, Z, V)
    v0 = ogreedy.init_v(p3d, F, G, j, 0)
    deltas = _brute_force_als(p3d, F, G, v0, delta_tol, 10)
    a = oals.als(p3d, F, G, v0, delta_tol=delta_tol, max_sweeps=10, u_method="dense",
                 v_method="dense")
    assert a.sweeps == len(deltas)
    assert a.delta == pytest.approx(deltas[-1], rel=1e-8, abs=1e-12)
    assert all(d > delta_tol for d in deltas[:-1])


def test_adaptive_als_sweep_cap(p3d):
    F, G = oop.residual_factors(p3d, np.zeros((p3d.n_y, 0)), np.zeros((0, 0)),
                                np.zeros((p3d.n_x, 0)))
    v0 = ogreedy.init_v(p3d, F, G, 0, 0)
    a = oals.als(p3d, F, G, v0, delta_tol=0.0, max_sweeps=3, u_method="dense", v_method="dense")
    assert a.sweeps == 3
