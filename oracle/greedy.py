"""Algorithm 1: greedy rank-1 method with Galerkin projection (FP64 oracle;
test infrastructure only).

Steps per greedy iteration j, in the paper's order:
  1. pick a unit initial vector v (left open by the paper; here
     v = R_j^T q / ||R_j^T q|| with q from SplitMix64 stream j);
  2. ALS sweeps on eqs. ALS_linsys / ALS_linsys_v while
     delta = | ||u_hat|| / ||v_hat|| - 1 | > 0.1;
  3. U_{j+1} = orth([U_j, u]), V_{j+1} = orth([V_j, v]) (here: classical
     Gram-Schmidt applied twice, appending a column);
  4. j <- j + 1 and solve eq. Proj_Sylv for Z_j (CG to tau/2, or a dense
     solve), warm-started from the previous core padded with zeros;
  5. R_j = D - A(U_j Z_j V_j^T) in factored form;
  6. delta W = ||U_j Z_j V_j^T - U_{j-1} Z_{j-1} V_{j-1}^T||_F / ||U_j Z_j V_j^T||_F;
repeat until j = max rank, delta W <= tau, or (added stopping test) the
relative residual ||R_j||_F / ||D||_F <= tau_res.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import galerkin, rng
from .als import als
from .metrics import d_norm, diff_norm, energy, fro_factored, low_rank_norm
from .operator import Problem, residual_factors


@dataclass
class GreedyOptions:
    max_rank: int = 20
    tau_dW: float = 0.0          # Algorithm 1's tau on delta W (0 = off)
    tau_res: float = 0.0         # relative residual stop (0 = off)
    als_delta: float = 0.1
    als_max_sweeps: int = 10
    als_fixed_sweeps: int = 0    # > 0: exactly this many sweeps per rank
    u_method: str = "direct"
    v_method: str = "smw"
    inner_rtol: float = 1e-12
    galerkin: str = "dense"      # "dense" or "cg"
    galerkin_rtol: float | None = None   # default: tau / 2
    seed: int = 0
    orth_tol: float = 1e-10


@dataclass
class GreedyResult:
    U: np.ndarray
    V: np.ndarray
    Z: np.ndarray
    history: list = field(default_factory=list)
    status: str = "ok"


def init_v(P: Problem, F, G, j: int, seed: int) -> np.ndarray:
    q = rng.uniform_pm1(seed, j, P.n_y)
    w = G @ (F.T @ q)
    return w / np.linalg.norm(w)


def cgs2_append(B: np.ndarray, w: np.ndarray, tol: float):
    """Append w to the orthonormal columns of B after two classical
    Gram-Schmidt passes; None when w is (numerically) in span(B)."""
    x = w.copy()
    for _ in range(2):
        x -= B @ (B.T @ x)
    nrm = float(np.linalg.norm(x))
    if nrm <= tol * float(np.linalg.norm(w)):
        return None
    return np.hstack([B, (x / nrm)[:, None]])


def greedy_solve(P: Problem, opt: GreedyOptions) -> GreedyResult:
    U = np.zeros((P.n_y, 0))
    V = np.zeros((P.n_x, 0))
    Z = np.zeros((0, 0))
    F, G = residual_factors(P, U, Z, V)
    dn = d_norm(P)
    tau = opt.tau_res if opt.tau_res > 0 else opt.tau_dW
    g_rtol = opt.galerkin_rtol if opt.galerkin_rtol is not None else max(tau, 1e-14) / 2
    res = GreedyResult(U, V, Z)
    t_start = time.perf_counter()
    for j in range(opt.max_rank):
        v0 = init_v(P, F, G, j, opt.seed)
        a = als(P, F, G, v0, opt.als_delta, opt.als_max_sweeps, opt.als_fixed_sweeps,
                opt.u_method, opt.v_method, opt.inner_rtol)
        Un = cgs2_append(U, a.u, opt.orth_tol)
        Vn = cgs2_append(V, a.v, opt.orth_tol)
        if Un is None or Vn is None:
            res.status = "breakdown"
            break
        pr = galerkin.project(P, Un, Vn)
        Z0 = np.zeros((j + 1, j + 1))
        Z0[:j, :j] = Z
        if opt.galerkin == "dense":
            Zn, git = galerkin.solve_dense(pr), 0
        else:
            Zn, git = galerkin.solve_cg(pr, Z0, rtol=g_rtol)
        dW = diff_norm(Un, Zn, Vn, U, Z, V) / low_rank_norm(Un, Zn, Vn)
        U, V, Z = Un, Vn, Zn
        F, G = residual_factors(P, U, Z, V)
        rel = fro_factored(F, G) / dn
        res.history.append(dict(rank=j + 1, relres=rel, dW=dW, energy=energy(P, U, Z, V),
                                sweeps=a.sweeps, als_delta=a.delta, galerkin_iters=git,
                                unorm=a.unorm, vnorm=a.vnorm,
                                seconds=time.perf_counter() - t_start))
        res.U, res.V, res.Z = U, V, Z
        if (opt.tau_res > 0 and rel <= opt.tau_res) or (opt.tau_dW > 0 and dW <= opt.tau_dW):
            break
    return res
