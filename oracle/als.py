"""ALS half-steps of the greedy rank-1 update (FP64 oracle; test
infrastructure only).

For a fixed unit v the minimiser u-hat of eq. minuv2 solves eq. ALS_linsys
    A_hat u = R_j v,
    A_hat = lambda ((v^T L_x^2 v) I + 2 (v^T L_x v) L_y + L_y^2)
            + sum_alpha diag(Omega_alpha) (v^T X_alpha)^2,
and for a fixed unit u the minimiser v-hat solves eq. ALS_linsys_v
    B_hat v = R_j^T u,
    B_hat = lambda (L_x^2 + 2 (u^T L_y u) L_x + (u^T L_y^2 u) I)
            + sum_alpha (u^T diag(Omega_alpha) u) X_alpha X_alpha^T.
The paper solves the first with a sparse direct solver and the second with
Sherman-Morrison-Woodbury around a sparse direct solve of the Laplacian
part; both are here, plus dense solves for tiny sizes and Jacobi-CG.
The residual R_j is given in factored form R_j = F G^T.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import Problem


# ---- coefficients ---------------------------------------------------------
def u_coeffs(P: Problem, v):
    """(a, b, d): a = v^T L_x^2 v, b = v^T L_x v, d_i = sum_a Omega_ia (v^T X_a)^2."""
    Lxv = P.Lx @ v
    a = float(Lxv @ Lxv)
    b = float(v @ Lxv)
    h = P.X.T @ v
    d = P.Omega @ (h * h)
    return a, b, d


def v_coeffs(P: Problem, u):
    """(c, e, g): c = u^T L_y u, e = u^T L_y^2 u, g_a = u^T diag(Omega_a) u."""
    Lyu = P.Ly @ u
    c = float(u @ Lyu)
    e = float(Lyu @ Lyu)
    g = P.Omega.T @ (u * u)
    return c, e, g


def u_matrix(P: Problem, v) -> sp.csr_matrix:
    a, b, d = u_coeffs(P, v)
    Iy = sp.identity(P.n_y, format="csr")
    return (P.lam * (a * Iy + 2.0 * b * P.Ly + P.Ly @ P.Ly) + sp.diags(d)).tocsr()


def v_matrix_sparse(P: Problem, c, e) -> sp.csr_matrix:
    """The Laplacian part lambda (L_x^2 + 2 c L_x + e I) of B_hat."""
    Ix = sp.identity(P.n_x, format="csr")
    return (P.lam * (P.Lx @ P.Lx + 2.0 * c * P.Lx + e * Ix)).tocsr()


def v_matrix_dense(P: Problem, u) -> np.ndarray:
    c, e, g = v_coeffs(P, u)
    S = v_matrix_sparse(P, c, e).toarray()
    return S + (P.X * g[None, :]) @ P.X.T


# ---- solvers --------------------------------------------------------------
def _jacobi_cg(matvec, diag, rhs, rtol, maxit):
    n = rhs.size
    Aop = spla.LinearOperator((n, n), matvec=matvec, dtype=np.float64)
    M = spla.LinearOperator((n, n), matvec=lambda r: r / diag, dtype=np.float64)
    x, info = spla.cg(Aop, rhs, rtol=rtol, atol=0.0, maxiter=maxit, M=M)
    return x


def solve_u(P: Problem, v, rhs, method="direct", rtol=1e-12, maxit=20000):
    A = u_matrix(P, v)
    if method == "dense":
        return sla.solve(A.toarray(), rhs, assume_a="pos")
    if method == "direct":
        return spla.splu(A.tocsc()).solve(rhs)
    if method == "cg":
        return _jacobi_cg(lambda p: A @ p, A.diagonal(), rhs, rtol, maxit)
    raise ValueError(method)


def solve_v(P: Problem, u, rhs, method="smw", rtol=1e-12, maxit=20000):
    c, e, g = v_coeffs(P, u)
    if method == "dense":
        return sla.solve(v_matrix_dense(P, u), rhs, assume_a="pos")
    if method == "smw":
        # B_hat = S + (X G^1/2)(X G^1/2)^T: Sherman-Morrison-Woodbury with a
        # sparse LU of S; the square root form needs no inverse of g.
        S = v_matrix_sparse(P, c, e)
        lu = spla.splu(S.tocsc())
        Xg = P.X * np.sqrt(np.maximum(g, 0.0))[None, :]
        SiXg = lu.solve(Xg)
        Sib = lu.solve(rhs)
        K = np.eye(P.n_inj) + Xg.T @ SiXg
        return Sib - SiXg @ np.linalg.solve(K, Xg.T @ Sib)
    if method == "cg":
        S = v_matrix_sparse(P, c, e)
        diag = S.diagonal() + (P.X * P.X) @ g
        return _jacobi_cg(lambda p: S @ p + P.X @ (g * (P.X.T @ p)), diag, rhs, rtol, maxit)
    raise ValueError(method)


# ---- one rank-1 ALS update -------------------------------------------------
@dataclass
class ALSResult:
    u: np.ndarray
    v: np.ndarray
    unorm: float
    vnorm: float
    sweeps: int
    delta: float


def als(P: Problem, F, G, v0, delta_tol=0.1, max_sweeps=10, fixed_sweeps=0,
        u_method="direct", v_method="smw", rtol=1e-12) -> ALSResult:
    """ALS loop of Algorithm 1 for the residual R_j = F G^T, starting from
    the unit vector v0.  Stops when |  ||u_hat|| / ||v_hat|| - 1 | <= delta_tol
    (at least one sweep, at most ``max_sweeps``), or after exactly
    ``fixed_sweeps`` sweeps when that is positive."""
    v = v0 / np.linalg.norm(v0)
    sweeps = 0
    delta = np.inf
    while True:
        uh = solve_u(P, v, F @ (G.T @ v), method=u_method, rtol=rtol)
        un = float(np.linalg.norm(uh))
        u = uh / un
        vh = solve_v(P, u, G @ (F.T @ u), method=v_method, rtol=rtol)
        vn = float(np.linalg.norm(vh))
        v = vh / vn
        delta = abs(un / vn - 1.0)
        sweeps += 1
        if fixed_sweeps > 0:
            if sweeps >= fixed_sweeps:
                break
        elif delta <= delta_tol or sweeps >= max_sweeps:
            break
    return ALSResult(u, v, un, vn, sweeps, delta)
