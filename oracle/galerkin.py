"""Galerkin refinement (FP64 oracle; test infrastructure only).

With U, V spanning the greedy bases, the Galerkin condition gives the
projected equation eq. Proj_Sylv for the j x j core Z:
    lambda (Z (V^T L_x^2 V) + 2 (U^T L_y U) Z (V^T L_x V) + (U^T L_y^2 U) Z)
    + sum_alpha (U^T diag(Omega_alpha) U) Z (V^T X_alpha X_alpha^T V)
    = U^T D V.
Since V^T X_alpha X_alpha^T V = h_alpha h_alpha^T with h_alpha = V^T X_alpha,
the data term is sum_alpha G_alpha Z h_alpha h_alpha^T, and U^T D V = S H^T
with S = U^T (Omega o Y), H = V^T X.  The paper solves it with a
matrix-valued CG warm-started from the previous core.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .operator import Problem


@dataclass
class Projected:
    G: np.ndarray     # n_inj x r x r, G[a] = U^T diag(Omega_a) U
    H: np.ndarray     # r x n_inj
    By1: np.ndarray   # U^T L_y U
    By2: np.ndarray   # U^T L_y^2 U
    Bx1: np.ndarray   # V^T L_x V
    Bx2: np.ndarray   # V^T L_x^2 V
    S: np.ndarray     # r x n_inj
    lam: float


def project(P: Problem, U, V) -> Projected:
    G = np.stack([U.T @ (P.Omega[:, a][:, None] * U) for a in range(P.n_inj)])
    LyU = P.Ly @ U
    LxV = P.Lx @ V
    return Projected(G=G, H=V.T @ P.X, By1=U.T @ LyU, By2=U.T @ (P.Ly @ LyU),
                     Bx1=V.T @ LxV, Bx2=V.T @ (P.Lx @ LxV), S=U.T @ P.OY, lam=P.lam)


def rhs(pr: Projected) -> np.ndarray:
    return pr.S @ pr.H.T


def apply_Ap(pr: Projected, Z) -> np.ndarray:
    out = pr.lam * (Z @ pr.Bx2 + 2.0 * pr.By1 @ Z @ pr.Bx1 + pr.By2 @ Z)
    ZH = Z @ pr.H
    for a in range(pr.H.shape[1]):
        out += np.outer(pr.G[a] @ ZH[:, a], pr.H[:, a])
    return out


def kron_projected(pr: Projected) -> np.ndarray:
    """The r^2 x r^2 matrix of Z -> A_p(Z) (vec stacks columns)."""
    r = pr.H.shape[0]
    I = np.eye(r)
    K = pr.lam * (np.kron(pr.Bx2.T, I) + 2.0 * np.kron(pr.Bx1.T, pr.By1) + np.kron(I, pr.By2))
    for a in range(pr.H.shape[1]):
        h = pr.H[:, a]
        K += np.kron(np.outer(h, h), pr.G[a])
    return K


def solve_dense(pr: Projected) -> np.ndarray:
    r = pr.H.shape[0]
    K = kron_projected(pr)
    z = sla.solve(K, rhs(pr).reshape(-1, order="F"), assume_a="pos")
    return z.reshape((r, r), order="F")


def solve_cg(pr: Projected, Z0, rtol=1e-12, maxit=None):
    """Matrix-valued CG on A_p(Z) = S H^T from Z0.  Stops when
    ||S H^T - A_p(Z)||_F <= rtol ||S H^T||_F.  Returns (Z, iterations)."""
    r = pr.H.shape[0]
    if maxit is None:
        maxit = max(10 * r * r, 100)
    B = rhs(pr)
    bn = np.linalg.norm(B)
    Z = Z0.copy()
    if bn == 0.0:
        return np.zeros_like(Z), 0
    R = B - apply_Ap(pr, Z)
    rr = float(np.sum(R * R))
    Pd = R.copy()
    it = 0
    while np.sqrt(rr) > rtol * bn and it < maxit:
        Q = apply_Ap(pr, Pd)
        alpha = rr / float(np.sum(Pd * Q))
        Z += alpha * Pd
        R -= alpha * Q
        rr_new = float(np.sum(R * R))
        Pd = R + (rr_new / rr) * Pd
        rr = rr_new
        it += 1
    return Z, it
