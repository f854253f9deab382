"""Exact solutions (FP64 oracle; test infrastructure only).

* ``solve_kron``: W* from a dense Cholesky factorisation of the Kronecker
  matrix of eq. system_matrix (tiny problems only: the matrix has
  (n_y n_x)^2 entries).
* ``dct_basis`` / ``box_eigen``: the eigenpairs of the graph Laplacian of a
  path (Neumann ends) are the DCT-II vectors cos(pi k (i + 1/2) / n) with
  eigenvalues 2 - 2 cos(pi k / n); a box's Laplacian is the Kronecker sum
  over its axes, so its eigenvectors are tensor products of these.
* ``solve_full_mask``: with Omega = 1 the data term compresses to
  C(W) = W X X^T (remark after eq. system_matrix); in the eigenbases of
  L_y and L_x the regulariser B(W) = L(L(W)) is diagonal, so each target
  mode i solves the n_x x n_x system
      w_i (lambda diag((mu_i + nu_k)^2) + Xt Xt^T) = d_i,  Xt = Q_x^T X.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .operator import Problem, kron_matrix, rhs_D, unvec, vec


def solve_kron(P: Problem) -> np.ndarray:
    """W* (n_y x n_x) by Cholesky of the Kronecker system."""
    A = kron_matrix(P)
    c = sla.cho_factor(A, lower=True)
    return unvec(sla.cho_solve(c, vec(rhs_D(P))), P.n_y, P.n_x)


def dct_basis(n: int):
    """Orthonormal eigenvectors (columns) and eigenvalues of the path-graph
    Laplacian with n vertices."""
    i = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    Q = np.cos(np.pi * k * (i + 0.5) / n)
    Q /= np.linalg.norm(Q, axis=0, keepdims=True)
    mu = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
    return Q, mu


def box_eigen(dims):
    """Eigenvectors / eigenvalues of the graph Laplacian of a full box whose
    voxels are numbered with the first axis fastest."""
    Q = np.ones((1, 1))
    mu = np.zeros(1)
    for n in dims:
        Qd, md = dct_basis(int(n))
        # new axis is slower than all previous ones
        Q = np.kron(Qd, Q)
        mu = (md[:, None] + mu[None, :]).reshape(-1)
    return Q, mu


def solve_full_mask(P: Problem, box_y, box_x) -> np.ndarray:
    """W* for Omega = 1 on full boxes (mask values in P are ignored)."""
    Qy, mu = box_eigen([d for d in box_y if d > 0])
    Qx, nu = box_eigen([d for d in box_x if d > 0])
    D = P.Y @ P.X.T                      # Omega = 1
    Dt = Qy.T @ D @ Qx
    Xt = Qx.T @ P.X
    XX = Xt @ Xt.T
    Wt = np.empty_like(Dt)
    for i in range(P.n_y):
        Ai = P.lam * np.diag((mu[i] + nu) ** 2) + XX
        Wt[i] = np.linalg.solve(Ai, Dt[i])   # Ai symmetric
    return Qy @ Wt @ Qx.T
