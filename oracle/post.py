"""Post-processing of a greedy solution W = U Z V^T (FP64 oracle; test
infrastructure only).

* ``core_svd``: the SVD of the solution from the SVD of its small core
  (section on the top-view results: Z is not diagonal, so with
  Z = Zu diag(s) Zv^T, W = (U Zu) diag(s) (V Zv)^T is the SVD of W when U
  and V have orthonormal columns);
* ``objective_factored``: the objective of eq. obj_fun, J(W) =
  1/2 ||P_Omega(W X - Y)||_F^2 + lambda/2 ||L_y W + W L_x^T||_F^2, for a
  factored W (the cost-against-rank curves of the real-data sections);
* ``entry_stats``: statistics of the entries of a low-rank W = A B^T
  (section on dropping the nonnegativity constraint: the count and size of
  the negative entries, and the distance to the projection max(0, W)),
  computed block by block over every entry.
"""
from __future__ import annotations

import numpy as np

from .metrics import fro_factored
from .operator import Problem


def core_svd(U, Z, V):
    """(Uh, s, Vh) with W = U Z V^T = Uh diag(s) Vh^T, s descending."""
    Zu, s, Zvt = np.linalg.svd(Z)
    return U @ Zu, s, V @ Zvt.T


def objective_factored(P: Problem, U, Z, V):
    """(J, misfit, regulariser) of eq. obj_fun for W = U Z V^T, each term in
    factored form: P_Omega(W X - Y) = Omega o (U Z (V^T X)) - Omega o Y
    (n_y x n_inj), and L_y W + W L_x^T = [L_y U, U] [V Z^T, L_x V Z^T]^T."""
    H = V.T @ P.X
    M = P.Omega * (U @ (Z @ H)) - P.OY
    misfit = 0.5 * float(np.sum(M * M))
    F = np.hstack([P.Ly @ U, U])
    G = np.hstack([V @ Z.T, (P.Lx @ V) @ Z.T])
    reg = 0.5 * P.lam * fro_factored(F, G) ** 2
    return misfit + reg, misfit, reg


STAT_KEYS = ("count_neg", "min", "max", "max_abs", "sum_sq", "sum_sq_neg")


def entry_stats(A, B, block=4096):
    """Statistics over every entry w of W = A B^T: number of negative
    entries, min, max, max |w|, sum w^2 (= ||W||_F^2) and sum of w^2 over the
    negative entries (= ||W - max(0, W)||_F^2)."""
    out = dict(count_neg=0.0, min=np.inf, max=-np.inf, max_abs=0.0, sum_sq=0.0, sum_sq_neg=0.0)
    for i0 in range(0, A.shape[0], block):
        W = A[i0:i0 + block] @ B.T
        neg = W < 0
        out["count_neg"] += float(np.count_nonzero(neg))
        out["min"] = min(out["min"], float(W.min()))
        out["max"] = max(out["max"], float(W.max()))
        out["max_abs"] = max(out["max_abs"], float(np.abs(W).max()))
        out["sum_sq"] += float(np.sum(W * W))
        out["sum_sq_neg"] += float(np.sum(W[neg] ** 2))
    return out
