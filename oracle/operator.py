"""Problem data, objective, operator and residual (FP64 oracle; test
infrastructure only, see the package docstring).

Notation follows the paper: W is n_y x n_x, X is n_x x n_inj, Y and Omega
are n_y x n_inj with Omega = 1 on observed entries, L_x and L_y are the
graph Laplacians of the source and target voxel graphs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Problem:
    Ly: sp.csr_matrix
    Lx: sp.csr_matrix
    X: np.ndarray       # n_x x n_inj
    Y: np.ndarray       # n_y x n_inj
    Omega: np.ndarray   # n_y x n_inj, float 0/1
    lam: float

    @property
    def n_y(self):
        return self.Ly.shape[0]

    @property
    def n_x(self):
        return self.Lx.shape[0]

    @property
    def n_inj(self):
        return self.X.shape[1]

    @property
    def OY(self):
        """Omega o Y, the only part of Y that enters the problem."""
        return self.Omega * self.Y


def problem_from_arrays(d: dict, lam: float | None = None) -> Problem:
    """Wrap generator arrays (CSR Laplacians, X, Y, Omega) as a Problem."""
    ny = d["Ly_rowptr"].size - 1
    nx = d["Lx_rowptr"].size - 1
    Ly = sp.csr_matrix((d["Ly_val"], d["Ly_colidx"], d["Ly_rowptr"]), shape=(ny, ny))
    Lx = sp.csr_matrix((d["Lx_val"], d["Lx_colidx"], d["Lx_rowptr"]), shape=(nx, nx))
    return Problem(Ly=Ly, Lx=Lx, X=np.asarray(d["X"], np.float64),
                   Y=np.asarray(d["Y"], np.float64),
                   Omega=np.asarray(d["Omega"], np.float64),
                   lam=float(d["lam"] if lam is None else lam))


# ---------------------------------------------------------------------------
# Objective (eq. obj_fun):  J(W) = 1/2 ||P_Omega(W X - Y)||_F^2
#                                 + lambda/2 ||L_y W + W L_x^T||_F^2
# ---------------------------------------------------------------------------
def objective(P: Problem, W: np.ndarray) -> float:
    loss = 0.5 * np.sum((P.Omega * (W @ P.X - P.Y)) ** 2)
    reg = 0.5 * P.lam * np.sum((P.Ly @ W + (P.Lx @ W.T).T) ** 2)
    return float(loss + reg)


# ---------------------------------------------------------------------------
# Operator form (eq. multitermSylv): A(W) = lambda B(W) + C(W),
#   B(W) = W L_x^2 + 2 L_y W L_x + L_y^2 W,
#   C(W) = sum_alpha diag(Omega_alpha) W X_alpha X_alpha^T,
#   D    = (Omega o Y) X^T.
# ---------------------------------------------------------------------------
def apply_B(P: Problem, W: np.ndarray) -> np.ndarray:
    Lx2W_T = P.Lx @ (P.Lx @ W.T)            # (W L_x^2)^T, L_x symmetric
    LyW = P.Ly @ W
    LyWLx = (P.Lx @ LyW.T).T
    return Lx2W_T.T + 2.0 * LyWLx + P.Ly @ LyW


def apply_C(P: Problem, W: np.ndarray) -> np.ndarray:
    out = np.zeros_like(W)
    for a in range(P.n_inj):
        xa = P.X[:, a]
        out += P.Omega[:, a][:, None] * np.outer(W @ xa, xa)
    return out


def apply_A(P: Problem, W: np.ndarray) -> np.ndarray:
    """A(W) for a dense W (n_y x n_x)."""
    return P.lam * apply_B(P, W) + apply_C(P, W)


def rhs_D(P: Problem) -> np.ndarray:
    """D = (Omega o Y) X^T, dense n_y x n_x."""
    return P.OY @ P.X.T


def kron_matrix(P: Problem) -> np.ndarray:
    """The (n_y n_x) x (n_y n_x) matrix of eq. system_matrix (vec stacks
    columns):  sum_alpha (X_a X_a^T) kron diag(Omega_a)
             + lambda (L_x^2 kron I + 2 L_x kron L_y + I kron L_y^2)."""
    Lx = P.Lx.toarray()
    Ly = P.Ly.toarray()
    Iy = np.eye(P.n_y)
    Ix = np.eye(P.n_x)
    A = P.lam * (np.kron(Lx @ Lx, Iy) + 2.0 * np.kron(Lx, Ly) + np.kron(Ix, Ly @ Ly))
    for a in range(P.n_inj):
        xa = P.X[:, a]
        A += np.kron(np.outer(xa, xa), np.diag(P.Omega[:, a]))
    return A


def vec(W: np.ndarray) -> np.ndarray:
    return W.reshape(-1, order="F")


def unvec(w: np.ndarray, n_y: int, n_x: int) -> np.ndarray:
    return w.reshape((n_y, n_x), order="F")


# ---------------------------------------------------------------------------
# Factored application A(U Z V^T).  Each term of multitermSylv keeps its
# low-rank structure (L_x symmetric):
#   W L_x^2      = U Z (L_x^2 V)^T
#   L_y W L_x    = (L_y U) Z (L_x V)^T
#   L_y^2 W      = (L_y^2 U) Z V^T
#   C(W)         = sum_a (Omega_a o (U Z V^T x_a)) x_a^T = (Omega o (U Z H)) X^T,
#                  H = V^T X.
# ---------------------------------------------------------------------------
@dataclass
class OpFactors:
    LyU: np.ndarray
    Ly2U: np.ndarray
    LxV: np.ndarray
    Lx2V: np.ndarray
    M: np.ndarray      # Omega o (U Z H), n_y x n_inj


def op_apply(P: Problem, U, Z, V) -> OpFactors:
    LyU = P.Ly @ U
    Ly2U = P.Ly @ LyU
    LxV = P.Lx @ V
    Lx2V = P.Lx @ LxV
    H = V.T @ P.X
    M = P.Omega * (U @ (Z @ H))
    return OpFactors(LyU, Ly2U, LxV, Lx2V, M)


def op_assemble(P: Problem, U, Z, V, f: OpFactors) -> np.ndarray:
    """Dense A(U Z V^T) from the factors (for checks at small sizes)."""
    return (P.lam * (U @ Z @ f.Lx2V.T + 2.0 * f.LyU @ Z @ f.LxV.T + f.Ly2U @ Z @ V.T)
            + f.M @ P.X.T)


def residual_factors(P: Problem, U, Z, V):
    """R = D - A(U Z V^T) = F_R G_R^T with
    F_R = [Omega o (Y - U Z H) | U | L_y U | L_y^2 U],
    G_R = [X | -lambda L_x^2 V Z^T | -2 lambda L_x V Z^T | -lambda V Z^T]."""
    if U.shape[1] == 0:
        return P.OY.copy(), P.X.copy()
    f = op_apply(P, U, Z, V)
    F = np.hstack([P.OY - f.M, U, f.LyU, f.Ly2U])
    G = np.hstack([P.X, -P.lam * f.Lx2V @ Z.T, -2.0 * P.lam * f.LxV @ Z.T,
                   -P.lam * V @ Z.T])
    return F, G
