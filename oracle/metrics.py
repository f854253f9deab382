"""Factored Frobenius norms and the paper's error measures (FP64 oracle;
test infrastructure only).

A product F G^T is never formed: ||F G^T||_F = ||R_F R_G^T||_F with thin QR
factors F = Q_F R_F and G = Q_G R_G.
"""
from __future__ import annotations

import numpy as np

from .operator import Problem, residual_factors


def fro_factored(F: np.ndarray, G: np.ndarray) -> float:
    """||F G^T||_F for tall F (n_y x k) and G (n_x x k)."""
    if F.shape[1] == 0:
        return 0.0
    rf = np.linalg.qr(F, mode="r")
    rg = np.linalg.qr(G, mode="r")
    return float(np.linalg.norm(rf @ rg.T))


def d_norm(P: Problem) -> float:
    """||D||_F = ||(Omega o Y) X^T||_F."""
    return fro_factored(P.OY, P.X)


def residual_norm(P: Problem, U, Z, V):
    """(||D - A(U Z V^T)||_F, relative value) -- the relative residual used
    as the outer stopping test."""
    F, G = residual_factors(P, U, Z, V)
    r = fro_factored(F, G)
    return r, r / d_norm(P)


def diff_norm(U1, Z1, V1, U2, Z2, V2) -> float:
    """||U1 Z1 V1^T - U2 Z2 V2^T||_F in factored form."""
    F = np.hstack([U1 @ Z1, -U2 @ Z2])
    G = np.hstack([V1, V2])
    return fro_factored(F, G)


def low_rank_norm(U, Z, V) -> float:
    return fro_factored(U @ Z, V)


def rms_error(U, Z, V, Ws_F, Ws_G, n_y, n_x):
    """E(W_r, W_*) = ||W_r - W_*||_F / sqrt(n_y n_x) and
    E_rel = ||W_r - W_*||_F / ||W_*||_F (section on the test problems),
    with W_* = Ws_F Ws_G^T given in factored form."""
    F = np.hstack([U @ Z, -Ws_F])
    G = np.hstack([V, Ws_G])
    d = fro_factored(F, G)
    return d / np.sqrt(n_y * n_x), d / fro_factored(Ws_F, Ws_G)


def energy(P: Problem, U, Z, V) -> float:
    """1/2 <W, A(W)> - <W, D> for W = U Z V^T (the A-norm error functional
    minimised by the greedy step, up to the constant 1/2 ||W*||_A^2)."""
    from .operator import op_apply
    f = op_apply(P, U, Z, V)
    # <W, A(W)> = tr(V Z^T U^T A(W)) evaluated through the factors
    UtAW = (P.lam * ((U.T @ U) @ Z @ (f.Lx2V.T @ V) + 2.0 * (U.T @ f.LyU) @ Z @ (f.LxV.T @ V)
                     + (U.T @ f.Ly2U) @ Z @ (V.T @ V))
            + (U.T @ f.M) @ (P.X.T @ V))
    WAW = float(np.sum(Z * UtAW))
    WD = float(np.sum(Z * ((U.T @ P.OY) @ (P.X.T @ V))))
    return 0.5 * WAW - WD
