"""Training and evaluation of the learned u-system preconditioner.

Training pairs come from the solver itself: an FP64 greedy solve of a
problem gives iterates W_j = U_j Z_j V_j^T; at each sampled j the u-system of
eq. ALS_linsys is built (``cr_u_system``) for the basis direction v = V[:, j]
(the ALS direction that rank j + 1 kept) and for a perturbed copy of it, and
solved to 1e-10 with Jacobi-PCG (``cr_u_solve``) for the target.  Training
and inference run in the library's HIP kernels; this module only drives
them.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import connreg


@dataclass
class Pairs:
    b: torch.Tensor      # (m, n_y) right-hand sides
    x: torch.Tensor      # (m, n_y) solutions
    d: torch.Tensor      # (m, n_y) data diagonals
    coef: np.ndarray     # (m, 2)  (c1, c0)
    seconds: float = 0.0

    def __len__(self):
        return int(self.b.shape[0])


def collect_pairs(prob: connreg.Problem, max_rank: int, every: int, perturb: float, seed: int,
                  rtol: float = 1e-10) -> Pairs:
    t0 = time.perf_counter()
    res = prob.greedy_solve(max_rank=max_rank, seed=seed)
    U, V, Z = res["U"], res["V"], res["Z"]
    rng = np.random.default_rng(seed + 12345)
    bs, xs, ds, cs = [], [], [], []
    for j in range(0, res["rank"], every):
        base = V[:, j].detach().clone()
        for k in range(2):
            v = base
            if k:
                noise = torch.tensor(rng.standard_normal(prob.n_x), device=base.device)
                v = base + perturb * noise / noise.norm()
            v = v / v.norm()
            rhs, d, coef = prob.u_system(U[:, :j], Z[:j, :j], V[:, :j], v)
            x = prob.u_solve(d, coef, rhs, rtol=rtol, maxit=50000)[0]
            bs.append(rhs)
            xs.append(x)
            ds.append(d)
            cs.append(coef)
    return Pairs(torch.stack(bs), torch.stack(xs), torch.stack(ds), np.array(cs),
                 time.perf_counter() - t0)


def concat(ps):
    return Pairs(torch.cat([p.b for p in ps]), torch.cat([p.x for p in ps]),
                 torch.cat([p.d for p in ps]), np.concatenate([p.coef for p in ps]),
                 sum(p.seconds for p in ps))


def train(pc: connreg.Pc, prob: connreg.Problem, data: Pairs, steps: int, batch: int = 8,
          lr: float = 2e-3, seed: int = 0, log=None):
    """Adam on random minibatches; returns the loss history."""
    rng = np.random.default_rng(seed)
    hist = []
    m = len(data)
    for s in range(steps):
        idx = rng.choice(m, size=min(batch, m), replace=False)
        it = torch.tensor(idx, device=data.b.device)
        lr_s = lr * (0.1 ** (s / max(1, steps)))  # exponential decay to lr/10
        loss = pc.train_step(prob, data.b[it], data.x[it], data.d[it], data.coef[idx], lr=lr_s)
        hist.append(loss)
        if log and (s % 50 == 0 or s == steps - 1):
            log(f"[lpc] step {s:4d} loss {loss:.4e}")
    return hist


def evaluate(prob: connreg.Problem, data: Pairs, pc: connreg.Pc | None, rtol: float = 1e-8,
             precond: str | None = None):
    """Iterations, seconds and final relative residual per system (precond as
    in Problem.u_solve)."""
    out = []
    for i in range(len(data)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, it, rr, fb, st = prob.u_solve(data.d[i], tuple(data.coef[i]), data.b[i], rtol=rtol,
                                         maxit=50000, pc=pc, precond=precond)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = float((x - data.x[i]).norm() / data.x[i].norm())
        out.append(dict(iters=it, seconds=dt, relres=rr, fallbacks=fb, status=st, err=err))
    return out
