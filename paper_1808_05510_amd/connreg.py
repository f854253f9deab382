"""Python binding of libconnreg (ctypes).  Argument marshalling only: every
step of the solver runs in the HIP library; torch supplies device memory and
the stream.  Loading fails loudly when the library has not been built.

Matrices cross the boundary column-major: a column-major n x k matrix is a
torch tensor of shape (n, k) with strides (1, ld).  ``colmajor`` makes one.
"""
from __future__ import annotations

import atexit
import ctypes
import json
import math
import os
import weakref
from ctypes import POINTER, c_double, c_int32, c_int64, c_uint64, c_void_p

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libconnreg.so")

CR_OK, CR_EINVAL, CR_ENOMEM, CR_EHIP, CR_ENONFINITE = 0, -1, -2, -3, -4
CR_NOTCONV, CR_BREAKDOWN, CR_PC_FALLBACK = 1, 2, 3
STATUS_NAMES = {0: "ok", -1: "einval", -2: "enomem", -3: "ehip", -4: "enonfinite",
                1: "notconv", 2: "breakdown", 3: "pc_fallback"}
PREC = {"fp64": 0, "mixed": 1}

EXPORTS = ["cr_problem_create", "cr_problem_destroy", "cr_rhs_norm", "cr_op_apply",
           "cr_op_apply_f32", "cr_op_apply_factors",
           "cr_op_apply_noalloc", "cr_core_svd", "cr_objective", "cr_entry_stats",
           "cr_problem_set_coarse", "cr_solve_opts_default", "cr_als_step", "cr_galerkin_project",
           "cr_residual_norm", "cr_greedy_solve", "cr_last_error", "cr_version",
           "cr_u_system", "cr_u_solve", "cr_problem_set_pc", "cr_pc_create", "cr_pc_destroy",
           "cr_pc_num_params", "cr_pc_get_params", "cr_pc_set_params", "cr_pc_forward",
           "cr_pc_vjp", "cr_pc_train_step", "cr_masked_gram", "cr_greedy_solve_batch",
           "cr_autotune_pcg", "cr_problem_set_tuning", "cr_problem_set_precond",
           "cr_problem_set_box"]


class CSR(ctypes.Structure):
    _fields_ = [("n", c_int64), ("rowptr", c_void_p), ("colidx", c_void_p), ("val", c_void_p)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("Ly", CSR), ("Lx", CSR), ("n_inj", c_int64),
                ("X", c_void_p), ("ldx", c_int64), ("Y", c_void_p), ("ldy", c_int64),
                ("Omega", c_void_p), ("ldo", c_int64), ("lambda_", c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("max_rank", c_int32), ("tau_dW", c_double), ("tau_res", c_double),
                ("als_delta", c_double), ("als_max_sweeps", c_int32),
                ("als_fixed_sweeps", c_int32), ("pcg_rtol", c_double), ("pcg_maxit", c_int32),
                ("galerkin_rtol", c_double), ("galerkin_maxit", c_int32), ("seed", c_uint64),
                ("orth_tol", c_double), ("pcg_vpt", c_int32), ("verbose", c_int32)]


class ALSStats(ctypes.Structure):
    _fields_ = [("sweeps", c_int32), ("delta", c_double), ("unorm", c_double),
                ("vnorm", c_double), ("pcg_iters_u", c_int32), ("pcg_iters_v", c_int32),
                ("pcg_notconv", c_int32)]


class RankInfo(ctypes.Structure):
    _fields_ = [("rank", c_int32), ("relres", c_double), ("dW", c_double), ("energy", c_double),
                ("sweeps", c_int32), ("pcg_iters", c_int32), ("galerkin_iters", c_int32),
                ("seconds", c_double), ("J", c_double)]


class EntryStats(ctypes.Structure):
    _fields_ = [("entries", c_double), ("count_neg", c_double), ("min", c_double),
                ("max", c_double), ("max_abs", c_double), ("sum_sq", c_double),
                ("sum_sq_neg", c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("rank", c_int32), ("relres", c_double), ("dW", c_double),
                ("pcg_iters", c_int64), ("galerkin_iters", c_int64), ("pcg_notconv", c_int32),
                ("seconds", c_double)]


RANK_CB = ctypes.CFUNCTYPE(None, POINTER(RankInfo), c_void_p)

_lib = None
# every open Problem / Pc handle; closed by an exit hook registered when the
# library is loaded (after torch's, so it runs before them: exit hooks run in
# reverse order), so that no handle is destroyed from a finaliser while the
# interpreter, torch or the HIP runtime are being torn down
_live = weakref.WeakSet()


def close_all():
    """Destroy every open handle (networks after the problems that use them)."""
    objs = list(_live)
    for o in objs:
        if isinstance(o, Problem):
            o.close()
    for o in objs:
        o.close()


def load(path: str = LIB_PATH):
    """Load libconnreg.so (raises when it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m "
                           "paper_1808_05510_amd.build (hipcc, gfx950); there is no CPU fallback")
    L = ctypes.CDLL(path)
    P = c_void_p
    L.cr_problem_create.argtypes = [POINTER(ProblemDesc), ctypes.c_int, P, POINTER(P)]
    L.cr_problem_destroy.argtypes = [P]
    L.cr_problem_destroy.restype = None
    L.cr_rhs_norm.argtypes = [P, POINTER(c_double)]
    L.cr_op_apply.argtypes = [P, c_int64, P, c_int64, P, c_int64, P, c_int64, P, c_int64, P,
                              c_int64]
    L.cr_op_apply_f32.argtypes = L.cr_op_apply.argtypes
    L.cr_op_apply_factors.argtypes = L.cr_op_apply.argtypes
    L.cr_op_apply_noalloc.argtypes = L.cr_op_apply.argtypes
    L.cr_core_svd.argtypes = [P, c_int64, P, c_int64, P, c_int64, P, c_int64, P, c_int64, P, P,
                              c_int64, POINTER(c_int32)]
    L.cr_objective.argtypes = [P, c_int64, P, c_int64, P, c_int64, P, c_int64, POINTER(c_double)]
    L.cr_entry_stats.argtypes = [P, c_int64, P, c_int64, P, c_int64, P, c_int64,
                                 POINTER(EntryStats)]
    L.cr_solve_opts_default.argtypes = [POINTER(SolveOpts)]
    L.cr_solve_opts_default.restype = None
    L.cr_als_step.argtypes = [P, c_int64, P, c_int64, P, c_int64, P, c_int64, P, P,
                              POINTER(SolveOpts), POINTER(ALSStats)]
    L.cr_galerkin_project.argtypes = [P, c_int64, P, c_int64, P, c_int64, P, c_int64, c_double,
                                      c_int32, POINTER(c_int32)]
    L.cr_residual_norm.argtypes = [P, c_int64, P, c_int64, P, c_int64, P, c_int64,
                                   POINTER(c_double), POINTER(c_double)]
    L.cr_greedy_solve.argtypes = [P, POINTER(SolveOpts), P, P, P, POINTER(c_int64),
                                  POINTER(SolveStats), RANK_CB, P]
    L.cr_u_system.argtypes = [P, c_int64, P, c_int64, P, c_int64, P, c_int64, P, P, P,
                              POINTER(c_double)]
    L.cr_u_solve.argtypes = [P, P, POINTER(c_double), P, P, c_double, c_int32, c_int32, P,
                             POINTER(c_int32), POINTER(c_double), POINTER(c_int32)]
    L.cr_problem_set_pc.argtypes = [P, P]
    L.cr_problem_set_precond.argtypes = [P, c_int32]
    L.cr_problem_set_box.argtypes = [P, c_int32, POINTER(c_int32)]
    L.cr_problem_set_coarse.argtypes = [P, c_int32, P, c_int32, c_int32]
    L.cr_pc_create.argtypes = [c_int32, c_int32, c_int32, c_int32, c_uint64, P, POINTER(P)]
    L.cr_pc_destroy.argtypes = [P]
    L.cr_pc_destroy.restype = None
    L.cr_pc_num_params.argtypes = [P]
    L.cr_pc_num_params.restype = c_int64
    L.cr_pc_get_params.argtypes = [P, P]
    L.cr_pc_set_params.argtypes = [P, P]
    L.cr_pc_forward.argtypes = [P, P, P]
    L.cr_pc_vjp.argtypes = [P, P, P, P]
    L.cr_pc_train_step.argtypes = [P, P, c_int32, P, P, P, POINTER(c_double), ctypes.c_float,
                                   POINTER(c_double)]
    L.cr_masked_gram.argtypes = [P, c_int64, P, c_int64, c_int32, P, c_int64]
    L.cr_greedy_solve_batch.argtypes = [c_int32, POINTER(P), POINTER(SolveOpts), POINTER(P),
                                        POINTER(P), POINTER(P), POINTER(c_int64),
                                        POINTER(SolveStats), POINTER(c_int32)]
    L.cr_autotune_pcg.argtypes = [P, c_int32, POINTER(c_int32), POINTER(c_int32),
                                  POINTER(c_double), POINTER(c_double)]
    L.cr_problem_set_tuning.argtypes = [P, c_int32, c_int32]
    L.cr_last_error.restype = ctypes.c_char_p
    L.cr_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("cr_problem_destroy", "cr_solve_opts_default", "cr_last_error",
                        "cr_version", "cr_pc_destroy", "cr_pc_num_params"):
            L[name].restype = ctypes.c_int
    _lib = L
    atexit.register(close_all)
    return L


class ConnRegError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status):
    if status < 0:
        raise ConnRegError(status, load().cr_last_error().decode())
    return status


def colmajor(a, device="cuda:0", dtype=torch.float64) -> torch.Tensor:
    """(n, k) tensor with column-major storage (strides (1, n))."""
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    a = np.asarray(a)
    if a.ndim == 1:
        a = a[:, None]
    return torch.tensor(np.ascontiguousarray(a.T)).to(device=device, dtype=dtype).T


def empty_colmajor(n, k, device="cuda:0", dtype=torch.float64) -> torch.Tensor:
    return torch.empty((k, n), device=device, dtype=dtype).T


def zeros_colmajor(n, k, device="cuda:0", dtype=torch.float64) -> torch.Tensor:
    return torch.zeros((k, n), device=device, dtype=dtype).T


def _ld(t: torch.Tensor) -> int:
    if t.dim() == 1 or t.shape[1] == 0:
        return max(t.shape[0], 1)
    if t.stride(0) != 1 and t.shape[0] > 1:
        raise ValueError("matrix must be column-major (stride(0) == 1)")
    return max(t.stride(1), t.shape[0]) if t.shape[1] > 1 else t.shape[0]


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load().cr_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Problem:
    """A problem handle on one device (see include/connreg.h)."""

    def __init__(self, data: dict, precision: str = "fp64", device: str = "cuda:0",
                 lam: float | None = None, stream: torch.cuda.Stream | None = None):
        L = load()
        self.device = torch.device(device)
        self.precision = precision
        with torch.cuda.device(self.device):
            self.stream = stream or torch.cuda.current_stream(self.device)
        self._host = {}
        for k in ("Ly", "Lx"):
            self._host[k] = (np.ascontiguousarray(data[k + "_rowptr"], np.int32),
                             np.ascontiguousarray(data[k + "_colidx"], np.int32),
                             np.ascontiguousarray(data[k + "_val"], np.float64))
        self.n_y = self._host["Ly"][0].size - 1
        self.n_x = self._host["Lx"][0].size - 1
        self.n_inj = int(np.asarray(data["X"]).shape[1])
        self.lam = float(data["lam"] if lam is None else lam)
        X = colmajor(data["X"], self.device)
        Y = colmajor(data["Y"], self.device)
        Om = colmajor(np.asarray(data["Omega"], np.uint8), self.device, torch.uint8)

        def csr(k):
            rp, ci, v = self._host[k]
            return CSR(rp.size - 1, rp.ctypes.data, ci.ctypes.data, v.ctypes.data)

        d = ProblemDesc(csr("Ly"), csr("Lx"), self.n_inj, X.data_ptr(), _ld(X), Y.data_ptr(),
                        _ld(Y), Om.data_ptr(), _ld(Om), self.lam)
        h = c_void_p()
        torch.cuda.synchronize(self.device)
        _check(L.cr_problem_create(ctypes.byref(d), PREC[precision],
                                   c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self._dtype = torch.float64
        _live.add(self)

    # -------------------------------------------------------------- helpers
    def close(self):
        if getattr(self, "h", None):
            torch.cuda.synchronize(self.device)
            load().cr_problem_destroy(self.h)
            self.h = None
        _live.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _col(self, a, dtype=torch.float64):
        if isinstance(a, torch.Tensor) and a.device == self.device and a.dtype == dtype and \
                (a.dim() == 1 or a.stride(0) == 1):
            return a
        return colmajor(a, self.device, dtype)

    def rhs_norm(self) -> float:
        out = c_double()
        _check(load().cr_rhs_norm(self.h, ctypes.byref(out)))
        return out.value

    # -------------------------------------------------------------- entry points
    def op_apply(self, U, Z, V, fp32: bool = False, out=None, noalloc: bool = False):
        """Returns (F, G) with F = [L_y U | L_y^2 U | Omega o (U Z H)] and
        G = [L_x V | L_x^2 V] (column-major device tensors).  out: (F, G)
        to write into; noalloc: the allocation-free entry point (FP64)."""
        dt = torch.float32 if fp32 else torch.float64
        r = int(U.shape[1])
        U, Z, V = self._col(U, dt), self._col(Z, dt), self._col(V, dt)
        if out is None:
            F = empty_colmajor(self.n_y, 2 * r + self.n_inj, self.device, dt)
            G = empty_colmajor(self.n_x, max(2 * r, 1), self.device, dt)
        else:
            F, G = out
        if noalloc:
            assert not fp32
            fn = load().cr_op_apply_noalloc
        else:
            fn = load().cr_op_apply_f32 if fp32 else load().cr_op_apply
        _check(fn(self.h, r, _ptr(U), _ld(U), _ptr(Z), max(_ld(Z), 1), _ptr(V), _ld(V),
                  _ptr(F), _ld(F), _ptr(G), _ld(G)))
        return F, G[:, : 2 * r]

    def op_apply_factors(self, U, Z, V):
        """Returns (F, G), n_y x k and n_x x k with k = 3r + n_inj and
        F G^T = A(U Z V^T) (column-major FP64 device tensors)."""
        r = int(U.shape[1])
        U, Z, V = self._col(U), self._col(Z), self._col(V)
        k = 3 * r + self.n_inj
        F = empty_colmajor(self.n_y, k, self.device)
        G = empty_colmajor(self.n_x, k, self.device)
        _check(load().cr_op_apply_factors(self.h, r, _ptr(U), _ld(U), _ptr(Z), max(_ld(Z), 1),
                                          _ptr(V), _ld(V), _ptr(F), _ld(F), _ptr(G), _ld(G)))
        return F, G

    def core_svd(self, U, Z, V):
        """SVD of W = U Z V^T from its core: returns (Uh, s, Vh, sweeps, status)
        with W = Uh diag(s) Vh^T (device tensors, s descending)."""
        r = int(U.shape[1])
        U, Z, V = self._col(U), self._col(Z), self._col(V)
        Uh = empty_colmajor(self.n_y, r, self.device)
        Vh = empty_colmajor(self.n_x, r, self.device)
        sv = torch.empty(r, device=self.device, dtype=torch.float64)
        sw = c_int32()
        st = _check(load().cr_core_svd(self.h, r, _ptr(U), _ld(U), _ptr(Z), max(_ld(Z), 1),
                                       _ptr(V), _ld(V), _ptr(Uh), _ld(Uh), _ptr(sv), _ptr(Vh),
                                       _ld(Vh), ctypes.byref(sw)))
        return Uh, sv, Vh, sw.value, STATUS_NAMES[st]

    def objective(self, U, Z, V):
        """(J, misfit, regulariser) of eq. obj_fun at W = U Z V^T (FP64)."""
        r = int(U.shape[1])
        U, Z, V = self._col(U), self._col(Z), self._col(V)
        out = (c_double * 3)()
        _check(load().cr_objective(self.h, r, _ptr(U), _ld(U), _ptr(Z), max(_ld(Z), 1), _ptr(V),
                                   _ld(V), out))
        return out[0], out[1], out[2]

    def entry_stats(self, U, Z, V):
        """Statistics over every entry of W = U Z V^T (dict)."""
        r = int(U.shape[1])
        U, Z, V = self._col(U), self._col(Z), self._col(V)
        es = EntryStats()
        _check(load().cr_entry_stats(self.h, r, _ptr(U), _ld(U), _ptr(Z), max(_ld(Z), 1),
                                     _ptr(V), _ld(V), ctypes.byref(es)))
        return {f: getattr(es, f) for f, _ in EntryStats._fields_}

    def als_step(self, U, Z, V, v0, **opts):
        r = int(U.shape[1])
        U, Z, V = self._col(U), self._col(Z), self._col(V)
        v = self._col(v0).reshape(-1).clone()
        u = torch.empty(self.n_y, device=self.device, dtype=torch.float64)
        o = default_opts(**opts)
        st = ALSStats()
        s = _check(load().cr_als_step(self.h, r, _ptr(U), _ld(U), _ptr(Z), max(_ld(Z), 1),
                                      _ptr(V), _ld(V), _ptr(v), _ptr(u), ctypes.byref(o),
                                      ctypes.byref(st)))
        stats = {f: getattr(st, f) for f, _ in ALSStats._fields_}
        stats["status"] = STATUS_NAMES[s]
        return u, v, stats

    def galerkin_project(self, U, V, Z0=None, rtol=1e-12, maxit=0):
        r = int(U.shape[1])
        U, V = self._col(U), self._col(V)
        Z = zeros_colmajor(r, r, self.device) if Z0 is None else self._col(Z0).clone()
        it = c_int32()
        s = _check(load().cr_galerkin_project(self.h, r, _ptr(U), _ld(U), _ptr(V), _ld(V),
                                              _ptr(Z), _ld(Z), rtol, maxit, ctypes.byref(it)))
        return Z, it.value, STATUS_NAMES[s]

    def residual_norm(self, U, Z, V):
        r = int(U.shape[1])
        U, Z, V = self._col(U), self._col(Z), self._col(V)
        a, b = c_double(), c_double()
        _check(load().cr_residual_norm(self.h, r, _ptr(U), _ld(U), _ptr(Z), max(_ld(Z), 1),
                                       _ptr(V), _ld(V), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def masked_gram(self, U, mode="fp64"):
        """G (n_inj, r, r) float64 device tensor, G[a] = U^T diag(Omega_a) U."""
        r = int(U.shape[1])
        U = self._col(U)
        G = torch.zeros((self.n_inj, r, r), device=self.device, dtype=torch.float64)
        _check(load().cr_masked_gram(self.h, r, _ptr(U), _ld(U), {"fp64": 0, "bf16": 1}[mode],
                                     _ptr(G), r))
        torch.cuda.synchronize(self.device)
        return G.transpose(1, 2)  # column-major blocks -> [a][row][col]

    def u_system(self, U, Z, V, v):
        """The u-system of eq. ALS_linsys at W = U Z V^T for unit v:
        returns (rhs, d, coef) with coef = (c1, c0) on the host."""
        r = int(U.shape[1])
        U, Z, V = self._col(U), self._col(Z), self._col(V)
        v = self._col(v).reshape(-1).contiguous()
        rhs = torch.empty(self.n_y, device=self.device, dtype=torch.float64)
        d = torch.empty(self.n_y, device=self.device, dtype=torch.float64)
        coef = (c_double * 2)()
        _check(load().cr_u_system(self.h, r, _ptr(U), _ld(U), _ptr(Z), max(_ld(Z), 1), _ptr(V),
                                  _ld(V), _ptr(v), _ptr(rhs), _ptr(d), coef))
        return rhs, d, (coef[0], coef[1])

    PRECOND = {"jacobi": 0, "base": 1, "learned": 2}

    def u_solve(self, d, coef, rhs, rtol=1e-8, maxit=5000, pc=None, precond=None):
        """Solve the u-system.  precond: "jacobi" (persistent Jacobi-PCG),
        "base" (flexible CG with the base step: spectral on a declared box,
        else Jacobi) or "learned" (base step refined by the network pc);
        default "learned" when pc is given, else "jacobi".
        Returns (x, iters, relres, fallbacks, status)."""
        kind = self.PRECOND[precond or ("learned" if pc is not None else "jacobi")]
        d = self._col(d).reshape(-1).contiguous()
        rhs = self._col(rhs).reshape(-1).contiguous()
        x = torch.empty(self.n_y, device=self.device, dtype=torch.float64)
        cf = (c_double * 2)(*coef)
        it, rr, fb = c_int32(), c_double(), c_int32()
        s = _check(load().cr_u_solve(self.h, _ptr(d), cf, _ptr(rhs), _ptr(x), rtol, maxit, kind,
                                     pc.h if pc is not None else None, ctypes.byref(it),
                                     ctypes.byref(rr), ctypes.byref(fb)))
        return x, it.value, rr.value, fb.value, STATUS_NAMES[s]

    def set_box(self, dims, which="target"):
        """Declare the target or source grid a full box (first axis fastest)."""
        w = {"target": 0, "source": 1}[which]
        _check(load().cr_problem_set_box(self.h, w, (c_int32 * 3)(*[int(v) for v in dims])))

    def set_coarse(self, coords, block):
        """Two-level preconditioner for the v-systems: aggregates = cubes of
        `block` voxels per axis of the source voxel coordinates (n_x x dim);
        block <= 0 switches it off."""
        c = np.ascontiguousarray(np.asarray(coords), dtype=np.int32)
        if c.ndim == 1:
            c = c[:, None]
        _check(load().cr_problem_set_coarse(self.h, 1, c.ctypes.data, int(c.shape[1]),
                                            int(block)))

    def set_precond(self, kind):
        """u-system preconditioner of the greedy solve: "jacobi", "base" or "learned"."""
        _check(load().cr_problem_set_precond(self.h, self.PRECOND[kind]))

    def set_pc(self, pc):
        _check(load().cr_problem_set_pc(self.h, pc.h if pc is not None else None))
        self._pc = pc

    def autotune(self, cu_share=0):
        """Pick the PCG voxels per thread by timing; returns (vpt_u, vpt_v, us_u, us_v)."""
        vu, vv, tu, tv = c_int32(), c_int32(), c_double(), c_double()
        _check(load().cr_autotune_pcg(self.h, cu_share, ctypes.byref(vu), ctypes.byref(vv),
                                      ctypes.byref(tu), ctypes.byref(tv)))
        return vu.value, vv.value, tu.value, tv.value

    def set_tuning(self, vpt_u, vpt_v):
        _check(load().cr_problem_set_tuning(self.h, vpt_u, vpt_v))

    def greedy_solve(self, resume=None, **opts):
        """Algorithm 1.  Returns dict(U, V, Z, rank, stats, history, status)."""
        o = default_opts(**opts)
        R = int(o.max_rank)
        U = zeros_colmajor(self.n_y, R, self.device)
        V = zeros_colmajor(self.n_x, R, self.device)
        Z = zeros_colmajor(R, R, self.device)
        rank = c_int64(0)
        if resume is not None:
            U0, Z0, V0 = resume
            r0 = int(U0.shape[1])
            U[:, :r0] = self._col(U0)
            V[:, :r0] = self._col(V0)
            Z[:r0, :r0] = self._col(Z0)
            rank.value = r0
        hist = []

        def cb(info, user):
            i = info.contents
            hist.append({f: getattr(i, f) for f, _ in RankInfo._fields_})

        cbf = RANK_CB(cb)
        st = SolveStats()
        torch.cuda.synchronize(self.device)
        s = _check(load().cr_greedy_solve(self.h, ctypes.byref(o), _ptr(U), _ptr(V), _ptr(Z),
                                          ctypes.byref(rank), ctypes.byref(st), cbf, None))
        r = rank.value
        stats = {f: getattr(st, f) for f, _ in SolveStats._fields_}
        return dict(U=U[:, :r], V=V[:, :r], Z=Z[:r, :r], rank=r, stats=stats, history=hist,
                    status=STATUS_NAMES[s])


class Pc:
    """Learned preconditioner network for the u-systems on a box grid."""

    def __init__(self, dims, channels=8, seed=0, device="cuda:0"):
        self.device = torch.device(device)
        self.dims = tuple(int(x) for x in dims)
        self.channels = channels
        with torch.cuda.device(self.device):
            st = torch.cuda.current_stream(self.device)
        h = c_void_p()
        _check(load().cr_pc_create(*self.dims, channels, seed, c_void_p(st.cuda_stream),
                                   ctypes.byref(h)))
        self.h = h
        self.n = int(np.prod(self.dims))
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            torch.cuda.synchronize(self.device)
            load().cr_pc_destroy(self.h)
            self.h = None
        _live.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self):
        return int(load().cr_pc_num_params(self.h))

    def get_params(self):
        out = np.empty(self.num_params(), np.float32)
        _check(load().cr_pc_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, w):
        w = np.ascontiguousarray(w, np.float32)
        assert w.size == self.num_params()
        _check(load().cr_pc_set_params(self.h, w.ctypes.data))

    def forward(self, inp):
        """inp: (4, N) float32 -> y (N,) float32 (device tensors)."""
        inp = torch.as_tensor(inp, device=self.device, dtype=torch.float32).contiguous()
        y = torch.empty(self.n, device=self.device, dtype=torch.float32)
        torch.cuda.synchronize(self.device)
        _check(load().cr_pc_forward(self.h, _ptr(inp), _ptr(y)))
        return y

    def vjp(self, inp, dy):
        inp = torch.as_tensor(inp, device=self.device, dtype=torch.float32).contiguous()
        dy = torch.as_tensor(dy, device=self.device, dtype=torch.float32).contiguous()
        g = np.empty(self.num_params(), np.float32)
        torch.cuda.synchronize(self.device)
        _check(load().cr_pc_vjp(self.h, _ptr(inp), _ptr(dy), g.ctypes.data))
        return g

    def train_step(self, prob, b, x, d, coef, lr=1e-3):
        """One Adam step on a batch: b, x, d (batch, n_y) float64 device tensors,
        coef (batch, 2) host array.  Returns the mean relative squared error."""
        b, x, d = (t.contiguous() for t in (b, x, d))
        coef = np.ascontiguousarray(coef, np.float64)
        loss = c_double()
        torch.cuda.synchronize(self.device)
        _check(load().cr_pc_train_step(self.h, prob.h, int(b.shape[0]), _ptr(b), _ptr(x), _ptr(d),
                                       coef.ctypes.data_as(POINTER(c_double)), lr,
                                       ctypes.byref(loss)))
        return loss.value


class TuningTable:
    """PCG grid shapes (voxels per thread of the u- and v-system grids) by
    problem-size bucket, kept in a JSON file: the first problem of a bucket is
    timed by cr_autotune_pcg, later problems of the bucket reuse the choice.
    A bucket is the precision, n_y and n_x in half-octaves, n_inj rounded up
    to a multiple of 16 and the CU share the grids are limited to."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.table = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    @staticmethod
    def bucket(prob: "Problem", cu_share: int = 0) -> str:
        def half_octave(n):
            return int(round(2 * math.log2(max(int(n), 1))))
        inj = 16 * ((int(prob.n_inj) + 15) // 16)
        return (f"{prob.precision}/ny{half_octave(prob.n_y)}/nx{half_octave(prob.n_x)}"
                f"/inj{inj}/share{int(cu_share)}")

    def apply(self, prob: "Problem", cu_share: int = 0, tune_missing: bool = True):
        """Set the problem's PCG shapes from its bucket (tuning it first when
        the bucket is new and tune_missing); returns the entry or None."""
        key = self.bucket(prob, cu_share)
        if key not in self.table:
            if not tune_missing:
                return None
            vu, vv, tu, tv = prob.autotune(cu_share)
            self.table[key] = dict(vpt_u=int(vu), vpt_v=int(vv), us_per_iter_u=float(tu),
                                   us_per_iter_v=float(tv))
            self.save()
        e = self.table[key]
        prob.set_tuning(int(e["vpt_u"]), int(e["vpt_v"]))
        return e

    def save(self):
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def greedy_solve_batch(problems, opts_list):
    """Algorithm 1 on several problems at once (one handle and stream each).
    Returns a list of dicts like Problem.greedy_solve (without history)."""
    n = len(problems)
    L = load()
    opts = (SolveOpts * n)(*[default_opts(**o) for o in opts_list])
    Us, Vs, Zs = [], [], []
    for p, o in zip(problems, opts):
        R = int(o.max_rank)
        Us.append(zeros_colmajor(p.n_y, R, p.device))
        Vs.append(zeros_colmajor(p.n_x, R, p.device))
        Zs.append(zeros_colmajor(R, R, p.device))
    P = c_void_p
    hs = (P * n)(*[p.h for p in problems])
    up = (P * n)(*[u.data_ptr() for u in Us])
    vp = (P * n)(*[v.data_ptr() for v in Vs])
    zp = (P * n)(*[z.data_ptr() for z in Zs])
    ranks = (c_int64 * n)()
    stats = (SolveStats * n)()
    sts = (c_int32 * n)()
    torch.cuda.synchronize()
    _check(L.cr_greedy_solve_batch(n, hs, opts, up, vp, zp, ranks, stats, sts))
    out = []
    for k in range(n):
        r = ranks[k]
        out.append(dict(U=Us[k][:, :r], V=Vs[k][:, :r], Z=Zs[k][:r, :r], rank=r,
                        stats={f: getattr(stats[k], f) for f, _ in SolveStats._fields_},
                        status=STATUS_NAMES.get(sts[k], sts[k])))
    return out
