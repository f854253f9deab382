"""Seeded synthetic inputs for the connectome regression problem.

This module only *draws* problem data: voxel geometries, the graph
Laplacians of their face-adjacency graphs (input of Algorithm 1 of the
paper), injection densities X, observation masks Omega (1 = observed) and
target densities Y.  It holds none of the solver's arithmetic (no operator,
no ALS, no Galerkin step) and is shared by the CPU oracle tests, the GPU
tests and the benchmark so that both sides read identical arrays.

Problem dictionaries use these keys (all numpy, float64 unless stated):

  Ly_rowptr, Ly_colidx (int32), Ly_val : CSR graph Laplacian of the target
  Lx_rowptr, Lx_colidx (int32), Lx_val : CSR graph Laplacian of the source
  X      n_x x n_inj   injection densities (nonnegative)
  Y      n_y x n_inj   target densities
  Omega  n_y x n_inj   uint8, 1 = observed, 0 = inside the injection hole
  lam    operator lambda (the normal equation uses lambda directly)
  max_rank, tau_res    Algorithm 1 rank cap and relative-residual stop
  Wt_a, Wt_g, Wt_h     W_true = sum_m a_m g_m h_m^T in factored form
                       (Wt_g n_y x m, Wt_h n_x x m); or Wt_dense for 1D
  coords_y, coords_x   integer voxel coordinates (n x dim)
  box_y, box_x         grid dims when the domain is a full box, else zeros

Draw order with ``numpy.random.default_rng(seed)``: injection centres,
injection amplitudes (shell workload only), W_true profile parameters,
noise matrix (n_y x n_inj, C order).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "graph_laplacian_csr", "box_coords", "toy_1d", "box_problem",
    "config1", "config1_small", "config2", "config2_tiny", "shell_problem",
    "config3", "config4_specs", "paper_toy", "cortex_2d", "tau_schedule",
]


# ---------------------------------------------------------------------------
# geometry -> graph Laplacian (L = Deg - Adj of the face-adjacency graph,
# unit weights, free boundary; the paper's L_x, L_y)
# ---------------------------------------------------------------------------
def graph_laplacian_csr(coords: np.ndarray):
    """CSR graph Laplacian of the face-adjacency graph of integer voxels.

    coords: (n, dim) int array of distinct voxel coordinates.  Voxel i is
    adjacent to j when their coordinates differ by one along one axis.
    Returns (rowptr int32, colidx int32 sorted per row, val float64).
    """
    coords = np.asarray(coords, dtype=np.int64)
    n, dim = coords.shape
    lo = coords.min(axis=0)
    c = coords - lo
    ext = c.max(axis=0) + 3
    strides = np.ones(dim, dtype=np.int64)
    for d in range(1, dim):
        strides[d] = strides[d - 1] * ext[d - 1]
    key = (c + 1) @ strides
    order = np.argsort(key)
    skey = key[order]
    rows, cols = [], []
    for d in range(dim):
        for sgn in (-1, 1):
            nk = key + sgn * strides[d]
            pos = np.searchsorted(skey, nk)
            pos = np.minimum(pos, n - 1)
            hit = skey[pos] == nk
            rows.append(np.nonzero(hit)[0])
            cols.append(order[pos[hit]])
    r = np.concatenate(rows)
    cl = np.concatenate(cols)
    deg = np.bincount(r, minlength=n)
    r_all = np.concatenate([r, np.arange(n)])
    c_all = np.concatenate([cl, np.arange(n)])
    v_all = np.concatenate([-np.ones(r.size), deg.astype(np.float64)])
    perm = np.lexsort((c_all, r_all))
    r_all, c_all, v_all = r_all[perm], c_all[perm], v_all[perm]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r_all + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr.astype(np.int32), c_all.astype(np.int32), v_all


def box_coords(dims) -> np.ndarray:
    """Voxel coordinates of a full box, first axis fastest."""
    dims = tuple(int(d) for d in dims)
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    # first axis fastest: transpose to Fortran flatten
    return np.stack([g.ravel(order="F") for g in grids], axis=1)


def _gauss(dist2: np.ndarray, sigma: float) -> np.ndarray:
    return np.exp(-dist2 / (2.0 * sigma * sigma))


def _pack(coords_y, coords_x, X, Y, Omega, lam, max_rank, tau_res, extra):
    ry, cy, vy = graph_laplacian_csr(coords_y)
    rx, cx, vx = graph_laplacian_csr(coords_x)
    p = dict(Ly_rowptr=ry, Ly_colidx=cy, Ly_val=vy,
             Lx_rowptr=rx, Lx_colidx=cx, Lx_val=vx,
             X=np.ascontiguousarray(X, dtype=np.float64),
             Y=np.ascontiguousarray(Y, dtype=np.float64),
             Omega=np.ascontiguousarray(Omega, dtype=np.uint8),
             lam=float(lam), max_rank=int(max_rank), tau_res=float(tau_res),
             coords_y=np.asarray(coords_y, np.int32),
             coords_x=np.asarray(coords_x, np.int32))
    p.update(extra)
    return p


# ---------------------------------------------------------------------------
# 1D toy: 200 voxels on a line, Gaussian bumps, Gaussian W_true
# ---------------------------------------------------------------------------
def toy_1d(n=200, n_inj=5, sigma_x=8.0, centre_lo=20.0, centre_hi=180.0,
           hole_r=10.0, wt_width=15.0, noise=0.01, lam=100.0, max_rank=20,
           tau_res=1e-8, seed=0):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(centre_lo, centre_hi, size=n_inj)
    pos = np.arange(n, dtype=np.float64)
    X = _gauss((pos[:, None] - centres[None, :]) ** 2, sigma_x)
    Omega = (np.abs(pos[:, None] - centres[None, :]) > hole_r).astype(np.uint8)
    Wt = _gauss((pos[:, None] - pos[None, :]) ** 2, wt_width)
    Ytrue = Wt @ X
    Y = Omega * Ytrue + noise * rng.standard_normal((n, n_inj))
    coords = pos.astype(np.int64)[:, None]
    return _pack(coords, coords, X, Y, Omega, lam, max_rank, tau_res,
                 dict(Wt_dense=Wt, box_y=np.array([n, 1, 1], np.int32),
                      box_x=np.array([n, 1, 1], np.int32), centres=centres))


def config1(seed=0):
    """Toy 1D, 200 voxels, n_inj 5, lambda 100, rank cap 20, relres 1e-8."""
    return toy_1d(seed=seed)


def config1_small(seed=0):
    """The 40-voxel variant of the toy: every length scaled by 0.2."""
    return toy_1d(n=40, sigma_x=1.6, centre_lo=4.0, centre_hi=36.0, hole_r=2.0,
                  wt_width=3.0, max_rank=40, seed=seed)


# ---------------------------------------------------------------------------
# The paper's own toy brain (section "Test problem: a toy brain"): S = T =
# [0, 1] on n lattice points, box-car injections, Omega = 1 - X, a Gaussian
# ridge about the diagonal plus an off-diagonal bump (eq. W_true_toy)
# ---------------------------------------------------------------------------
def paper_toy(n=200, n_inj=5, noise=0.1, lam=100.0, max_rank=140, tau_dW=1e-7,
              omega_ones=False, quadrature=False, seed=1):
    """Readings where the paper is silent: lattice points x_i = i / (n - 1);
    injection widths 0.12 + 0.1 eps (eps ~ U(0, 1), drawn first), centres
    uniform so that the injection stays inside [0, 1] (drawn second);
    W_true[i, k] = f(target y_i, source x_k) with the bump at source 0.8,
    target 0.1 (so the lower-left corner of W is near zero, where the paper
    finds its negative entries); Y = W_true X (quadrature=False) or
    W_true X / n (quadrature=True), zero inside the injection, plus N(0, noise^2)
    (drawn third).  omega_ones: the ablation with Omega = 1 everywhere."""
    rng = np.random.default_rng(seed)
    widths = 0.12 + 0.1 * rng.uniform(0.0, 1.0, size=n_inj)
    centres = rng.uniform(widths / 2, 1.0 - widths / 2)
    pos = np.arange(n, dtype=np.float64) / (n - 1)
    X = (np.abs(pos[:, None] - centres[None, :]) <= widths[None, :] / 2).astype(np.float64)
    Omega = np.ones_like(X, dtype=np.uint8) if omega_ones else (1 - X).astype(np.uint8)
    yt, xs = pos[:, None], pos[None, :]
    Wt = (np.exp(-((xs - yt) / 0.4) ** 2)
          + 0.9 * np.exp(-((xs - 0.8) ** 2 + (yt - 0.1) ** 2) / 0.2 ** 2))
    Ytrue = Wt @ X / (n if quadrature else 1.0)
    Y = (1 - X) * Ytrue + noise * rng.standard_normal((n, n_inj))
    coords = np.arange(n, dtype=np.int64)[:, None]
    return _pack(coords, coords, X, Y, Omega, lam, max_rank, 0.0,
                 dict(Wt_dense=Wt, box_y=np.array([n, 1, 1], np.int32),
                      box_x=np.array([n, 1, 1], np.int32), centres=centres, widths=widths,
                      tau_dW=float(tau_dW)))


# ---------------------------------------------------------------------------
# 3D boxes (target box, source box embedded at an offset)
# ---------------------------------------------------------------------------
def _wtrue_params(rng, m, box_t, box_s, w_lo, w_hi):
    cg = rng.uniform(0.0, 1.0, size=(m, 3)) * (np.asarray(box_t, float) - 1)
    ch = rng.uniform(0.0, 1.0, size=(m, 3)) * (np.asarray(box_s, float) - 1)
    wg = rng.uniform(w_lo, w_hi, size=m)
    wh = rng.uniform(w_lo, w_hi, size=m)
    a = rng.uniform(0.5, 1.0, size=m)
    return cg, ch, wg, wh, a


def _profiles(coords, cen, wid):
    cf = coords.astype(np.float64)
    out = np.empty((coords.shape[0], cen.shape[0]))
    for k in range(cen.shape[0]):
        d2 = ((cf - cen[k]) ** 2).sum(1)
        out[:, k] = _gauss(d2, wid[k])
    return out


def box_problem(box_y=(40, 40, 40), box_x=(30, 30, 30), offset=(5, 5, 5),
                n_inj=64, sigma=2.5, hole_r=3.0, wt_rank=8, wt_w=(4.0, 10.0),
                noise=0.01, lam=1e3, max_rank=60, tau_res=1e-4, seed=0):
    """Target box, source box at ``offset`` inside it (target coordinates)."""
    rng = np.random.default_rng(seed)
    cy = box_coords(box_y)
    cx = box_coords(box_x)
    off = np.asarray(offset, dtype=np.float64)
    centres = rng.uniform(0.0, 1.0, size=(n_inj, 3)) * (np.asarray(box_x, float) - 1)
    cxf = cx.astype(np.float64)
    cyf = cy.astype(np.float64)
    X = np.empty((cx.shape[0], n_inj))
    Omega = np.empty((cy.shape[0], n_inj), dtype=np.uint8)
    for a in range(n_inj):
        X[:, a] = _gauss(((cxf - centres[a]) ** 2).sum(1), sigma)
        Omega[:, a] = (((cyf - (centres[a] + off)) ** 2).sum(1) > hole_r ** 2)
    cg, ch, wg, wh, amp = _wtrue_params(rng, wt_rank, box_y, box_x, *wt_w)
    G = _profiles(cy, cg, wg)
    H = _profiles(cx, ch, wh)
    Ytrue = (G * amp[None, :]) @ (H.T @ X)
    Yobs = Omega * Ytrue
    rms = math.sqrt(float(np.mean(Yobs[Omega > 0] ** 2))) if Omega.any() else 1.0
    Y = Yobs + noise * rms * rng.standard_normal(Yobs.shape)
    return _pack(cy, cx, X, Y, Omega, lam, max_rank, tau_res,
                 dict(Wt_a=amp, Wt_g=G, Wt_h=H,
                      box_y=np.array(box_y, np.int32), box_x=np.array(box_x, np.int32),
                      centres=centres))


def config2(lam=1e3, seed=0):
    """3D grids: 40^3 target (64,000), 30^3 source (27,000), n_inj 64."""
    return box_problem(lam=lam, seed=seed)


def config2_tiny(seed=0, lam=10.0):
    """Tiny 3D variant for dense checks: 6x5x4 target, 4x4x3 source."""
    return box_problem(box_y=(6, 5, 4), box_x=(4, 4, 3), offset=(1, 0, 0),
                       n_inj=6, sigma=1.0, hole_r=1.0, wt_rank=3, wt_w=(1.5, 3.0),
                       lam=lam, max_rank=120, tau_res=1e-12, seed=seed)


# ---------------------------------------------------------------------------
# shells: two mirrored ellipsoidal shells in a 132 x 80 x 114 grid
# ---------------------------------------------------------------------------
def _shell_mask(grid, centre, semi, inner):
    g = np.stack(np.meshgrid(*[np.arange(n, dtype=np.float64) for n in grid],
                             indexing="ij"), -1)
    q = (((g - centre) / semi) ** 2).sum(-1)
    return (q <= 1.0) & (q > inner * inner)


def _largest_component(mask):
    from scipy import ndimage
    lab, nlab = ndimage.label(mask)  # default structure = face connectivity
    if nlab <= 1:
        return mask
    sizes = np.bincount(lab.ravel())
    sizes[0] = 0
    return lab == int(np.argmax(sizes))


def _mask_coords(mask):
    idx = np.nonzero(mask.ravel(order="F"))[0]
    return np.stack(np.unravel_index(idx, mask.shape, order="F"), axis=1)


def shell_masks(grid=(132, 80, 114), semi=(60.0, 36.0, 26.0), target_count=131072):
    """Right and left shells (mirror images about the mid plane of axis 2)."""
    grid = tuple(grid)
    sem = np.asarray(semi)
    cen_r = np.array([(grid[0] - 1) / 2.0, (grid[1] - 1) / 2.0,
                      (grid[2] - 1) / 2.0 + sem[2] + 2.5])
    lo, hi = 0.0, 1.0
    best = None
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        m = _shell_mask(grid, cen_r, sem, mid)
        cnt = int(m.sum())
        if best is None or abs(cnt - target_count) < abs(best[1] - target_count):
            best = (mid, cnt)
        if cnt > target_count:
            lo = mid
        else:
            hi = mid
    right = _largest_component(_shell_mask(grid, cen_r, sem, best[0]))
    left = right[:, :, ::-1]
    return right, left


def shell_problem(grid=(132, 80, 114), semi=(60.0, 36.0, 26.0), target_count=131072,
                  n_inj=128, sigma=3.0, cheb_r=4, wt_rank=8, wt_w=(6.0, 20.0),
                  mult_noise=0.05, lam=1e3, max_rank=100, tau_res=1e-4, seed=0):
    """Target = both shells, source = right shell (same physical voxels)."""
    right, left = shell_masks(grid, semi, target_count)
    tgt = right | left
    cy = _mask_coords(tgt)
    cx = _mask_coords(right)
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, cx.shape[0], size=n_inj)
    centres = cx[pick].astype(np.float64) + rng.uniform(-0.5, 0.5, size=(n_inj, 3))
    amps = rng.lognormal(0.0, 0.5, size=n_inj)
    cxf = cx.astype(np.float64)
    X = np.empty((cx.shape[0], n_inj))
    Omega = np.empty((cy.shape[0], n_inj), dtype=np.uint8)
    for a in range(n_inj):
        X[:, a] = amps[a] * _gauss(((cxf - centres[a]) ** 2).sum(1), sigma)
        cheb = np.abs(cy - centres[a]).max(axis=1)
        Omega[:, a] = cheb > cheb_r
    gmin = np.zeros(3)
    gbox = np.asarray(grid, float)
    cg = rng.uniform(0.0, 1.0, size=(wt_rank, 3)) * (gbox - 1) + gmin
    ch = rng.uniform(0.0, 1.0, size=(wt_rank, 3)) * (gbox - 1) + gmin
    wg = rng.uniform(*wt_w, size=wt_rank)
    wh = rng.uniform(*wt_w, size=wt_rank)
    amp = rng.uniform(0.5, 1.0, size=wt_rank)
    G = _profiles(cy, cg, wg)
    H = _profiles(cx, ch, wh)
    Ytrue = (G * amp[None, :]) @ (H.T @ X)
    Y = (Omega * Ytrue) * (1.0 + mult_noise * rng.standard_normal(Ytrue.shape))
    return _pack(cy, cx, X, Y, Omega, lam, max_rank, tau_res,
                 dict(Wt_a=amp, Wt_g=G, Wt_h=H, box_y=np.zeros(3, np.int32),
                      box_x=np.zeros(3, np.int32), centres=centres))


def config3(seed=0):
    """Cortex-shaped shells: n_y ~ 262,144, n_x ~ 131,072, n_inj 128."""
    return shell_problem(seed=seed)


# ---------------------------------------------------------------------------
# 2-D cortical maps: stand-ins for the paper's top-view and flatmap data
# (two mirrored hemispheres on a pixel lattice, 5-point graph Laplacians,
# 126 injections, Omega = 1{X <= 0.4} as for the real data)
# ---------------------------------------------------------------------------
def _ellipse_count(a, b):
    yy, xx = np.mgrid[-int(b) - 1:int(b) + 2, -int(a) - 1:int(a) + 2]
    return int(np.count_nonzero((xx / a) ** 2 + (yy / b) ** 2 <= 1.0))


def hemisphere_masks_2d(per_hemi, aspect=1.35, gap=2):
    """Two mirrored elliptical hemispheres (semi-axes a = aspect b) whose
    pixel counts are within 0.1% of per_hemi (b found by bisection)."""
    lo, hi = 2.0, 4000.0
    for _ in range(60):
        b = 0.5 * (lo + hi)
        if _ellipse_count(aspect * b, b) < per_hemi:
            lo = b
        else:
            hi = b
    b = hi
    a = aspect * b
    nyg = 2 * int(b) + 3
    nxg = 2 * (2 * int(a) + 3) + gap
    yy, xx = np.mgrid[0:nyg, 0:nxg].astype(np.float64)
    cy0 = (nyg - 1) / 2.0
    cl = int(a) + 1.0
    cr = nxg - 1 - cl
    left = ((xx - cl) / a) ** 2 + ((yy - cy0) / b) ** 2 <= 1.0
    right = ((xx - cr) / a) ** 2 + ((yy - cy0) / b) ** 2 <= 1.0
    return right, left


def cortex_2d(kind="topview", n_inj=126, sigma=(3.0, 6.0), wt_rank=8, wt_w=(8.0, 30.0),
              mult_noise=0.05, lam_bar=None, max_rank=500, seed=0):
    """kind "topview": n_y ~ 44,478, n_x ~ 22,239 (the paper's top view has
    n_y = 44,478, n_x = 22,377); "flatmap": n_y ~ 126,847, n_x ~ 63,424
    (paper: 126,847 / 63,435).  Target = both hemispheres, source = the
    right one (same pixels).  Injections: centres on random source pixels,
    X = Gaussian of width U[sigma], peak 1 (values in [0, 1], about 30 to
    500 pixels above 0.1); Omega = 0 where the injection density at the
    target pixel exceeds 0.4 (the paper's rule for its data).  W_true as
    for the cortex shells (rank-8 Gaussian profiles), multiplicative noise.
    lambda = lambda_bar n_inj / n_x with the paper's lambda_bar (1e6 top
    view, 3e7 flatmap)."""
    per = {"topview": 22239, "flatmap": 63424}[kind]
    if lam_bar is None:
        lam_bar = {"topview": 1e6, "flatmap": 3e7}[kind]
    right, left = hemisphere_masks_2d(per)
    cy = _mask_coords(right | left)
    cx = _mask_coords(right)
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, cx.shape[0], size=n_inj)
    centres = cx[pick].astype(np.float64) + rng.uniform(-0.5, 0.5, size=(n_inj, 2))
    widths = rng.uniform(sigma[0], sigma[1], size=n_inj)
    cxf, cyf = cx.astype(np.float64), cy.astype(np.float64)
    X = np.empty((cx.shape[0], n_inj))
    Omega = np.empty((cy.shape[0], n_inj), dtype=np.uint8)
    for a in range(n_inj):
        X[:, a] = _gauss(((cxf - centres[a]) ** 2).sum(1), widths[a])
        Omega[:, a] = _gauss(((cyf - centres[a]) ** 2).sum(1), widths[a]) <= 0.4
    grid = np.asarray(right.shape, float)
    cg = rng.uniform(0.0, 1.0, size=(wt_rank, 2)) * (grid - 1)
    ch = rng.uniform(0.0, 1.0, size=(wt_rank, 2)) * (grid - 1)
    wg = rng.uniform(*wt_w, size=wt_rank)
    wh = rng.uniform(*wt_w, size=wt_rank)
    amp = rng.uniform(0.5, 1.0, size=wt_rank)
    G = _profiles(cy, cg, wg)
    H = _profiles(cx, ch, wh)
    Ytrue = (G * amp[None, :]) @ (H.T @ X)
    Y = (Omega * Ytrue) * (1.0 + mult_noise * rng.standard_normal(Ytrue.shape))
    lam = lam_bar * n_inj / cx.shape[0]
    return _pack(cy, cx, X, Y, Omega, lam, max_rank, 0.0,
                 dict(Wt_a=amp, Wt_g=G, Wt_h=H, box_y=np.zeros(3, np.int32),
                      box_x=np.zeros(3, np.int32), centres=centres, lam_bar=float(lam_bar)))


def tau_schedule(r, r_lo=125, r_hi=1000, tau_lo=1e-3, tau_hi=1e-6):
    """The paper's stopping tolerances for its real-data runs: geometric in r
    from tau_lo at r_lo to tau_hi at r_hi."""
    t = math.log(r / r_lo) / math.log(r_hi / r_lo)
    return float(tau_lo * (tau_hi / tau_lo) ** t)


@dataclass
class BatchSpec:
    box_y: tuple
    box_x: tuple
    n_inj: int
    lam: float
    seed: int


def _near_cubic(n):
    a = max(2, int(round(n ** (1.0 / 3.0))))
    b = a
    c = max(2, int(round(n / (a * b))))
    return (a, b, c)


def config4_specs(spec_seed=0, count=16):
    """Sizes of the 16 uneven box problems (each then built by box_problem)."""
    rng = np.random.default_rng(spec_seed)
    out = []
    for k in range(count):
        ny = int(rng.integers(20000, 120001))
        nx = ny // 2
        ninj = int(rng.integers(16, 129))
        lam = float(10.0 ** rng.uniform(1.0, 4.0))
        by = _near_cubic(ny)
        bx = _near_cubic(nx)
        out.append(BatchSpec(by, bx, ninj, lam, 1000 + k))
    return out
