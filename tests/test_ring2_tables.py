"""Host logic: the tables of rows of L^2 (csrc/ring2.hpp) that the two-barrier
PCG and the fused operator sweep read, built on the CPU by a small driver and
checked against the squared Laplacian itself (scipy sparse products of the
graph Laplacian the ELL table encodes).

  * two-barrier form: diag, ELL-slot and ring-2 coefficients reproduce L^2 w;
  * window form: every tile's intervals stage the voxels its rows read, and
    the packed entries reproduce L w and L^2 w from the staged window;
  * fit limits: a renumbered box has rows but no windows; width 8 has neither.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1808_05510_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1808_05510_amd", "csrc")
W2_TILE, W2_NI, W2_MAX, W2_NE, W2_NL = 64, 12, 1024, 25, 7
W2_TAB = 2 + 2 * W2_NI
R2_NX, R2_NC = W2_NE - W2_NL, W2_NE


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("ring2") / "ring2_driver")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "ring2_driver.cpp"),
                    "-o", out], check=True)
    return out


def ell(rowptr, colidx):
    """Self-padded ELL table as the library builds it: width = max degree
    rounded up to an even number in [2, 8], neighbours in CSR order."""
    n = len(rowptr) - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    off = colidx != rows
    deg = np.bincount(rows[off], minlength=n)
    K = min(8, max(2, (int(deg.max()) + 1) // 2 * 2))
    nbr = np.repeat(np.arange(n, dtype=np.int32)[None, :], K, 0)
    r_, c_ = rows[off], colidx[off]
    slot = np.arange(len(r_)) - np.searchsorted(r_, np.arange(n))[r_]
    nbr[slot, r_] = c_
    return K, nbr


def laplacian(n, K, nbr):
    N = sp.csr_matrix((np.ones(K * n), (np.tile(np.arange(n), K), nbr.ravel())), shape=(n, n))
    return (K * sp.identity(n, format="csr") - N).tocsr()


def run(driver, tmp_path, n, K, nbr):
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.int64(n).tobytes() + np.int32(K).tobytes() + nbr.astype(np.int32).tobytes())
    subprocess.run([driver, str(src), str(dst)], check=True)
    raw = np.fromfile(dst, dtype=np.uint8)
    rows, wins = raw[:8].view(np.int32)
    o = 8
    out = dict(rows=bool(rows), windows=bool(wins))
    if rows:
        out["r2idx"] = raw[o:o + 4 * R2_NX * n].view(np.int32).reshape(R2_NX, n)
        o += 4 * R2_NX * n
        out["r2cf"] = raw[o:o + R2_NC * n].view(np.int8).reshape(R2_NC, n)
        o += R2_NC * n
    if wins:
        nt = (n + W2_TILE - 1) // W2_TILE
        out["w2tab"] = raw[o:o + 4 * nt * W2_TAB].view(np.int32).reshape(nt, W2_TAB)
        o += 4 * nt * W2_TAB
        out["w2ent"] = raw[o:o + 4 * W2_NE * n].view(np.uint32).reshape(W2_NE, n)
        o += 4 * W2_NE * n
    assert o == len(raw)
    return out


def line(n=200):
    L = sp.diags([-np.ones(n - 1), np.r_[1, 2 * np.ones(n - 2), 1], -np.ones(n - 1)], [-1, 0, 1])
    L = L.tocsr()
    return L.indptr, L.indices


def grid2d(nx=23, ny=17):
    idx = np.arange(nx * ny).reshape(ny, nx)
    rows, cols = [], []
    for dy, dx in ((0, 1), (1, 0)):
        a = idx[:ny - dy, :nx - dx].ravel()
        b = idx[dy:, dx:].ravel()
        rows += [a, b]
        cols += [b, a]
    A = sp.csr_matrix((np.ones(sum(len(r) for r in rows)), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nx * ny,) * 2)
    L = (sp.diags(np.asarray(A.sum(1)).ravel()) - A).tocsr()
    L.sort_indices()
    return L.indptr, L.indices


def box():
    d = synth.box_problem(box_y=(11, 10, 9), box_x=(8, 7, 9), offset=(1, 2, 0), n_inj=4, sigma=1.5,
                          hole_r=1.5, wt_rank=2, wt_w=(2.0, 4.0), lam=30.0, seed=8)
    return d["Ly_rowptr"], d["Ly_colidx"]


def scrambled():
    # 2,688 voxels renumbered at random: a tile's rows of L^2 then read more
    # voxels than one window holds
    d = synth.box_problem(box_y=(16, 14, 12), box_x=(8, 7, 9), offset=(1, 2, 0), n_inj=4,
                          sigma=1.5, hole_r=1.5, wt_rank=2, wt_w=(2.0, 4.0), lam=30.0, seed=7)
    rp, ci = d["Ly_rowptr"], d["Ly_colidx"]
    n = len(rp) - 1
    L = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    perm = np.random.default_rng(3).permutation(n)
    Lp = L[perm][:, perm].tocsr()
    Lp.sort_indices()
    return Lp.indptr, Lp.indices


@pytest.mark.parametrize("geom,wins", [(line, True), (grid2d, True), (box, True),
                                        (scrambled, False)])
def test_ring2_tables_reproduce_l_and_l2(driver, tmp_path, geom, wins):
    rp, ci = geom()
    K, nbr = ell(np.asarray(rp), np.asarray(ci))
    n = nbr.shape[1]
    t = run(driver, tmp_path, n, K, nbr)
    assert t["rows"] and t["windows"] == wins
    L = laplacian(n, K, nbr)
    w = np.random.default_rng(0).standard_normal((n, 3))
    Lw, L2w = L @ w, L @ (L @ w)
    # two-barrier form
    idx = t["r2idx"].astype(np.int64)
    cf = t["r2cf"].astype(np.float64)
    assert idx.min() >= 0 and idx.max() < n
    l2 = cf[0][:, None] * w
    for k in range(K):
        l2 += cf[1 + k][:, None] * w[nbr[k]]
    for e in range(R2_NX):
        l2 += cf[W2_NL + e][:, None] * w[idx[e]]
    assert np.abs(l2 - L2w).max() <= 1e-13 * np.abs(L2w).max()
    if not wins:
        return
    ent = t["w2ent"]
    pos = (ent & 0xFFFF).astype(np.int64)
    c2 = ((ent.astype(np.int32) << 8) >> 24).astype(np.float64)
    c1 = (ent.astype(np.int32) >> 24).astype(np.float64)
    assert np.all(c1[W2_NL:] == 0)
    for tile, it in enumerate(t["w2tab"]):
        nint, tot = int(it[0]), int(it[1])
        assert 1 <= nint <= W2_NI and 1 <= tot <= W2_MAX
        starts, pref = it[2:2 + W2_NI], it[2 + W2_NI:]
        assert pref[0] == 0 and np.all(np.diff(starts[:nint]) > 0)
        # the kernel's staging map: window element e comes from voxel src[e]
        q = np.searchsorted(pref[:nint], np.arange(tot), side="right") - 1
        src = starts[q] + (np.arange(tot) - pref[q])
        assert src.min() >= 0 and src.max() < n
        v0, v1 = tile * W2_TILE, min(n, (tile + 1) * W2_TILE)
        P = pos[:, v0:v1]
        assert P.max() < tot
        assert np.array_equal(src[P[0]], np.arange(v0, v1))  # entry 0: the voxel itself
        win = w[src]
        s1 = np.einsum("ev,evc->vc", c1[:, v0:v1], win[P])
        s2 = np.einsum("ev,evc->vc", c2[:, v0:v1], win[P])
        assert np.abs(s1 - Lw[v0:v1]).max() <= 1e-13 * np.abs(Lw).max()
        assert np.abs(s2 - L2w[v0:v1]).max() <= 1e-13 * np.abs(L2w).max()


def test_ring2_tables_width_eight_has_none(driver, tmp_path):
    """A voxel with 7 or 8 neighbours (ELL width 8) is beyond both forms."""
    n = 40
    A = sp.lil_matrix((n, n))
    for i in range(n):
        for d in (1, 2, 3, 4):
            A[i, (i + d) % n] = A[(i + d) % n, i] = 1
    A = A.tocsr()
    L = (sp.diags(np.asarray(A.sum(1)).ravel()) - A).tocsr()
    L.sort_indices()
    K, nbr = ell(L.indptr, L.indices)
    assert K == 8
    t = run(driver, tmp_path, n, K, nbr)
    assert not t["rows"] and not t["windows"]
