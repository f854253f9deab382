"""The allocation-free operator application (cr_op_apply_noalloc, workspace
in a static device array) against cr_op_apply on the same inputs, through
the C ABI: two calls in a row, the second with a smaller input (smaller
rank on a smaller problem), at the FP64 parity bars of the operator
(1e-13 for the stencil blocks, 1e-12 for the masked product; the split-K
depth of H = V^T X may differ, so the data term can differ in rounding)."""
import numpy as np
import pytest
import torch

from paper_1808_05510_amd import connreg, synth
from tests.helpers import max_rel, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(d, r, seed):
    g = connreg.Problem(d, "fp64", DEV)
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((g.n_y, r))
    V = rng.standard_normal((g.n_x, r))
    Z = rng.standard_normal((r, r))
    return g, U, Z, V


def _compare(g, U, Z, V):
    r = U.shape[1]
    F1, G1 = g.op_apply(U, Z, V)
    F2, G2 = g.op_apply(U, Z, V, noalloc=True)
    torch.cuda.synchronize()
    F1, G1, F2, G2 = (t.cpu().numpy() for t in (F1, G1, F2, G2))
    assert F2.shape == F1.shape and G2.shape == G1.shape
    if r:
        assert max_rel(F2[:, :2 * r], F1[:, :2 * r]) < 1e-13
        assert max_rel(G2, G1) < 1e-13
    assert max_rel(F2[:, 2 * r:], F1[:, 2 * r:]) < 1e-12
    assert rel(F2, F1) < 1e-12


def test_noalloc_matches_op_apply_two_calls_second_smaller():
    big = synth.box_problem(box_y=(11, 10, 9), box_x=(8, 7, 9), offset=(1, 2, 0), n_inj=37,
                            sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 4.0), lam=30.0, seed=4)
    g, U, Z, V = _case(big, 100, 1)
    _compare(g, U, Z, V)
    small = synth.config2_tiny(seed=2)
    g2, U2, Z2, V2 = _case(small, 7, 2)
    _compare(g2, U2, Z2, V2)
    # and the first handle again, at a smaller rank, after the other call
    _compare(g, U[:, :12].copy(), Z[:12, :12].copy(), V[:, :12].copy())
    g.close()
    g2.close()


def test_noalloc_full_shells_r100():
    """The benchmark's operator shape (n_y 262,136, n_inj 128, r 100)."""
    d = synth.config3(seed=0)
    g, U, Z, V = _case(d, 100, 3)
    _compare(g, U, Z, V)
    _compare(g, U[:, :40].copy(), Z[:40, :40].copy(), V[:, :40].copy())
    g.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    d = synth.box_problem(box_y=(11, 10, 9), box_x=(8, 7, 9), offset=(1, 2, 0), n_inj=37,
                          sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 4.0), lam=30.0, seed=4)
    g, U, Z, V = _case(d, 257, 5)
    with pytest.raises(connreg.ConnRegError, match="scratch"):
        g.op_apply(U, Z, V, noalloc=True)
    g.close()


def test_noalloc_op_apply_replays_in_a_captured_graph():
    """The callers the entry point is for: captured once into a graph (on the
    handle's stream, its fork to the auxiliary stream and join included) and
    replayed with new inputs copied into the captured buffers; every replay,
    with eager work and a synchronisation between replays, equals the eager
    call on the same inputs exactly (the same kernels in the same shapes)."""
    d = synth.box_problem(box_y=(11, 10, 9), box_x=(8, 7, 9), offset=(1, 2, 0), n_inj=37,
                          sigma=1.5, hole_r=1.5, wt_rank=4, wt_w=(2.0, 4.0), lam=30.0, seed=4)
    s = torch.cuda.Stream(DEV)
    g = connreg.Problem(d, "fp64", DEV, stream=s)
    r = 24
    gen = torch.Generator(device=DEV).manual_seed(7)

    def colmajor_randn(n, k):
        return torch.randn((k, n), device=DEV, dtype=torch.float64, generator=gen).T

    U, Z, V = colmajor_randn(g.n_y, r), colmajor_randn(r, r), colmajor_randn(g.n_x, r)
    F = connreg.empty_colmajor(g.n_y, 2 * r + g.n_inj, DEV)
    G = connreg.empty_colmajor(g.n_x, 2 * r, DEV)
    with torch.cuda.stream(s):
        g.op_apply(U, Z, V, out=(F, G), noalloc=True)
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        g.op_apply(U, Z, V, out=(F, G), noalloc=True)
    s.synchronize()
    try:
        for k in range(4):
            with torch.cuda.stream(s):
                U.copy_(colmajor_randn(g.n_y, r))
                Z.copy_(colmajor_randn(r, r))
                V.copy_(colmajor_randn(g.n_x, r))
                graph.replay()
            s.synchronize()
            Fg, Gg = F.cpu().numpy(), G.cpu().numpy()
            with torch.cuda.stream(s):
                Fe, Ge = g.op_apply(U, Z, V, noalloc=True)
            s.synchronize()
            assert np.array_equal(Fg, Fe.cpu().numpy()), k
            assert np.array_equal(Gg, Ge.cpu().numpy()), k
    finally:
        del graph
        g.close()
