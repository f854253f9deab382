"""Pins of the network reference: convolution orientation by brute-force
loops, pooling / upsampling by definition, gradients by central differences.
CPU only."""
import numpy as np
import torch

from oracle import lpc


def brute_conv(x, W, b):
    C, nz, ny, nx = x.shape
    co = W.shape[0]
    out = np.zeros((co, nz, ny, nx))
    for o in range(co):
        for z in range(nz):
            for y in range(ny):
                for xx in range(nx):
                    s = b[o]
                    for k in range(27):
                        dz, dy, dx = k // 9 - 1, (k // 3) % 3 - 1, k % 3 - 1
                        zz, yy, x2 = z + dz, y + dy, xx + dx
                        if 0 <= zz < nz and 0 <= yy < ny and 0 <= x2 < nx:
                            s += sum(W[o, c].reshape(-1)[k] * x[c, zz, yy, x2] for c in range(C))
                    out[o, z, y, xx] = s
    return out


def test_conv_matches_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 4, 5))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    got = lpc.conv(torch.tensor(x), torch.tensor(W), torch.tensor(b)).numpy()
    assert np.allclose(got, brute_conv(x, W, b), atol=1e-12)


def test_pool_and_up_by_definition():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 4))
    p = lpc.pool(torch.tensor(x)).numpy()
    assert p.shape == (2, 2, 3, 2)
    for c in range(2):
        for Z in range(2):
            for Y in range(3):
                for X in range(2):
                    s = 0.0
                    for i in range(8):
                        z, y, xx = 2 * Z + (i >> 2), 2 * Y + ((i >> 1) & 1), 2 * X + (i & 1)
                        if z < 3 and y < 5 and xx < 4:
                            s += x[c, z, y, xx]
                    assert abs(p[c, Z, Y, X] - s / 8) < 1e-14
    u = lpc.up(torch.tensor(p), (3, 5, 4)).numpy()
    assert u[1, 2, 4, 3] == p[1, 1, 2, 1]


def test_vjp_central_differences():
    rng = np.random.default_rng(2)
    C, dims = 3, (4, 4, 2)
    n = int(np.prod(dims))
    npar = sum(co * ci * 27 + co for ci, co in [(4, C), (C, C), (C, C), (C, C), (C, 1)])
    w = rng.standard_normal(npar) * 0.3
    inp = rng.standard_normal((4, n))
    dy = rng.standard_normal(n)
    y, g = lpc.forward_vjp(w, C, dims, inp, dy)
    h = 1e-6
    for idx in rng.choice(npar, 12, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        fp = lpc.forward_vjp(wp, C, dims, inp, dy)[0] @ dy
        fm = lpc.forward_vjp(wm, C, dims, inp, dy)[0] @ dy
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx])), (idx, fd, g[idx])
