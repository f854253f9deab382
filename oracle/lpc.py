"""Reference of the preconditioner network (FP64, plain PyTorch CPU ops;
test infrastructure only).  The network is the library's design choice, not
the paper's (the paper reports no preconditioner for the ALS systems); this
module states it plainly so the GPU forward and gradients can be checked:

  a0 = relu(conv(in, W0, b0))     a1 = relu(conv(a0, W1, b1))
  p  = pool(a1)                   a2 = relu(conv(p, W2, b2))
  a3 = relu(conv(a2, W3, b3))     s  = up(a3) + a1
  y  = conv(s, W4, b4)

conv: 3x3x3 cross-correlation with zero padding, tap k = 9(dz+1) + 3(dy+1)
+ (dx+1), out[co, z, y, x] = b[co] + sum W[co, ci, k] in[ci, z+dz, y+dy, x+dx];
pool: coarse voxel (X, Y, Z) = sum of its children (2X+i, 2Y+j, 2Z+k) / 8,
children outside the grid counting as zero; up: nearest (child takes its
parent's value).  Arrays are (C, nz, ny, nx), voxel index x + nx (y + ny z).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def unpack(params: np.ndarray, C: int):
    """Split the flat parameter vector (layer order W0, b0, ..., W4, b4)."""
    ci = [4, C, C, C, C]
    co = [C, C, C, C, 1]
    out, k = [], 0
    for l in range(5):
        nw = co[l] * ci[l] * 27
        W = torch.tensor(params[k:k + nw], dtype=torch.float64).reshape(co[l], ci[l], 3, 3, 3)
        k += nw
        b = torch.tensor(params[k:k + co[l]], dtype=torch.float64)
        k += co[l]
        out.append((W, b))
    assert k == params.size
    return out


def conv(x, W, b):
    return F.conv3d(x[None], W, b, padding=1)[0]


def pool(x):
    C, nz, ny, nx = x.shape
    pz, py, px = nz % 2, ny % 2, nx % 2
    x = F.pad(x, (0, px, 0, py, 0, pz))
    C, Z, Y, X = x.shape
    return x.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).sum(dim=(2, 4, 6)) / 8.0


def up(x, shape):
    nz, ny, nx = shape
    x = x.repeat_interleave(2, 1).repeat_interleave(2, 2).repeat_interleave(2, 3)
    return x[:, :nz, :ny, :nx]


def forward(layers, inp):
    """inp: (4, nz, ny, nx) float64 tensor -> y (nz, ny, nx)."""
    (W0, b0), (W1, b1), (W2, b2), (W3, b3), (W4, b4) = layers
    a0 = torch.relu(conv(inp, W0, b0))
    a1 = torch.relu(conv(a0, W1, b1))
    p = pool(a1)
    a2 = torch.relu(conv(p, W2, b2))
    a3 = torch.relu(conv(a2, W3, b3))
    s = up(a3, a1.shape[1:]) + a1
    return conv(s, W4, b4)[0]


def forward_vjp(params: np.ndarray, C: int, dims, inp: np.ndarray, dy: np.ndarray):
    """y = net(inp) and the gradient of <y, dy> with respect to the flat
    parameters (layer order as in ``unpack``).  dims = (nx, ny, nz)."""
    nx, ny, nz = dims
    layers = unpack(params, C)
    for W, b in layers:
        W.requires_grad_(True)
        b.requires_grad_(True)
    x = torch.tensor(inp, dtype=torch.float64).reshape(4, nz, ny, nx)
    y = forward(layers, x)
    g = torch.tensor(dy, dtype=torch.float64).reshape(nz, ny, nx)
    (y * g).sum().backward()
    grad = np.concatenate([np.concatenate([W.grad.reshape(-1).numpy(), b.grad.numpy()])
                           for W, b in layers])
    return y.detach().reshape(-1).numpy(), grad
