"""Plain FP64 reference of the warm-start network's layers, for gradient checks.

TEST INFRASTRUCTURE ONLY: only the test-suite may import it.  It shares no code
with the HIP kernels.  Tensors are (nz, ny, nx, c) arrays (channel last); 3x3x3
weights are (cout, 27, cin) with tap = (dz+1)*9 + (dy+1)*3 + (dx+1).

Each function is the textbook definition: a 3x3x3 convolution with zero padding,
its adjoints with respect to the input and to the weights, 2x2x2 average pooling,
nearest-neighbour upsampling, a 1x1x1 head, a weighted masked mean squared error and one
Adam step (Kingma and Ba, 2015).  ``np.einsum`` serves as the contraction.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, dz, dy, dx):
    """s[z, y, x] = x[z+dz, y+dy, x+dx], zero outside."""
    nz, ny, nx = x.shape[:3]
    out = np.zeros_like(x)
    zs, ys, xs = slice(max(0, -dz), nz - max(0, dz)), slice(max(0, -dy), ny - max(0, dy)), slice(max(0, -dx), nx - max(0, dx))
    zt, yt, xt = slice(max(0, dz), nz - max(0, -dz)), slice(max(0, dy), ny - max(0, -dy)), slice(max(0, dx), nx - max(0, -dx))
    out[zs, ys, xs] = x[zt, yt, xt]
    return out


def conv3d(x, w, b=None, relu=False):
    """y[v, co] = b[co] + sum_{tap, ci} w[co, tap, ci] x[v + tap, ci]."""
    x = np.asarray(x, np.float64)
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += np.einsum("zyxc,oc->zyxo", _shift(x, dz, dy, dx), w[:, t, :])
    if b is not None:
        y += b
    return np.maximum(y, 0.0) if relu else y


def conv3d_dgrad(dy, w):
    """Adjoint in x: dx[v, ci] = sum_{tap, co} w[co, tap, ci] dy[v - tap, co]."""
    dx = np.zeros(dy.shape[:3] + (w.shape[2],))
    for t, (dz, ddy, ddx) in enumerate(TAPS):
        dx += _shift(np.einsum("zyxo,oc->zyxc", dy, w[:, t, :]), -dz, -ddy, -ddx)
    return dx


def conv3d_wgrad(x, dy):
    """Adjoint in w: dw[co, tap, ci] = sum_v dy[v, co] x[v + tap, ci]; db[co] = sum_v dy[v, co]."""
    dw = np.zeros((dy.shape[3], 27, x.shape[3]))
    for t, (dz, ddy, ddx) in enumerate(TAPS):
        dw[:, t, :] = np.einsum("zyxo,zyxc->oc", dy, _shift(x, dz, ddy, ddx))
    return dw, dy.sum(axis=(0, 1, 2))


def pool(x):
    nz, ny, nx, c = x.shape
    return x.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).mean(axis=(1, 3, 5))


def pool_bwd(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_bwd(dy):
    nz, ny, nx, c = dy.shape
    return dy.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).sum(axis=(1, 3, 5))


def head(x, w, b, base=None):
    out = np.einsum("zyxc,c->zyx", x, w) + b
    return out + base if base is not None else out


def mse(pred, target, mask, weight=None):
    """sum over masked voxels of w (pred - target)^2, divided by the masked count."""
    m = mask.astype(bool)
    d = np.where(m, pred - target, 0.0)
    w = np.ones_like(d) if weight is None else np.asarray(weight, np.float64)
    n = m.sum()
    return float((w * d * d).sum() / n), 2.0 * w * d / n


def adam(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- the whole network

LEVELS = (16, 32, 64, 128)
IN_CH = 16


def unet_forward(P, feat):
    """FP64 forward of the warm-start U-Net: P maps layer names to (w (cout, 27, cin), b)
    and 'head' to (w (c,), b scalar); feat is (nz, ny, nx, 16)."""
    c = lambda name, x: conv3d(x, P[name][0], P[name][1], relu=True)  # noqa: E731
    e1 = c("e1b", c("e1a", feat))
    e2 = c("e2b", c("e2a", pool(e1)))
    e3 = c("e3b", c("e3a", pool(e2)))
    b4 = c("b4b", c("b4a", pool(e3)))
    d3 = c("d3b", c("d3a", np.concatenate([e3, up(b4)], axis=3)))
    d2 = c("d2b", c("d2a", np.concatenate([e2, up(d3)], axis=3)))
    d1 = c("d1b", c("d1a", np.concatenate([e1, up(d2)], axis=3)))
    return head(d1, P["head"][0], P["head"][1])
