"""Pins of the FP64 network-layer oracle (CPU)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import conv as C


def _rand(rng, *shape):
    return rng.standard_normal(shape)


def test_conv3d_matches_scipy_correlate():
    """Each (co, ci) pair is a 3-D correlation with zero padding (scipy.ndimage)."""
    rng = np.random.default_rng(0)
    x = _rand(rng, 4, 5, 6, 3)
    w = _rand(rng, 2, 27, 3)
    b = _rand(rng, 2)
    y = C.conv3d(x, w, b)
    for co in range(2):
        ref = np.full(x.shape[:3], b[co])
        for ci in range(3):
            ref += ndimage.correlate(x[..., ci], w[co, :, ci].reshape(3, 3, 3), mode="constant", cval=0.0)
        assert np.allclose(y[..., co], ref, atol=1e-12)


def test_conv3d_adjoints_dot_product():
    """<dy, conv(x)> = <dgrad(dy), x> and = <wgrad(x, dy), w> (bias-free)."""
    rng = np.random.default_rng(1)
    x = _rand(rng, 4, 4, 6, 5)
    w = _rand(rng, 3, 27, 5)
    dy = _rand(rng, 4, 4, 6, 3)
    lhs = np.sum(dy * C.conv3d(x, w))
    assert np.sum(C.conv3d_dgrad(dy, w) * x) == pytest.approx(lhs, rel=1e-12)
    dw, db = C.conv3d_wgrad(x, dy)
    assert np.sum(dw * w) == pytest.approx(lhs, rel=1e-12)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


def test_conv3d_wgrad_finite_difference():
    rng = np.random.default_rng(2)
    x = _rand(rng, 3, 4, 4, 2)
    w = _rand(rng, 2, 27, 2)
    dy = _rand(rng, 3, 4, 4, 2)
    dw, _ = C.conv3d_wgrad(x, dy)
    for (o, t, i) in [(0, 0, 0), (1, 13, 1), (0, 26, 1), (1, 5, 0)]:
        e = np.zeros_like(w)
        e[o, t, i] = 1e-6
        fd = (np.sum(dy * C.conv3d(x, w + e)) - np.sum(dy * C.conv3d(x, w - e))) / 2e-6
        assert dw[o, t, i] == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(3)
    x = _rand(rng, 4, 6, 8, 3)
    dyp = _rand(rng, 2, 3, 4, 3)
    assert np.sum(dyp * C.pool(x)) == pytest.approx(np.sum(C.pool_bwd(dyp) * x), rel=1e-12)
    xs = _rand(rng, 2, 3, 4, 3)
    dyu = _rand(rng, 4, 6, 8, 3)
    assert np.sum(dyu * C.up(xs)) == pytest.approx(np.sum(C.up_bwd(dyu) * xs), rel=1e-12)
    assert np.allclose(C.pool(np.ones((2, 2, 2, 1))), 1.0)


def test_mse_gradient_and_adam_first_step():
    rng = np.random.default_rng(4)
    p, t = _rand(rng, 3, 4, 5), _rand(rng, 3, 4, 5)
    mask = rng.random((3, 4, 5)) < 0.6
    loss, g = C.mse(p, t, mask)
    e = np.zeros_like(p)
    e[1, 2, 3] = 1e-6
    fd = (C.mse(p + e, t, mask)[0] - C.mse(p - e, t, mask)[0]) / 2e-6
    assert g[1, 2, 3] == pytest.approx(fd, rel=1e-6, abs=1e-12)
    # weighted: a weight of 2 on one voxel is the same as counting that voxel twice
    w = np.ones_like(p)
    w[1, 2, 3] = 2.0
    lw, gw = C.mse(p, t, mask, w)
    d = np.where(mask, p - t, 0.0)
    assert lw == pytest.approx(((d * d).sum() + d[1, 2, 3] ** 2) / mask.sum(), rel=1e-12)
    fdw = (C.mse(p + e, t, mask, w)[0] - C.mse(p - e, t, mask, w)[0]) / 2e-6
    assert gw[1, 2, 3] == pytest.approx(fdw, rel=1e-6, abs=1e-12)
    # Adam's first step from zero moments moves each weight by lr * g / (|g| + eps)
    g = _rand(rng, 10)
    p0 = _rand(rng, 10)
    p1, m, v = C.adam(p0, np.zeros(10), np.zeros(10), g, 1, lr=1e-3, eps=1e-8)
    assert np.allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
