"""Warm-start network kernels on the GPU against the FP64 layer oracle.

Inputs are rounded to BF16 before both sides see them, so the oracle computes on
exactly the values the kernels read; FP32-accumulated outputs then agree to the
accumulation order (relative 1e-4 here), BF16 outputs to one BF16 rounding."""
import numpy as np
import pytest

from oracle import conv as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def U():
    from paper_1410_1914_amd import lbm, unet

    lbm.require_gpu()
    unet.load()
    return unet


def _bf(rng, *shape, scale=1.0):
    """Random values exactly representable in BF16 (returned as float64)."""
    import torch

    x = torch.tensor(rng.standard_normal(shape) * scale, dtype=torch.float32).to(torch.bfloat16)
    return x.to(torch.float64).numpy()


def _dev_bf16(a):
    import torch

    return torch.tensor(np.asarray(a), dtype=torch.float32).to(torch.bfloat16).cuda()


def _dev_f32(a):
    import torch

    return torch.tensor(np.asarray(a), dtype=torch.float32).cuda()


def _host(t):
    import torch

    torch.cuda.synchronize()
    return t.to(torch.float64).cpu().numpy()


def _wmat(w, cin, kpad):
    """(cout, 27, cin) -> (cout, kpad) with k = tap * cin + ci, zero padded."""
    cout = w.shape[0]
    m = np.zeros((cout, kpad))
    m[:, :27 * cin] = w.reshape(cout, 27 * cin)
    return m


def test_mfma_lane_layout(U):
    rng = np.random.default_rng(0)
    A, B = _bf(rng, 16, 32), _bf(rng, 32, 16)
    d = _dev_f32(np.zeros((16, 16)))
    U.unet_mfma_selftest(_dev_f32(A), _dev_f32(B), d)
    assert np.allclose(_host(d), A @ B, rtol=1e-5, atol=1e-5)


CONV = [  # cin, cout, (ldx, offx), (ldy, offy), relu
    (16, 16, (16, 0), (16, 0), True),
    (16, 32, (48, 16), (32, 0), False),
    (48, 192, (48, 0), (192, 0), True),
    (32, 64, (32, 0), (96, 32), True),
    (64, 48, (64, 0), (48, 0), False),
]


@pytest.mark.parametrize("cin,cout,xs,ys,relu", CONV)
def test_conv3d_forward(U, cin, cout, xs, ys, relu):
    import torch

    rng = np.random.default_rng(cin + cout)
    shape = (4, 6, 9)  # 216 voxels: four workgroups, the last one ragged
    ldx, offx = xs
    ldy, offy = ys
    xbuf = _bf(rng, *shape, ldx)
    x = xbuf[..., offx:offx + cin]
    w = _bf(rng, cout, 27, cin, scale=0.2)
    b = _bf(rng, cout)
    kp = U.unet_kpad(cin)
    y = torch.zeros(shape + (ldy,), dtype=torch.bfloat16, device="cuda")
    y32 = torch.zeros(shape + (cout,), dtype=torch.float32, device="cuda")
    U.unet_conv3d_fwd(_dev_bf16(xbuf), ldx, offx, _dev_bf16(_wmat(w, cin, kp)), _dev_f32(b), y, ldy, offy, y32,
                      shape, cin, cout, relu)
    ref = C.conv3d(x, w, b, relu=relu)
    got = _host(y32)
    assert np.allclose(got, ref, rtol=1e-4, atol=1e-4)
    yb = _host(y)
    assert np.allclose(yb[..., offy:offy + cout], ref, rtol=1e-2, atol=1e-2)
    assert np.all(yb[..., :offy] == 0) and np.all(yb[..., offy + cout:] == 0)


@pytest.mark.parametrize("shape,cin", [((26, 258, 130), 16), ((26, 258, 130), 32), ((98, 516, 130), 16)])
def test_conv3d_forward_on_a_large_grid(U, shape, cin):
    """The launch forms for large grids, ragged in every direction (x in tiles of 64,
    y in tiles of 4), 32 output channels written at offset 16 of 48-channel rows:
    16 input channels march through runs of planes (runs of 6 on 26 planes, of 32 on
    98 planes, the last run short); 32 take four output planes per workgroup (2048
    workgroups or more).  Boxes at the corners and inside are compared with the
    oracle; every output voxel is written, the other channels are left alone."""
    import torch

    rng = np.random.default_rng(7 + cin + shape[0])
    cout, ldy, offy = 32, 48, 16
    nwg = -(-shape[2] // 64) * -(-shape[1] // 4) * -(-shape[0] // 4) * (cout // 16)
    assert nwg >= 2048
    x = _bf(rng, *shape, cin)
    w = _bf(rng, cout, 27, cin, scale=0.2)
    b = _bf(rng, cout)
    # a negative sentinel: ReLU outputs are never below 0
    y = torch.full(shape + (ldy,), -7.0, dtype=torch.bfloat16, device="cuda")
    y32 = torch.full(shape + (cout,), -7.0, dtype=torch.float32, device="cuda")
    U.unet_conv3d_fwd(_dev_bf16(x), cin, 0, _dev_bf16(_wmat(w, cin, U.unet_kpad(cin))), _dev_f32(b), y, ldy, offy,
                      y32, shape, cin, cout, True)
    got32, gotb = _host(y32), _host(y)
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    nz, ny, nx = shape
    for z0, y0, x0 in [(0, 0, 0), (nz - 6, ny - 9, nx - 70), (9, 120, 30), (0, ny - 5, 60), (nz - 3, 2, nx - 3),
                       (20, 200, 60)]:
        dz, dy, dx = min(6, nz - z0), min(9, ny - y0), min(70, nx - x0)
        ref = C.conv3d(xp[z0:z0 + dz + 2, y0:y0 + dy + 2, x0:x0 + dx + 2], w, b, relu=True)[1:-1, 1:-1, 1:-1]
        box = (slice(z0, z0 + dz), slice(y0, y0 + dy), slice(x0, x0 + dx))
        assert np.allclose(got32[box], ref, rtol=1e-4, atol=1e-4), (z0, y0, x0)
        assert np.allclose(gotb[box][..., offy:offy + cout], ref, rtol=1e-2, atol=1e-2), (z0, y0, x0)
    # every output written (no sentinel left), the other channels untouched
    assert np.all(got32 >= 0) and np.all(gotb[..., offy:offy + cout] >= 0)
    assert np.all(gotb[..., :offy] == -7.0) and np.all(gotb[..., offy + cout:] == -7.0)
    # a second launch gives the same bits everywhere (the copies of the next planes
    # run under the products: a missing wait shows here first)
    y2 = torch.full(shape + (cout,), -7.0, dtype=torch.float32, device="cuda")
    U.unet_conv3d_fwd(_dev_bf16(x), cin, 0, _dev_bf16(_wmat(w, cin, U.unet_kpad(cin))), _dev_f32(b), y, ldy, offy,
                      y2, shape, cin, cout, True)
    assert np.array_equal(_host(y2), got32)


@pytest.mark.parametrize("shape,c1,c2,cout", [((6, 10, 70), 16, 32, 16), ((26, 258, 130), 16, 32, 32),
                                               ((4, 8, 8), 64, 128, 64)])
def test_conv3d_forward_over_a_concatenation_with_an_upsampled_tensor(U, shape, c1, c2, cout):
    """unet_conv3d_fwd_cat (the decoder's input read in place) equals unet_up_fwd into
    the rows of a concatenation followed by unet_conv3d_fwd, bit for bit, on a small
    grid, a large ragged one (the four-plane launch form) and the bottom level's
    channel counts; on the small grids also the oracle's convolution of [x, up(x2)]."""
    import torch

    rng = np.random.default_rng(c1 + c2 + shape[0])
    half = tuple(n // 2 for n in shape)
    cin = c1 + c2
    x = _bf(rng, *shape, c1)
    x2 = _bf(rng, *half, c2)
    w = _bf(rng, cout, 27, cin, scale=0.2)
    b = _bf(rng, cout)
    wd, bd = _dev_bf16(_wmat(w, cin, U.unet_kpad(cin))), _dev_f32(b)
    cat = torch.zeros(shape + (cin,), dtype=torch.bfloat16, device="cuda")
    cat[..., :c1] = _dev_bf16(x)
    U.unet_up_fwd(_dev_bf16(x2), c2, 0, cat, cin, c1, shape, c2)
    outs = []
    for fused in (False, True):
        y = torch.full(shape + (cout,), -7.0, dtype=torch.bfloat16, device="cuda")
        y32 = torch.full(shape + (cout,), -7.0, dtype=torch.float32, device="cuda")
        if fused:
            U.unet_conv3d_fwd_cat(_dev_bf16(x), c1, 0, c1, _dev_bf16(x2), c2, 0, wd, bd, y, cout, 0, y32, shape, cin,
                                  cout, True)
        else:
            U.unet_conv3d_fwd(cat, cin, 0, wd, bd, y, cout, 0, y32, shape, cin, cout, True)
        outs.append((_host(y), _host(y32)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert np.all(outs[1][1] >= 0)  # every output written (ReLU; the sentinel is negative)
    if np.prod(shape) <= 5000:
        ref = C.conv3d(np.concatenate([x, C.up(x2)], axis=-1), w, b, relu=True)
        assert np.allclose(outs[1][1], ref, rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("shape,with_base", [((6, 10, 70), True), ((26, 258, 130), False), ((98, 40, 130), True)])
def test_last_convolution_with_the_head(U, shape, with_base):
    """unet_conv3d_fwd_head equals unet_conv3d_fwd (16 -> 16, ReLU) followed by
    unet_head_fwd, bit for bit, with and without a base field, on ragged grids whose
    z runs end short; the small one also against the oracle's convolution and head."""
    import torch

    rng = np.random.default_rng(shape[0] + with_base)
    x = _bf(rng, *shape, 16)
    w = _bf(rng, 16, 27, 16, scale=0.2)
    b = _bf(rng, 16)
    hw, hb = rng.standard_normal(16), rng.standard_normal(1)
    base = rng.standard_normal(shape) if with_base else None
    xd, wd, bd = _dev_bf16(x), _dev_bf16(_wmat(w, 16, U.unet_kpad(16))), _dev_f32(b)
    hwd, hbd = _dev_f32(hw), _dev_f32(hb)
    based = _dev_f32(base) if with_base else None
    y = torch.zeros(shape + (16,), dtype=torch.bfloat16, device="cuda")
    U.unet_conv3d_fwd(xd, 16, 0, wd, bd, y, 16, 0, None, shape, 16, 16, True)
    sep = torch.zeros(shape, dtype=torch.float32, device="cuda")
    U.unet_head_fwd(y, 16, hwd, hbd, based, sep, int(np.prod(shape)), 16)
    fused = torch.full(shape, -7.0, dtype=torch.float32, device="cuda")
    U.unet_conv3d_fwd_head(xd, 16, 0, wd, bd, hwd, hbd, based, fused, shape)
    assert np.array_equal(_host(fused), _host(sep))
    if np.prod(shape) <= 5000:
        # the head reads the BF16-rounded convolution: round the oracle's the same way
        # (an FP32 sum next to a rounding boundary may round one BF16 step apart)
        yr = torch.tensor(C.conv3d(x, w, b, relu=True), dtype=torch.float32).to(torch.bfloat16).double().numpy()
        ref = yr @ hw + hb[0] + (base if with_base else 0.0)
        assert np.allclose(_host(fused), ref, rtol=1e-3, atol=0.15)


@pytest.mark.parametrize("cin,cout", [(16, 16), (48, 16), (32, 64), (192, 64)])
def test_conv3d_backward_data(U, cin, cout):
    import torch

    rng = np.random.default_rng(7 + cin)
    shape = (4, 4, 8)
    w = _bf(rng, cout, 27, cin, scale=0.2)
    dy = _bf(rng, *shape, cout)
    wt = torch.zeros(cin * U.unet_kpad(cout), dtype=torch.bfloat16, device="cuda")
    U.unet_conv3d_wtrans(_dev_bf16(_wmat(w, cin, U.unet_kpad(cin))), wt, cin, cout)
    dx = torch.zeros(shape + (cin,), dtype=torch.bfloat16, device="cuda")
    dx32 = torch.zeros(shape + (cin,), dtype=torch.float32, device="cuda")
    U.unet_conv3d_fwd(_dev_bf16(dy), cout, 0, wt, None, dx, cin, 0, dx32, shape, cout, cin, False)
    assert np.allclose(_host(dx32), C.conv3d_dgrad(dy, w), rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("cin,cout,ld,off", [(16, 16, 16, 0), (48, 32, 96, 64), (64, 128, 128, 0)])
def test_conv3d_weight_gradient(U, cin, cout, ld, off):
    import torch

    rng = np.random.default_rng(11 + cin)
    shape = (4, 6, 8)
    x = _bf(rng, *shape, cin)
    dybuf = _bf(rng, *shape, ld)
    dy = dybuf[..., off:off + cout]
    kp = U.unet_kpad(cin)
    dw = torch.zeros((cout, kp), dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    U.unet_conv3d_wgrad(_dev_bf16(x), cin, 0, _dev_bf16(dybuf), ld, off, shape, cin, cout, dw, db)
    rdw, rdb = C.conv3d_wgrad(x, dy)
    got = _host(dw)
    assert np.allclose(got[:, :27 * cin], rdw.reshape(cout, -1), rtol=1e-4, atol=1e-4)
    assert np.all(got[:, 27 * cin:] == 0)
    assert np.allclose(_host(db), rdb, rtol=1e-4, atol=1e-4)


def test_pool_up_relu(U):
    import torch

    rng = np.random.default_rng(5)
    shape, c = (4, 6, 8), 16
    x = _bf(rng, *shape, 32)
    y = torch.zeros((2, 3, 4, 16), dtype=torch.bfloat16, device="cuda")
    U.unet_pool_fwd(_dev_bf16(x), 32, 16, y, 16, 0, shape, c)
    assert np.allclose(_host(y), C.pool(x[..., 16:]), rtol=8e-3, atol=1e-3)
    # backward accumulates
    dy = _bf(rng, 2, 3, 4, c)
    base = _bf(rng, *shape, c)
    dx = _dev_bf16(base)
    U.unet_pool_bwd(_dev_bf16(dy), c, 0, dx, c, 0, shape, c)
    assert np.allclose(_host(dx), base + C.pool_bwd(dy), rtol=8e-3, atol=1e-2)
    xs = _bf(rng, 2, 3, 4, c)
    yu = torch.zeros(shape + (48,), dtype=torch.bfloat16, device="cuda")
    U.unet_up_fwd(_dev_bf16(xs), c, 0, yu, 48, 16, shape, c)
    assert np.array_equal(_host(yu)[..., 16:32], C.up(xs))
    dyu = _bf(rng, *shape, 48)
    dxs = torch.zeros((2, 3, 4, c), dtype=torch.bfloat16, device="cuda")
    U.unet_up_bwd(_dev_bf16(dyu), 48, 32, dxs, c, 0, shape, c)
    assert np.allclose(_host(dxs), C.up_bwd(dyu[..., 32:]), rtol=8e-3, atol=1e-2)
    # ReLU backward zeroes the gradient where the output is not positive
    yv = _bf(rng, 10, c)
    d = _bf(rng, 10, c)
    dd = _dev_bf16(d)
    U.unet_relu_bwd(_dev_bf16(yv), c, 0, dd, c, 0, 10, c)
    assert np.array_equal(_host(dd), np.where(yv > 0, d, 0.0))


def test_head_mse_adam(U):
    import torch

    rng = np.random.default_rng(9)
    nvox, c = 500, 16
    x = _bf(rng, nvox, c)
    w, b = rng.standard_normal(c), rng.standard_normal(1)
    base = rng.standard_normal(nvox)
    out = torch.zeros(nvox, dtype=torch.float32, device="cuda")
    U.unet_head_fwd(_dev_bf16(x), c, _dev_f32(w), _dev_f32(b), _dev_f32(base), out, nvox, c)
    ref = x @ w + b[0] + base
    assert np.allclose(_host(out), ref, rtol=1e-5, atol=1e-4)
    dout = rng.standard_normal(nvox)
    dx = torch.zeros((nvox, c), dtype=torch.bfloat16, device="cuda")
    dw = torch.zeros(c, dtype=torch.float32, device="cuda")
    db = torch.zeros(1, dtype=torch.float32, device="cuda")
    U.unet_head_bwd(_dev_bf16(x), c, _dev_f32(w), _dev_f32(dout), dx, dw, db, nvox, c)
    douf = dout.astype(np.float32).astype(np.float64)
    assert np.allclose(_host(dw), x.T @ douf, rtol=1e-4, atol=1e-4)
    assert _host(db)[0] == pytest.approx(douf.sum(), rel=1e-4, abs=1e-4)
    assert np.allclose(_host(dx), np.outer(douf, w), rtol=1e-2, atol=1e-2)
    # masked MSE
    pred, tgt = rng.standard_normal(nvox), rng.standard_normal(nvox)
    mask = (rng.random(nvox) < 0.7).astype(np.uint8)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    g = torch.zeros(nvox, dtype=torch.float32, device="cuda")
    U.unet_mse(_dev_f32(pred), _dev_f32(tgt), torch.tensor(mask).cuda(), g, loss, nvox, int(mask.sum()))
    rl, rg = C.mse(pred, tgt, mask)
    assert _host(loss)[0] == pytest.approx(rl, rel=1e-5)
    assert np.allclose(_host(g), rg, rtol=1e-5, atol=1e-7)
    wt = rng.random(nvox) * 4
    loss.zero_()
    U.unet_mse(_dev_f32(pred), _dev_f32(tgt), torch.tensor(mask).cuda(), g, loss, nvox, int(mask.sum()), _dev_f32(wt))
    rl, rg = C.mse(pred, tgt, mask, wt.astype(np.float32).astype(np.float64))
    assert _host(loss)[0] == pytest.approx(rl, rel=1e-5)
    assert np.allclose(_host(g), rg, rtol=1e-5, atol=1e-7)
    # Adam: two steps against the oracle
    n = 1000
    p0, g1, g2 = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
    p, m, v = _dev_f32(p0), _dev_f32(np.zeros(n)), _dev_f32(np.zeros(n))
    pb = torch.zeros(n, dtype=torch.bfloat16, device="cuda")
    rp, rm, rv = p0, np.zeros(n), np.zeros(n)
    for t, gg in ((1, g1), (2, g2)):
        U.unet_adam(p, m, v, _dev_f32(gg), pb, n, 1e-2, 0.9, 0.999, 1e-8, t)
        rp, rm, rv = C.adam(rp, rm, rv, gg.astype(np.float32).astype(np.float64), t, 1e-2)
    assert np.allclose(_host(p), rp, rtol=1e-5, atol=1e-6)
    assert np.allclose(_host(pb), rp, rtol=1e-2, atol=1e-2)


def test_features(U):
    import torch

    rng = np.random.default_rng(3)
    shape = (3, 4, 10)
    act = (rng.random(shape) < 0.6).astype(np.uint8)
    ncat = rng.integers(0, 7, shape).astype(np.uint8)
    tau = 0.5 + rng.random(shape) * 0.5 + 1e-3
    om = np.where(act, 1 / tau, 0).astype(np.float32)
    feat = torch.zeros(shape + (16,), dtype=torch.bfloat16, device="cuda")
    wt = torch.full(shape, -1.0, dtype=torch.float32, device="cuda")
    U.unet_features(torch.tensor(act).cuda(), torch.tensor(ncat).cuda(), _dev_f32(om), 1.0, feat, shape, wt, 0.5, 8.0)
    f = _host(feat)
    t32 = 1.0 / om.astype(np.float64)
    drel = np.maximum((t32 - 0.5) / 0.5, 1e-9)
    want1 = np.where(act, np.log10(drel) / 3, 0)
    x = np.arange(10, dtype=np.float64)
    assert np.array_equal(f[..., 0], act.astype(float))
    assert np.allclose(f[..., 1], want1, atol=1e-2)
    assert np.allclose(f[..., 2], np.where(act, ncat / 6, 0), atol=1e-2)
    for c, prof in ((3, np.exp(-x / 24)), (4, np.exp(-x / 96)), (5, np.exp(-(9 - x) / 24))):
        assert np.allclose(f[..., c], np.broadcast_to(prof, shape), rtol=1e-2, atol=1e-3)
    assert np.all(f[..., 6:] == 0)
    assert np.allclose(_host(wt), np.where(act, np.minimum(8.0, np.sqrt(1 / drel)), 0), rtol=1e-5)
    U.unet_features(torch.tensor(act).cuda(), torch.tensor(ncat).cuda(), _dev_f32(om), 1.0, feat, shape, wt, 1.0, 3.0)
    assert np.allclose(_host(wt), np.where(act, np.minimum(3.0, 1 / drel), 0), rtol=1e-5)


def _oracle_params(net):
    """The network's parameters as the FP64 oracle network takes them (convolution
    weights rounded to BF16, as the kernels read them)."""
    import torch

    P = {}
    for name, cin, cout in net.specs:
        wb = net.W[name].to(torch.bfloat16).to(torch.float64).cpu().numpy()[:, :27 * cin].reshape(cout, 27, cin)
        P[name] = (wb, net.B[name].cpu().numpy().astype(np.float64))
    P["head"] = (net.W["head"].cpu().numpy().astype(np.float64), float(net.B["head"].cpu().numpy()[0]))
    return P


def test_network_gradient_matches_finite_differences(U):
    """The whole backward pass of the BF16 network (unet_forward, unet_backward of
    one library handle) against FP64 finite differences of the oracle network along
    two directions per layer checked."""
    import torch

    rng = np.random.default_rng(1)
    shape = (8, 8, 8)
    net = U.UNet(seed=3)
    feat = _bf(rng, *shape, 16)
    feat[..., 4:] = 0
    target = rng.standard_normal(shape) * 0.1
    mask = (rng.random(shape) < 0.7).astype(np.uint8)
    count = int(mask.sum())
    fd_t = _dev_bf16(feat.reshape(-1, 16))
    pred = net.forward(fd_t, shape, train=True)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    g_out = torch.zeros(pred.numel(), dtype=torch.float32, device="cuda")
    U.unet_mse(pred, _dev_f32(target.ravel()), torch.tensor(mask.ravel()).cuda(), g_out, loss, pred.numel(), count)
    net.backward(fd_t, g_out, shape)
    grads = net.grads(shape)
    torch.cuda.synchronize()

    P = _oracle_params(net)
    ref_pred = C.unet_forward(P, feat)
    assert np.allclose(_host(pred).reshape(shape), ref_pred, rtol=5e-2, atol=5e-2 * np.abs(ref_pred).max())

    def L(Pp):
        return C.mse(C.unet_forward(Pp, feat), target, mask)[0]

    for name in ("e1a", "e2b", "b4b", "d3a", "d1b"):
        cin = dict((n, c) for n, c, _ in net.specs)[name]
        wo, wc, bo, cout = net._layout[name]
        g = grads[wo:wo + wc].view(cout, -1).cpu().numpy().astype(np.float64)[:, :27 * cin]
        g = g.reshape(P[name][0].shape)
        for d in (g / np.linalg.norm(g), rng.standard_normal(g.shape)):
            d = d / np.linalg.norm(d)
            eps = 1e-3
            Pp = dict(P)
            Pm = dict(P)
            Pp[name] = (P[name][0] + eps * d, P[name][1])
            Pm[name] = (P[name][0] - eps * d, P[name][1])
            fd = (L(Pp) - L(Pm)) / (2 * eps)
            an = float(np.sum(g * d))
            assert an == pytest.approx(fd, rel=0.15, abs=0.05 * np.linalg.norm(g)), (name, an, fd)


def test_network_forward_matches_the_oracle_network(U):
    """unet_forward of a 16 x 24 x 32 handle (three poolings, every level ragged in
    channels and sizes) against the FP64 oracle network on the same BF16 inputs and
    weights; the handle's own buffers (unet_features_buffer) give the same result."""
    import torch

    rng = np.random.default_rng(21)
    shape = (16, 24, 32)
    net = U.UNet(seed=5)
    net.B["e2a"].copy_(torch.linspace(-0.1, 0.1, 32))  # nonzero biases reach the output
    net.B["head"].fill_(0.25)
    net.touch()
    feat = _bf(rng, *shape, 16)
    base = rng.standard_normal(shape).astype(np.float32)
    out = net.forward(_dev_bf16(feat.reshape(-1, 16)), shape, base=_dev_f32(base.ravel()))
    ref = C.unet_forward(_oracle_params(net), feat) + base
    err = np.abs(_host(out).reshape(shape) - ref).max()
    assert err < 2e-2 * np.abs(ref).max(), err


def test_predict_is_features_forward_and_inverse_target(U):
    """unet_predict on device solver fields equals unet_features + unet_forward +
    the inverse target map called one by one, for the log target with and without
    a depth mask and for the corrector target."""
    import torch

    rng = np.random.default_rng(22)
    shape = (8, 16, 24)
    act = (rng.random(shape) < 0.6).astype(np.uint8)
    ncat = np.where(act, rng.integers(0, 4, shape), 0).astype(np.uint8)
    tau = np.where(act, 0.5 + 0.5 * 10 ** rng.uniform(-3, 0, shape), 1.0)
    om = np.where(act, 1.0 / tau, 0.0).astype(np.float32)
    depth = rng.integers(0, 8, shape).astype(np.uint8)
    a, n, o, d = (torch.tensor(v).cuda() for v in (act, ncat, om, depth))
    net = U.UNet(seed=6)
    feat = torch.empty((int(np.prod(shape)), 16), dtype=torch.bfloat16, device="cuda")
    U.unet_features(a, n, o, 1.0, feat, shape)
    y = net.forward(feat, shape)
    V = y.numel()
    for kind, dep in ((U.UNET_TARGET_LOG, None), (U.UNET_TARGET_LOG, d), (U.UNET_TARGET_CORRECTOR, None)):
        tgt = U.unet_target(kind=kind, eps=1e-3, cmax=1.5, c_in=1.0, c_out=0.0,
                            depth=dep.data_ptr() if dep is not None else None, depth_max=3)
        got = net.predict(a, n, o, 1.0, tgt)
        want = torch.empty(V, dtype=torch.float32, device="cuda")
        if kind == U.UNET_TARGET_CORRECTOR:
            U.unet_corrector_map(y, want, V, shape[2], 1.0, 0.0, True, 1.5)
        elif dep is not None:
            U.unet_start_field(y, dep, 3, 1e-3, 1.5, want, V)
        else:
            U.unet_log_map(y, want, V, 1e-3, True, 1.5)
        torch.cuda.synchronize()
        assert torch.equal(got.view(-1), want), kind


def test_train_step_is_forward_backward_adam(U):
    """unet_train_step equals unet_forward, unet_mse, unet_backward and
    unet_adam_step called one by one (two networks from the same parameters).

    The weight gradients and the loss are sums over voxels that thread blocks add
    with FP32 atomics, so their last bits depend on the order the blocks finish in
    and two runs need not be bit-identical.  Adam turns a gradient into a step of
    +-lr whatever its size, so a rounding-level difference moves a parameter by
    rounding only, except where the gradient itself is at rounding level and its
    sign can flip: almost every parameter must agree to 1e-7, and none may differ by
    more than two steps."""
    import torch

    rng = np.random.default_rng(23)
    shape = (8, 8, 16)
    feat = _dev_bf16(_bf(rng, *shape, 16).reshape(-1, 16))
    target = _dev_f32(rng.standard_normal(int(np.prod(shape))) * 0.1)
    mask = torch.tensor((rng.random(int(np.prod(shape))) < 0.8).astype(np.uint8)).cuda()
    count = int(mask.sum())
    a, b = U.UNet(seed=7), U.UNet(seed=7)
    for step in range(2):
        la = a.train_step(feat, shape, target, mask, count, 1e-3)
        pred = b.forward(feat, shape, train=True)
        lb = torch.zeros(1, dtype=torch.float32, device="cuda")
        g = torch.zeros_like(pred)
        U.unet_mse(pred, target, mask, g, lb, pred.numel(), count)
        b.backward(feat, g, shape)
        b.adam_step(shape, 1e-3)
        torch.cuda.synchronize()
        assert float(la) == pytest.approx(float(lb), rel=1e-6), step
        d = (a.params - b.params).abs()
        assert float(d.max()) <= 2 * 2e-3, step
        assert float((d > 1e-7).float().mean()) < 1e-3, step
    assert a.t == b.t == 2
    # a step moved the parameters
    assert not torch.equal(a.params, U.UNet(seed=7).params)


def test_log_map_round_trip(U):
    import torch

    rng = np.random.default_rng(12)
    c = np.concatenate([rng.random(1000) * 1.3, [-0.5, 0.0, 5.0]])
    y = torch.zeros(c.size, dtype=torch.float32, device="cuda")
    U.unet_log_map(_dev_f32(c), y, c.size, 1e-3, False)
    c32 = c.astype(np.float32).astype(np.float64)
    assert np.allclose(_host(y), np.log(np.maximum(c32, 0) + 1e-3), rtol=1e-6, atol=1e-6)
    back = torch.zeros_like(y)
    U.unet_log_map(y, back, c.size, 1e-3, True, 1.5)
    assert np.allclose(_host(back), np.clip(c32, 0, 1.5), rtol=1e-5, atol=1e-6)


def test_start_field_masks_deep_voxels(U):
    import torch

    rng = np.random.default_rng(13)
    n = 3000
    y = np.log(rng.random(n) * 1.4 + 1e-3)
    depth = rng.integers(0, 6, n).astype(np.uint8)
    depth[:10] = 255
    c = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
    U.unet_start_field(_dev_f32(y), torch.tensor(depth).cuda(), 2, 1e-3, 1.2, c, n)
    y32 = y.astype(np.float32).astype(np.float64)
    want = np.where(depth <= 2, np.clip(np.exp(y32) - 1e-3, 0, 1.2), 0.0)
    assert np.allclose(_host(c), want, rtol=1e-5, atol=1e-6)


def test_corrector_map_round_trip(U):
    import torch

    rng = np.random.default_rng(14)
    nz, ny, nx = 3, 4, 20
    c = rng.random((nz, ny, nx)) * 0.9 + 0.05
    y = torch.zeros(c.size, dtype=torch.float32, device="cuda")
    U.unet_corrector_map(_dev_f32(c), y, c.size, nx, 1.0, 0.0, False)
    lin = 1.0 - (np.arange(nx) + 0.5) / nx
    c32 = c.astype(np.float32).astype(np.float64)
    assert np.allclose(_host(y).reshape(c.shape), nx * (c32 - lin), rtol=1e-5, atol=1e-5)
    back = torch.zeros_like(y)
    U.unet_corrector_map(y, back, c.size, nx, 1.0, 0.0, True, 1.5)
    assert np.allclose(_host(back).reshape(c.shape), c32, rtol=1e-5, atol=1e-6)
