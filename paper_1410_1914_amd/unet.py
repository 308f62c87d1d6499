"""Binding of include/unet.h and the warm-start network built from those kernels.

``UNet`` is a 3-D U-Net with four levels of 16, 32, 64 and 128 channels: two
3x3x3 convolutions with ReLU per level, 2x2x2 average pooling on the way down,
nearest-neighbour upsampling and channel concatenation with the skip tensor on the
way up, and a 1x1x1 output head.  Every forward and backward operation is a
kernel of ``_libunet.so`` (BF16 MFMA convolutions with FP32 accumulation, FP32
weight gradients, Adam on FP32 master weights); this module only allocates the
buffers (torch tensors on the GPU) and calls the kernels in order.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_libunet.so")

_P = ctypes.c_void_p
_i32, _i64, _f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float

SIGNATURES = {
    "unet_kpad": ([_i32], _i32),
    "unet_conv3d_fwd": ([_P, _i32, _i32, _P, _P, _P, _i32, _i32, _P, _i32, _i32, _i32, _i32, _i32, _i32, _P], _i32),
    "unet_conv3d_wtrans": ([_P, _P, _i32, _i32, _P], _i32),
    "unet_conv3d_wgrad": ([_P, _i32, _i32, _P, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _P, _P, _P], _i32),
    "unet_relu_bwd": ([_P, _i32, _i32, _P, _i32, _i32, _i64, _i32, _P], _i32),
    "unet_pool_fwd": ([_P, _i32, _i32, _P, _i32, _i32, _i32, _i32, _i32, _i32, _P], _i32),
    "unet_pool_bwd": ([_P, _i32, _i32, _P, _i32, _i32, _i32, _i32, _i32, _i32, _P], _i32),
    "unet_up_fwd": ([_P, _i32, _i32, _P, _i32, _i32, _i32, _i32, _i32, _i32, _P], _i32),
    "unet_up_bwd": ([_P, _i32, _i32, _P, _i32, _i32, _i32, _i32, _i32, _i32, _P], _i32),
    "unet_head_fwd": ([_P, _i32, _P, _P, _P, _P, _i64, _i32, _P], _i32),
    "unet_head_bwd": ([_P, _i32, _P, _P, _P, _P, _P, _i64, _i32, _P], _i32),
    "unet_mse": ([_P, _P, _P, _P, _P, _P, _i64, _i64, _P], _i32),
    "unet_adam": ([_P, _P, _P, _P, _P, _i64, _f32, _f32, _f32, _f32, _i32, _P], _i32),
    "unet_to_bf16": ([_P, _P, _i64, _P], _i32),
    "unet_zero": ([_P, _i64, _P], _i32),
    "unet_log_map": ([_P, _P, _i64, _f32, _i32, _f32, _P], _i32),
    "unet_start_field": ([_P, _P, _i32, _f32, _f32, _P, _i64, _P], _i32),
    "unet_corrector_map": ([_P, _P, _i64, _i32, _f32, _f32, _i32, _f32, _P], _i32),
    "unet_features": ([_P, _P, _P, _f32, _P, _P, _f32, _f32, _i32, _i32, _i32, _P], _i32),
    "unet_mfma_selftest": ([_P, _P, _P, _P], _i32),
}

_lib = None


def load():
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (share torch's HIP runtime)

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH} (run paper_1410_1914_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _call(name, *args):
    st = getattr(load(), name)(*args)
    if st != 0:
        raise RuntimeError(f"{name} failed with status {st}")


def _ptr(t):
    return t.data_ptr() if t is not None else None


def _stream():
    import torch

    return torch.cuda.current_stream().cuda_stream


# ------------------------------------------------------------------ thin wrappers (same names)

def unet_kpad(cin):
    return int(load().unet_kpad(cin))


def unet_conv3d_fwd(x, ldx, offx, w, b, y, ldy, offy, y32, shape, cin, cout, relu):
    nz, ny, nx = shape
    _call("unet_conv3d_fwd", _ptr(x), ldx, offx, _ptr(w), _ptr(b), _ptr(y), ldy, offy, _ptr(y32), nz, ny, nx, cin,
          cout, int(relu), _stream())


def unet_conv3d_wtrans(w, wt, cin, cout):
    _call("unet_conv3d_wtrans", _ptr(w), _ptr(wt), cin, cout, _stream())


def unet_conv3d_wgrad(x, ldx, offx, dy, lddy, offdy, shape, cin, cout, dw, db):
    nz, ny, nx = shape
    _call("unet_conv3d_wgrad", _ptr(x), ldx, offx, _ptr(dy), lddy, offdy, nz, ny, nx, cin, cout, _ptr(dw), _ptr(db),
          _stream())


def unet_relu_bwd(y, ldy, offy, d, ldd, offd, nvox, c):
    _call("unet_relu_bwd", _ptr(y), ldy, offy, _ptr(d), ldd, offd, nvox, c, _stream())


def unet_pool_fwd(x, ldx, offx, y, ldy, offy, shape, c):
    _call("unet_pool_fwd", _ptr(x), ldx, offx, _ptr(y), ldy, offy, *shape, c, _stream())


def unet_pool_bwd(dy, ldy, offy, dx, ldx, offx, shape, c):
    _call("unet_pool_bwd", _ptr(dy), ldy, offy, _ptr(dx), ldx, offx, *shape, c, _stream())


def unet_up_fwd(x, ldx, offx, y, ldy, offy, shape, c):
    _call("unet_up_fwd", _ptr(x), ldx, offx, _ptr(y), ldy, offy, *shape, c, _stream())


def unet_up_bwd(dy, ldy, offy, dx, ldx, offx, shape, c):
    _call("unet_up_bwd", _ptr(dy), ldy, offy, _ptr(dx), ldx, offx, *shape, c, _stream())


def unet_head_fwd(x, ldx, w, b, base, out, nvox, c):
    _call("unet_head_fwd", _ptr(x), ldx, _ptr(w), _ptr(b), _ptr(base), _ptr(out), nvox, c, _stream())


def unet_head_bwd(x, ldx, w, dout, dx, dw, db, nvox, c):
    _call("unet_head_bwd", _ptr(x), ldx, _ptr(w), _ptr(dout), _ptr(dx), _ptr(dw), _ptr(db), nvox, c, _stream())


def unet_mse(pred, target, mask, dout, loss, nvox, count, weight=None):
    _call("unet_mse", _ptr(pred), _ptr(target), _ptr(mask), _ptr(weight), _ptr(dout), _ptr(loss), nvox, count,
          _stream())


def unet_adam(p, m, v, g, pb, n, lr, b1, b2, eps, t):
    _call("unet_adam", _ptr(p), _ptr(m), _ptr(v), _ptr(g), _ptr(pb), n, lr, b1, b2, eps, t, _stream())


def unet_to_bf16(src, dst, n):
    _call("unet_to_bf16", _ptr(src), _ptr(dst), n, _stream())


def unet_zero(t):
    _call("unet_zero", _ptr(t), t.numel() * t.element_size(), _stream())


def unet_features(active, n_cat, omega, tau_ref, feat, shape, weight=None, weight_power=0.5, weight_cap=32.0):
    _call("unet_features", _ptr(active), _ptr(n_cat), _ptr(omega), tau_ref, _ptr(feat), _ptr(weight), weight_power,
          weight_cap, *shape, _stream())


def unet_log_map(src, dst, n, eps, inverse, cmax=2.0):
    _call("unet_log_map", _ptr(src), _ptr(dst), n, eps, 1 if inverse else 0, cmax, _stream())


def unet_start_field(y, depth, depth_max, eps, cmax, c, n):
    _call("unet_start_field", _ptr(y), _ptr(depth), depth_max, eps, cmax, _ptr(c), n, _stream())


def unet_corrector_map(src, dst, nvox, nx, c_in, c_out, inverse, cmax=2.0):
    _call("unet_corrector_map", _ptr(src), _ptr(dst), nvox, nx, c_in, c_out, 1 if inverse else 0, cmax, _stream())


def unet_mfma_selftest(a, b, d):
    _call("unet_mfma_selftest", _ptr(a), _ptr(b), _ptr(d), _stream())


# ------------------------------------------------------------------ the network

IN_CH = 16
LEVELS = (16, 32, 64, 128)


def layer_specs():
    """(name, cin, cout) of every 3x3x3 convolution, in forward order."""
    c1, c2, c3, c4 = LEVELS
    return [("e1a", IN_CH, c1), ("e1b", c1, c1), ("e2a", c1, c2), ("e2b", c2, c2),
            ("e3a", c2, c3), ("e3b", c3, c3), ("b4a", c3, c4), ("b4b", c4, c4),
            ("d3a", c4 + c3, c3), ("d3b", c3, c3), ("d2a", c3 + c2, c2), ("d2b", c2, c2),
            ("d1a", c2 + c1, c1), ("d1b", c1, c1)]


def conv_flops(shape):
    """Multiply-add flops (2 per MAC) of the 3x3x3 convolutions of one forward pass
    on a (nz, ny, nx) grid; the backward pass costs about twice that (data and
    weight gradients)."""
    level = {"e1": 0, "d1": 0, "e2": 1, "d2": 1, "e3": 2, "d3": 2, "b4": 3}
    vox = [int(np.prod([s // (2 ** l) for s in shape])) for l in range(4)]
    return sum(2 * 27 * cin * cout * vox[level[name[:2]]] for name, cin, cout in layer_specs())


class UNet:
    """Parameters (FP32 masters + BF16 copies, Adam moments) and forward/backward."""

    def __init__(self, device="cuda", seed=0):
        import torch

        load()
        self.device = torch.device(device)
        self.specs = layer_specs()
        rng = np.random.default_rng(seed)
        self.W, self.B, self.Wb = {}, {}, {}
        for name, cin, cout in self.specs:
            kp = unet_kpad(cin)
            w = np.zeros((cout, kp), np.float32)
            w[:, :27 * cin] = rng.normal(0.0, np.sqrt(2.0 / (27 * cin)), (cout, 27 * cin))
            self.W[name] = torch.from_numpy(w).to(self.device)
            self.B[name] = torch.zeros(cout, dtype=torch.float32, device=self.device)
        c1 = LEVELS[0]
        self.W["head"] = torch.from_numpy(rng.normal(0.0, 0.1 / np.sqrt(c1), c1).astype(np.float32)).to(self.device)
        self.B["head"] = torch.zeros(1, dtype=torch.float32, device=self.device)
        self._sync_bf16()
        self.m = {k: torch.zeros_like(v) for k, v in self.W.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.W.items()}
        self.mb = {k: torch.zeros_like(v) for k, v in self.B.items()}
        self.vb = {k: torch.zeros_like(v) for k, v in self.B.items()}
        self.t = 0
        self.target_eps = 0.0  # > 0: the network predicts ln(C + target_eps) instead of C
        self._bufs = None

    # parameters -------------------------------------------------------------
    def _sync_bf16(self):
        import torch

        for name, _, _ in self.specs:
            wb = torch.empty(self.W[name].shape, dtype=torch.bfloat16, device=self.device)
            unet_to_bf16(self.W[name], wb, wb.numel())
            self.Wb[name] = wb

    def state_dict(self):
        d = {f"W_{k}": v.cpu().numpy() for k, v in self.W.items()}
        d.update({f"B_{k}": v.cpu().numpy() for k, v in self.B.items()})
        d["target_eps"] = np.array(self.target_eps, np.float64)
        return d

    def load_state_dict(self, d):
        import torch

        for k in self.W:
            self.W[k] = torch.from_numpy(np.asarray(d[f"W_{k}"], np.float32)).to(self.device)
            self.B[k] = torch.from_numpy(np.asarray(d[f"B_{k}"], np.float32)).to(self.device)
        self.target_eps = float(d["target_eps"]) if "target_eps" in d else 0.0
        self._sync_bf16()

    def save(self, path):
        np.savez(path, **self.state_dict())

    @classmethod
    def from_file(cls, path, device="cuda"):
        net = cls(device)
        with np.load(path, allow_pickle=False) as d:
            net.load_state_dict({k: d[k] for k in d.files})
        return net

    def n_params(self):
        return sum(int(27 * cin * cout + cout) for _, cin, cout in self.specs) + LEVELS[0] + 1

    # buffers ----------------------------------------------------------------
    def _alloc(self, shape, train):
        import torch

        key = (tuple(shape), train)
        if self._bufs is not None and self._bufs["key"] == key:
            return self._bufs
        for s in shape:
            if s % 8:
                raise ValueError("grid sizes must be multiples of 8 (three 2x poolings)")
        c1, c2, c3, c4 = LEVELS
        dims = [tuple(shape), tuple(s // 2 for s in shape), tuple(s // 4 for s in shape), tuple(s // 8 for s in shape)]
        V = [int(np.prod(d)) for d in dims]
        bf = lambda v, c: torch.zeros((v, c), dtype=torch.bfloat16, device=self.device)  # noqa: E731
        b = {"key": key, "dims": dims, "V": V,
             "a1": bf(V[0], c1), "cat1": bf(V[0], c1 + c2), "d1a": bf(V[0], c1), "d1b": bf(V[0], c1),
             "p2": bf(V[1], c1), "a2": bf(V[1], c2), "cat2": bf(V[1], c2 + c3), "d2a": bf(V[1], c2), "d2b": bf(V[1], c2),
             "p3": bf(V[2], c2), "a3": bf(V[2], c3), "cat3": bf(V[2], c3 + c4), "d3a": bf(V[2], c3), "d3b": bf(V[2], c3),
             "p4": bf(V[3], c3), "b4a": bf(V[3], c4), "b4b": bf(V[3], c4),
             "out": torch.zeros(V[0], dtype=torch.float32, device=self.device)}
        if train:
            for k in list(b):
                if isinstance(b[k], torch.Tensor) and b[k].dtype == torch.bfloat16:
                    b["g_" + k] = torch.zeros_like(b[k])
            b["g_out"] = torch.zeros(V[0], dtype=torch.float32, device=self.device)
            b["wt"] = torch.zeros(max(cin * unet_kpad(cout) for _, cin, cout in self.specs), dtype=torch.bfloat16,
                                  device=self.device)
            self.gW = {k: torch.zeros_like(v) for k, v in self.W.items()}
            self.gB = {k: torch.zeros_like(v) for k, v in self.B.items()}
            b["loss"] = torch.zeros(1, dtype=torch.float32, device=self.device)
        self._bufs = b
        return b

    # forward ----------------------------------------------------------------
    def _conv(self, name, x, ldx, offx, y, ldy, offy, dims, cin, cout, relu=True):
        unet_conv3d_fwd(x, ldx, offx, self.Wb[name], self.B[name], y, ldy, offy, None, dims, cin, cout, relu)

    def forward(self, feat, shape, train=False, base=None):
        """feat: (V, 16) BF16 features on `shape`; returns the FP32 prediction (V,)."""
        b = self._alloc(shape, train)
        c1, c2, c3, c4 = LEVELS
        d0, d1, d2, d3 = b["dims"]
        self._conv("e1a", feat, IN_CH, 0, b["a1"], c1, 0, d0, IN_CH, c1)
        self._conv("e1b", b["a1"], c1, 0, b["cat1"], c1 + c2, 0, d0, c1, c1)
        unet_pool_fwd(b["cat1"], c1 + c2, 0, b["p2"], c1, 0, d0, c1)
        self._conv("e2a", b["p2"], c1, 0, b["a2"], c2, 0, d1, c1, c2)
        self._conv("e2b", b["a2"], c2, 0, b["cat2"], c2 + c3, 0, d1, c2, c2)
        unet_pool_fwd(b["cat2"], c2 + c3, 0, b["p3"], c2, 0, d1, c2)
        self._conv("e3a", b["p3"], c2, 0, b["a3"], c3, 0, d2, c2, c3)
        self._conv("e3b", b["a3"], c3, 0, b["cat3"], c3 + c4, 0, d2, c3, c3)
        unet_pool_fwd(b["cat3"], c3 + c4, 0, b["p4"], c3, 0, d2, c3)
        self._conv("b4a", b["p4"], c3, 0, b["b4a"], c4, 0, d3, c3, c4)
        self._conv("b4b", b["b4a"], c4, 0, b["b4b"], c4, 0, d3, c4, c4)
        unet_up_fwd(b["b4b"], c4, 0, b["cat3"], c3 + c4, c3, d2, c4)
        self._conv("d3a", b["cat3"], c3 + c4, 0, b["d3a"], c3, 0, d2, c3 + c4, c3)
        self._conv("d3b", b["d3a"], c3, 0, b["d3b"], c3, 0, d2, c3, c3)
        unet_up_fwd(b["d3b"], c3, 0, b["cat2"], c2 + c3, c2, d1, c3)
        self._conv("d2a", b["cat2"], c2 + c3, 0, b["d2a"], c2, 0, d1, c2 + c3, c2)
        self._conv("d2b", b["d2a"], c2, 0, b["d2b"], c2, 0, d1, c2, c2)
        unet_up_fwd(b["d2b"], c2, 0, b["cat1"], c1 + c2, c1, d0, c2)
        self._conv("d1a", b["cat1"], c1 + c2, 0, b["d1a"], c1, 0, d0, c1 + c2, c1)
        self._conv("d1b", b["d1a"], c1, 0, b["d1b"], c1, 0, d0, c1, c1)
        unet_head_fwd(b["d1b"], c1, self.W["head"], self.B["head"], base, b["out"], b["V"][0], c1)
        return b["out"]

    # backward ---------------------------------------------------------------
    def _conv_bwd(self, name, x, ldx, offx, y, ldy, offy, gy, ldg, offg, gx, ldgx, offgx, dims, cin, cout):
        """gy holds dL/dy (post-ReLU) at [offg, offg+cout); overwritten with dL/dpre.
        Accumulates weight and bias gradients; writes dL/dx into gx when given."""
        b = self._bufs
        nv = int(np.prod(dims))
        unet_relu_bwd(y, ldy, offy, gy, ldg, offg, nv, cout)
        unet_conv3d_wgrad(x, ldx, offx, gy, ldg, offg, dims, cin, cout, self.gW[name], self.gB[name])
        if gx is not None:
            unet_conv3d_wtrans(self.Wb[name], b["wt"], cin, cout)
            unet_conv3d_fwd(gy, ldg, offg, b["wt"], None, gx, ldgx, offgx, None, dims, cout, cin, False)

    def backward(self, feat, dout):
        b = self._bufs
        c1, c2, c3, c4 = LEVELS
        d0, d1, d2, d3 = b["dims"]
        for k in self.gW:
            unet_zero(self.gW[k])
            unet_zero(self.gB[k])
        for k in ("g_cat1", "g_cat2", "g_cat3"):
            unet_zero(b[k])
        unet_head_bwd(b["d1b"], c1, self.W["head"], dout, b["g_d1b"], self.gW["head"], self.gB["head"], b["V"][0], c1)
        self._conv_bwd("d1b", b["d1a"], c1, 0, b["d1b"], c1, 0, b["g_d1b"], c1, 0, b["g_d1a"], c1, 0, d0, c1, c1)
        self._conv_bwd("d1a", b["cat1"], c1 + c2, 0, b["d1a"], c1, 0, b["g_d1a"], c1, 0, b["g_cat1"], c1 + c2, 0, d0,
                       c1 + c2, c1)
        unet_up_bwd(b["g_cat1"], c1 + c2, c1, b["g_d2b"], c2, 0, d0, c2)
        self._conv_bwd("d2b", b["d2a"], c2, 0, b["d2b"], c2, 0, b["g_d2b"], c2, 0, b["g_d2a"], c2, 0, d1, c2, c2)
        self._conv_bwd("d2a", b["cat2"], c2 + c3, 0, b["d2a"], c2, 0, b["g_d2a"], c2, 0, b["g_cat2"], c2 + c3, 0, d1,
                       c2 + c3, c2)
        unet_up_bwd(b["g_cat2"], c2 + c3, c2, b["g_d3b"], c3, 0, d1, c3)
        self._conv_bwd("d3b", b["d3a"], c3, 0, b["d3b"], c3, 0, b["g_d3b"], c3, 0, b["g_d3a"], c3, 0, d2, c3, c3)
        self._conv_bwd("d3a", b["cat3"], c3 + c4, 0, b["d3a"], c3, 0, b["g_d3a"], c3, 0, b["g_cat3"], c3 + c4, 0, d2,
                       c3 + c4, c3)
        unet_up_bwd(b["g_cat3"], c3 + c4, c3, b["g_b4b"], c4, 0, d2, c4)
        self._conv_bwd("b4b", b["b4a"], c4, 0, b["b4b"], c4, 0, b["g_b4b"], c4, 0, b["g_b4a"], c4, 0, d3, c4, c4)
        self._conv_bwd("b4a", b["p4"], c3, 0, b["b4a"], c4, 0, b["g_b4a"], c4, 0, b["g_p4"], c3, 0, d3, c3, c4)
        unet_pool_bwd(b["g_p4"], c3, 0, b["g_cat3"], c3 + c4, 0, d2, c3)
        self._conv_bwd("e3b", b["a3"], c3, 0, b["cat3"], c3 + c4, 0, b["g_cat3"], c3 + c4, 0, b["g_a3"], c3, 0, d2, c3, c3)
        self._conv_bwd("e3a", b["p3"], c2, 0, b["a3"], c3, 0, b["g_a3"], c3, 0, b["g_p3"], c2, 0, d2, c2, c3)
        unet_pool_bwd(b["g_p3"], c2, 0, b["g_cat2"], c2 + c3, 0, d1, c2)
        self._conv_bwd("e2b", b["a2"], c2, 0, b["cat2"], c2 + c3, 0, b["g_cat2"], c2 + c3, 0, b["g_a2"], c2, 0, d1, c2, c2)
        self._conv_bwd("e2a", b["p2"], c1, 0, b["a2"], c2, 0, b["g_a2"], c2, 0, b["g_p2"], c1, 0, d1, c1, c2)
        unet_pool_bwd(b["g_p2"], c1, 0, b["g_cat1"], c1 + c2, 0, d0, c1)
        self._conv_bwd("e1b", b["a1"], c1, 0, b["cat1"], c1 + c2, 0, b["g_cat1"], c1 + c2, 0, b["g_a1"], c1, 0, d0, c1, c1)
        self._conv_bwd("e1a", feat, IN_CH, 0, b["a1"], c1, 0, b["g_a1"], c1, 0, None, 0, 0, d0, IN_CH, c1)

    def adam_step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        for k in self.W:
            wb = self.Wb.get(k)
            unet_adam(self.W[k], self.m[k], self.v[k], self.gW[k], wb, self.W[k].numel(), lr, b1, b2, eps, self.t)
            unet_adam(self.B[k], self.mb[k], self.vb[k], self.gB[k], None, self.B[k].numel(), lr, b1, b2, eps, self.t)

    def train_step(self, feat, shape, target, mask, count, lr, weight=None):
        """One Adam step on the (weighted) masked MSE between the prediction and target."""
        b = self._alloc(shape, True)
        pred = self.forward(feat, shape, train=True)
        unet_zero(b["loss"])
        unet_mse(pred, target, mask, b["g_out"], b["loss"], b["V"][0], count, weight)
        self.backward(feat, b["g_out"])
        self.adam_step(lr)
        return b["loss"]
