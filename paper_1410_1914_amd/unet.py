"""Binding of include/unet.h and the warm-start network.

The network is the library's ``unet_net`` object: a 3-D U-Net with four levels of
16, 32, 64 and 128 channels (two 3x3x3 convolutions with ReLU per level, 2x2x2
average pooling on the way down, nearest-neighbour upsampling and channel
concatenation with the skip tensor on the way up, a 1x1x1 output head) whose
forward pass, backward pass, Adam step and prediction are single C calls running
the kernels of ``_libunet.so`` (BF16 MFMA convolutions with FP32 accumulation,
FP32 weight gradients, Adam on FP32 master weights).  ``UNet`` holds the flat
parameter array and the torch-owned workspaces of its handles; the layer wrappers
below expose the individual kernels with the same names as the C calls.
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
    "unet_conv3d_fwd_head": ([_P, _i32, _i32, _P, _P, _P, _P, _P, _P, _i32, _i32, _i32, _P], _i32),
    "unet_conv3d_fwd_cat": ([_P, _i32, _i32, _i32, _P, _i32, _i32, _P, _P, _P, _i32, _i32, _P, _i32, _i32, _i32, _i32,
                             _i32, _i32, _P], _i32),
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
    "unet_param_count": ([], _i64),
    "unet_param_tensor": ([_i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                           ctypes.POINTER(_i64), ctypes.POINTER(_i64)], _i32),
    "unet_create": ([_i32, _i32, _i32, _i32, ctypes.POINTER(_P)], _i32),
    "unet_workspace_bytes": ([_P, ctypes.POINTER(ctypes.c_size_t)], _i32),
    "unet_bind": ([_P, _P, ctypes.c_size_t, _P], _i32),
    "unet_set_params": ([_P, _P], _i32),
    "unet_get_params": ([_P, _P, _P], _i32),
    "unet_forward": ([_P, _P, _P, _P], _i32),
    "unet_backward": ([_P, _P, _P], _i32),
    "unet_adam_step": ([_P, _f32, _f32, _f32, _f32], _i32),
    "unet_train_step": ([_P, _P, _P, _P, _P, _i64, _f32, _P], _i32),
    "unet_predict": ([_P, _P, _P, _P, _f32, ctypes.c_void_p, _P], _i32),
    "unet_features_buffer": ([_P, ctypes.POINTER(_P), ctypes.POINTER(_P)], _i32),
    "unet_destroy": ([_P], None),
}

UNET_TARGET_LOG, UNET_TARGET_CORRECTOR, UNET_TARGET_PLAIN = 0, 1, 2


class unet_target(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("kind", _i32), ("eps", _f32), ("cmax", _f32),
                ("c_in", _f32), ("c_out", _f32), ("depth", _P), ("depth_max", _i32)]

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


def unet_conv3d_fwd_cat(x, ldx, offx, cin1, x2, ldx2, offx2, w, b, y, ldy, offy, y32, shape, cin, cout, relu):
    nz, ny, nx = shape
    _call("unet_conv3d_fwd_cat", _ptr(x), ldx, offx, cin1, _ptr(x2), ldx2, offx2, _ptr(w), _ptr(b), _ptr(y), ldy, offy,
          _ptr(y32), nz, ny, nx, cin, cout, int(relu), _stream())


def unet_conv3d_fwd_head(x, ldx, offx, w, b, hw, hb, base, out, shape):
    nz, ny, nx = shape
    _call("unet_conv3d_fwd_head", _ptr(x), ldx, offx, _ptr(w), _ptr(b), _ptr(hw), _ptr(hb), _ptr(base), _ptr(out),
          nz, ny, nx, _stream())


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


def param_count():
    return int(load().unet_param_count())


def param_tensor(t):
    """(cin, cout, w_offset, w_count, b_offset) of parameter tensor t of the flat array
    (0..13 the convolutions in forward order, 14 the head)."""
    cin, cout = _i32(), _i32()
    wo, wc, bo = _i64(), _i64(), _i64()
    _call("unet_param_tensor", t, ctypes.byref(cin), ctypes.byref(cout), ctypes.byref(wo), ctypes.byref(wc),
          ctypes.byref(bo))
    return cin.value, cout.value, wo.value, wc.value, bo.value


class _Handle:
    """One unet_net handle bound to a torch-owned workspace (a grid and a mode)."""

    def __init__(self, shape, train, device):
        import torch

        h = _P()
        _call("unet_create", int(shape[0]), int(shape[1]), int(shape[2]), 1 if train else 0, ctypes.byref(h))
        self.h = h
        nb = ctypes.c_size_t()
        _call("unet_workspace_bytes", self.h, ctypes.byref(nb))
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        _call("unet_bind", self.h, ptr, nb.value, _stream())
        self.version = -1
        self.shape, self.train = tuple(shape), train

    def close(self):
        if self.h:
            load().unet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class UNet:
    """The warm-start network of include/unet.h (unet_net): parameters in one flat
    FP32 device array (``params``; ``W`` and ``B`` are views of it per tensor), and
    one library handle per grid and mode, created on first use.  Forward, backward,
    the Adam step and prediction are single ABI calls; this class only allocates
    the workspaces and keeps the handles' parameters current."""

    def __init__(self, device="cuda", seed=0):
        import torch

        load()
        self.device = torch.device(device)
        self.specs = layer_specs()
        self.params = torch.zeros(param_count(), dtype=torch.float32, device=self.device)
        self.W, self.B = {}, {}
        self._layout = {}
        for t, (name, cin, cout) in enumerate(self.specs + [("head", LEVELS[0], 1)]):
            ci, co, wo, wc, bo = param_tensor(t)
            assert (ci, co) == (cin, cout), (name, ci, co)
            self._layout[name] = (wo, wc, bo, co)
            self.W[name] = self.params[wo:wo + wc].view(cout, -1) if name != "head" else self.params[wo:wo + wc]
            self.B[name] = self.params[bo:bo + co]
        rng = np.random.default_rng(seed)
        host = np.zeros(self.params.numel(), np.float32)
        for name, cin, cout in self.specs:
            wo, wc, bo, _ = self._layout[name]
            kp = wc // cout
            w = np.zeros((cout, kp), np.float32)
            w[:, :27 * cin] = rng.normal(0.0, np.sqrt(2.0 / (27 * cin)), (cout, 27 * cin))
            host[wo:wo + wc] = w.ravel()
        c1 = LEVELS[0]
        wo, wc, _, _ = self._layout["head"]
        host[wo:wo + wc] = rng.normal(0.0, 0.1 / np.sqrt(c1), c1).astype(np.float32)
        self.params.copy_(torch.from_numpy(host))
        self.version = 0  # bumped whenever the parameters change
        self.t = 0
        self.target_eps = 0.0  # > 0: the network predicts ln(C + target_eps) instead of C
        self._handles = {}

    # parameters -------------------------------------------------------------
    def touch(self):
        """Call after changing ``params`` (or a W / B view) in place."""
        self.version += 1

    def state_dict(self):
        d = {f"W_{k}": v.cpu().numpy() for k, v in self.W.items()}
        d.update({f"B_{k}": v.cpu().numpy() for k, v in self.B.items()})
        d["target_eps"] = np.array(self.target_eps, np.float64)
        return d

    def load_state_dict(self, d):
        import torch

        for k in self.W:
            self.W[k].copy_(torch.from_numpy(np.asarray(d[f"W_{k}"], np.float32).reshape(self.W[k].shape)))
            self.B[k].copy_(torch.from_numpy(np.asarray(d[f"B_{k}"], np.float32).reshape(self.B[k].shape)))
        self.target_eps = float(d["target_eps"]) if "target_eps" in d else 0.0
        self.touch()

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

    # handles ----------------------------------------------------------------
    def handle(self, shape, train=False):
        """The bound handle for a grid (created on first use) with current parameters."""
        import torch

        key = (tuple(int(s) for s in shape), bool(train))
        for s in key[0]:
            if s % 8:
                raise ValueError("grid sizes must be multiples of 8 (three 2x poolings)")
        h = self._handles.get(key)
        if h is None:
            h = _Handle(key[0], key[1], self.device)
            self._handles[key] = h
        if h.version != self.version:
            torch.cuda.current_stream(self.device).synchronize()
            _call("unet_set_params", h.h, self.params.data_ptr())
            h.version = self.version
        return h

    def release(self, shape=None):
        """Free the handles (of one grid, or all)."""
        for key in [k for k in self._handles if shape is None or k[0] == tuple(shape)]:
            self._handles.pop(key).close()

    def _pull(self, h):
        """After an optimiser step on handle h: its parameters are the current ones."""
        _call("unet_get_params", h.h, self.params.data_ptr(), None)
        self.version += 1
        h.version = self.version

    # network ----------------------------------------------------------------
    def forward(self, feat, shape, train=False, base=None, out=None):
        """feat: (V, 16) BF16 features on `shape`; returns the FP32 prediction (V,)."""
        import torch

        h = self.handle(shape, train)
        if out is None:
            out = torch.empty(int(np.prod(shape)), dtype=torch.float32, device=self.device)
        _call("unet_forward", h.h, _ptr(feat), _ptr(base), out.data_ptr())
        return out

    def backward(self, feat, dout, shape):
        """Parameter gradients for dout (FP32 per voxel) after forward(train=True)."""
        h = self.handle(shape, True)
        _call("unet_backward", h.h, _ptr(feat), dout.data_ptr())

    def grads(self, shape):
        """The flat FP32 parameter gradients of the last backward (a new tensor)."""
        import torch

        g = torch.empty_like(self.params)
        _call("unet_get_params", self.handle(shape, True).h, None, g.data_ptr())
        return g

    def adam_step(self, shape, lr, b1=0.9, b2=0.999, eps=1e-8):
        h = self.handle(shape, True)
        _call("unet_adam_step", h.h, lr, b1, b2, eps)
        self.t += 1
        self._pull(h)

    def train_step(self, feat, shape, target, mask, count, lr, weight=None):
        """One Adam step on the (weighted) masked MSE between the prediction and target;
        returns the loss (a one-element device tensor, before the step)."""
        import torch

        h = self.handle(shape, True)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        _call("unet_train_step", h.h, _ptr(feat), target.data_ptr(), mask.data_ptr(), _ptr(weight), int(count), lr,
              loss.data_ptr())
        self.t += 1
        self._pull(h)
        return loss

    def predict(self, active, n_cat, omega, tau_ref, target):
        """Start field (FP32 dense tensor on the grid of ``active``) from the solver's
        dense device fields; ``target`` is a unet_target."""
        import torch

        shape = tuple(active.shape)
        h = self.handle(shape, False)
        c = torch.empty(shape, dtype=torch.float32, device=self.device)
        target.struct_size = ctypes.sizeof(unet_target)
        _call("unet_predict", h.h, active.data_ptr(), _ptr(n_cat), omega.data_ptr(), tau_ref,
              ctypes.addressof(target), c.data_ptr())
        return c
