"""Binding of the warm-start network (include/ivx_unet.h): argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

UNET_EXPORTS = ("ivx_unet_create", "ivx_unet_destroy", "ivx_unet_param_count", "ivx_unet_get_params",
                "ivx_unet_set_params", "ivx_unet_forward", "ivx_unet_train_step", "ivx_unet_loss_grad",
                "ivx_nn_conv3x3",
                "ivx_nn_conv3x3_grad_weight", "ivx_nn_conv3x3_flip", "ivx_nn_to_bf16", "ivx_nn_pool2",
                "ivx_nn_pool2_grad", "ivx_nn_up2", "ivx_nn_up2_grad")


def _lib():
    from . import load_library

    lib = load_library("f32")
    if getattr(lib, "_unet_ready", False):
        return lib
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.ivx_unet_create.argtypes = [i32, i32, i32, i32, i32, ctypes.c_uint64, ctypes.POINTER(vp)]
    lib.ivx_unet_destroy.argtypes = [vp]
    lib.ivx_unet_param_count.argtypes = [vp]
    lib.ivx_unet_param_count.restype = i64
    lib.ivx_unet_get_params.argtypes = [vp, vp]
    lib.ivx_unet_set_params.argtypes = [vp, vp]
    lib.ivx_unet_forward.argtypes = [vp, vp, vp, i32, vp]
    lib.ivx_unet_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp]
    lib.ivx_unet_loss_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.ivx_nn_conv3x3.argtypes = [vp, i32, i32, i32, i32, vp, vp, i32, i32, vp, i32, vp, vp]
    lib.ivx_nn_conv3x3_grad_weight.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp, vp]
    lib.ivx_nn_conv3x3_flip.argtypes = [vp, i32, i32, vp, vp]
    lib.ivx_nn_to_bf16.argtypes = [vp, i64, vp, vp]
    lib.ivx_nn_pool2.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    lib.ivx_nn_pool2_grad.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp]
    lib.ivx_nn_up2.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    lib.ivx_nn_up2_grad.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    for f in UNET_EXPORTS:
        if f != "ivx_unet_param_count":
            getattr(lib, f).restype = ctypes.c_int
    lib._unet_ready = True
    return lib


def _check(code):
    if code != 0:
        from . import IvxError

        raise IvxError(code, _lib().ivx_last_error().decode())


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream():
    import torch

    return torch.cuda.current_stream().cuda_stream


class UNet:
    """4-level U-Net on [batch][height][width] images (see include/ivx_unet.h)."""

    def __init__(self, levels=4, base=32, max_batch=16, height=256, width=256, seed=0):
        self.lib = _lib()
        self.levels, self.base, self.max_batch, self.height, self.width = levels, base, max_batch, height, width
        h = ctypes.c_void_p()
        _check(self.lib.ivx_unet_create(levels, base, max_batch, height, width, seed, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ivx_unet_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return int(self.lib.ivx_unet_param_count(self._h))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.param_count, dtype=np.float32)
        _check(self.lib.ivx_unet_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.param_count
        _check(self.lib.ivx_unet_set_params(self._h, p.ctypes.data))

    def forward(self, x, out=None):
        import torch

        x = x.to(torch.float32).contiguous()
        if out is None:
            out = torch.empty_like(x)
        _check(self.lib.ivx_unet_forward(self._h, _ptr(x), _ptr(out), x.shape[0], _stream()))
        return out

    def loss_grad(self, x, target):
        """(loss, gradient as a host float32 array) without updating the parameters."""
        import torch

        x = x.to(torch.float32).contiguous()
        target = target.to(torch.float32).contiguous()
        g = np.empty(self.param_count, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float64)
        _check(self.lib.ivx_unet_loss_grad(self._h, _ptr(x), _ptr(target), x.shape[0], g.ctypes.data,
                                           loss.ctypes.data, _stream()))
        return float(loss[0]), g

    def train_step(self, x, target, lr) -> float:
        import torch

        x = x.to(torch.float32).contiguous()
        target = target.to(torch.float32).contiguous()
        loss = np.zeros(1, dtype=np.float64)
        _check(self.lib.ivx_unet_train_step(self._h, _ptr(x), _ptr(target), x.shape[0], float(lr),
                                            loss.ctypes.data, _stream()))
        return float(loss[0])


# ------------------------------------------------------------------ single layers
def to_bf16(x):
    import torch

    x = x.to(torch.float32).contiguous()
    out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(_lib().ivx_nn_to_bf16(_ptr(x), x.numel(), _ptr(out), _stream()))
    return out


def conv3x3(x, w_bf16, bias=None, relu=False, mask=None, accumulate=False, out=None):
    import torch

    n, h, w, cin = x.shape
    cout = w_bf16.shape[0]
    if out is None:
        out = torch.zeros((n, h, w, cout), dtype=torch.float32, device=x.device)
    _check(_lib().ivx_nn_conv3x3(_ptr(x), n, h, w, cin, _ptr(w_bf16), _ptr(bias), cout, int(relu), _ptr(mask),
                                 int(accumulate), _ptr(out), _stream()))
    return out


def conv3x3_grad_weight(x, dy):
    import torch

    n, h, w, cin = x.shape
    cout = dy.shape[-1]
    dw = torch.empty((cout, 3, 3, cin), dtype=torch.float32, device=x.device)
    db = torch.empty(cout, dtype=torch.float32, device=x.device)
    _check(_lib().ivx_nn_conv3x3_grad_weight(_ptr(x), _ptr(dy), n, h, w, cin, cout, _ptr(dw), _ptr(db), _stream()))
    return dw, db


def conv3x3_flip(w_bf16):
    import torch

    cout, _, _, cin = w_bf16.shape
    out = torch.empty((cin, 3, 3, cout), dtype=torch.int16, device=w_bf16.device)
    _check(_lib().ivx_nn_conv3x3_flip(_ptr(w_bf16), cin, cout, _ptr(out), _stream()))
    return out


def pool2(x):
    import torch

    n, h, w, c = x.shape
    out = torch.empty((n, h // 2, w // 2, c), dtype=torch.float32, device=x.device)
    _check(_lib().ivx_nn_pool2(_ptr(x), n, h, w, c, _ptr(out), _stream()))
    return out


def pool2_grad(x, dy, accumulate_into=None):
    import torch

    n, h, w, c = x.shape
    dx = torch.zeros_like(x) if accumulate_into is None else accumulate_into
    _check(_lib().ivx_nn_pool2_grad(_ptr(x), _ptr(dy), n, h, w, c, int(accumulate_into is not None), _ptr(dx),
                                    _stream()))
    return dx


def up2(x):
    import torch

    n, h, w, c = x.shape
    out = torch.empty((n, 2 * h, 2 * w, c), dtype=torch.float32, device=x.device)
    _check(_lib().ivx_nn_up2(_ptr(x), n, h, w, c, _ptr(out), _stream()))
    return out


def up2_grad(dy):
    import torch

    n, h2, w2, c = dy.shape
    out = torch.empty((n, h2 // 2, w2 // 2, c), dtype=torch.float32, device=dy.device)
    _check(_lib().ivx_nn_up2_grad(_ptr(dy), n, h2 // 2, w2 // 2, c, _ptr(out), _stream()))
    return out
