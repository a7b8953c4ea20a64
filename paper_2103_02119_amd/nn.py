"""Python binding of include/lbm_nn.h (the warm-start network's kernels in
liblbm.so).  Argument marshalling only: device pointers are taken from torch
tensors (plumbing: torch owns the memory, the kernels do the work); a
negative status raises NNError.  There is no CPU fallback."""
from __future__ import annotations

import ctypes

from . import lbm as _lbm

EXPORTS = ("lbm_nn_conv3x3_fwd", "lbm_nn_conv3x3_dgrad", "lbm_nn_conv3x3_wgrad_work",
           "lbm_nn_conv3x3_wgrad", "lbm_nn_relu_bwd", "lbm_nn_avgpool2_fwd",
           "lbm_nn_avgpool2_bwd", "lbm_nn_upsample2_fwd", "lbm_nn_upsample2_bwd",
           "lbm_nn_conv1x1_fwd", "lbm_nn_conv1x1_work", "lbm_nn_conv1x1_bwd", "lbm_nn_mse_work",
           "lbm_nn_mse", "lbm_nn_adam", "lbm_nn_cast_weights", "lbm_nn_cast_bf16")

_V = ctypes.c_void_p
_I = ctypes.c_int
_Z = ctypes.c_size_t
_F = ctypes.c_float
_sigs = {
    "lbm_nn_conv3x3_fwd": [_V, _I, _V, _I, _I, _I, _I, _V, _V, _I, _I, _V, _V],
    "lbm_nn_conv3x3_dgrad": [_V, _I, _I, _I, _I, _V, _V, _I, _V, _I, _I, _V],
    "lbm_nn_conv3x3_wgrad_work": [_I, _I, _I, _I, _I, _I],
    "lbm_nn_conv3x3_wgrad": [_V, _I, _V, _I, _I, _I, _I, _V, _I, _V, _V, _V, _Z, _V],
    "lbm_nn_relu_bwd": [_V, _V, _V, _Z, _V],
    "lbm_nn_avgpool2_fwd": [_V, _I, _I, _I, _I, _V, _V],
    "lbm_nn_avgpool2_bwd": [_V, _I, _I, _I, _I, _V, _I, _V],
    "lbm_nn_upsample2_fwd": [_V, _I, _I, _I, _I, _V, _V],
    "lbm_nn_upsample2_bwd": [_V, _I, _I, _I, _I, _V, _V],
    "lbm_nn_conv1x1_fwd": [_V, _I, _I, _V, _V, _I, _V, _V],
    "lbm_nn_conv1x1_work": [_I, _I, _I],
    "lbm_nn_conv1x1_bwd": [_V, _V, _I, _I, _V, _I, _V, _V, _V, _V, _Z, _V],
    "lbm_nn_mse_work": [_I, _I],
    "lbm_nn_mse": [_V, _V, _V, _I, _I, _V, _F, _V, _V, _V, _Z, _V],
    "lbm_nn_adam": [_V, _V, _V, _V, _Z, _F, _F, _F, _F, _I, _V],
    "lbm_nn_cast_weights": [_V, _I, _I, _V, _V, _V],
    "lbm_nn_cast_bf16": [_V, _Z, _V, _V],
}
_lib = None


class NNError(RuntimeError):
    pass


def load():
    global _lib
    if _lib is None:
        L = _lbm.load()
        for name, args in _sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _Z if name.endswith("_work") else _I
        _lib = L
    return _lib


def _p(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else t.data_ptr()


def _s(stream):
    return None if stream is None else int(stream)


def _call(name, *args):
    rc = getattr(load(), name)(*args)
    if rc != 0:
        raise NNError(f"{name} failed with status {rc}")


def lbm_nn_conv3x3_fwd(x1, c1, x2, c2, n, h, w, wt, bias, cout, relu, y, stream=None):
    _call("lbm_nn_conv3x3_fwd", _p(x1), c1, _p(x2), c2, n, h, w, _p(wt), _p(bias), cout,
          1 if relu else 0, _p(y), _s(stream))


def lbm_nn_conv3x3_dgrad(gy, n, h, w, cout, wd, gx1, c1, gx2, c2, accumulate, stream=None):
    _call("lbm_nn_conv3x3_dgrad", _p(gy), n, h, w, cout, _p(wd), _p(gx1), c1, _p(gx2), c2,
          1 if accumulate else 0, _s(stream))


def lbm_nn_conv3x3_wgrad_work(c1, c2, n, h, w, cout):
    return load().lbm_nn_conv3x3_wgrad_work(c1, c2, n, h, w, cout)


def lbm_nn_conv3x3_wgrad(x1, c1, x2, c2, n, h, w, gy, cout, gw, gb, work, stream=None):
    _call("lbm_nn_conv3x3_wgrad", _p(x1), c1, _p(x2), c2, n, h, w, _p(gy), cout, _p(gw), _p(gb),
          _p(work), work.numel() * work.element_size(), _s(stream))


def lbm_nn_relu_bwd(gy, y, g, stream=None):
    _call("lbm_nn_relu_bwd", _p(gy), _p(y), _p(g), g.numel(), _s(stream))


def lbm_nn_avgpool2_fwd(x, n, h, w, c, y, stream=None):
    _call("lbm_nn_avgpool2_fwd", _p(x), n, h, w, c, _p(y), _s(stream))


def lbm_nn_avgpool2_bwd(gy, n, h, w, c, gx, accumulate, stream=None):
    _call("lbm_nn_avgpool2_bwd", _p(gy), n, h, w, c, _p(gx), 1 if accumulate else 0, _s(stream))


def lbm_nn_upsample2_fwd(x, n, h, w, c, y, stream=None):
    _call("lbm_nn_upsample2_fwd", _p(x), n, h, w, c, _p(y), _s(stream))


def lbm_nn_upsample2_bwd(gy, n, h, w, c, gx, stream=None):
    _call("lbm_nn_upsample2_bwd", _p(gy), n, h, w, c, _p(gx), _s(stream))


def lbm_nn_conv1x1_fwd(x, m, cin, w, b, cout, y, stream=None):
    _call("lbm_nn_conv1x1_fwd", _p(x), m, cin, _p(w), _p(b), cout, _p(y), _s(stream))


def lbm_nn_conv1x1_work(m, cin, cout):
    return load().lbm_nn_conv1x1_work(m, cin, cout)


def lbm_nn_conv1x1_bwd(x, gy, m, cin, w, cout, gx, gw, gb, work, stream=None):
    _call("lbm_nn_conv1x1_bwd", _p(x), _p(gy), m, cin, _p(w), cout, _p(gx), _p(gw), _p(gb),
          _p(work), work.numel() * work.element_size(), _s(stream))


def lbm_nn_mse_work(m, c):
    return load().lbm_nn_mse_work(m, c)


def lbm_nn_mse(pred, target, fluid, m, c, cw, count, grad, loss, work, stream=None):
    _call("lbm_nn_mse", _p(pred), _p(target), _p(fluid), m, c, _p(cw), float(count), _p(grad),
          _p(loss), _p(work), work.numel() * work.element_size(), _s(stream))


def lbm_nn_adam(p, g, m, v, lr, b1, b2, eps, step, stream=None):
    _call("lbm_nn_adam", _p(p), _p(g), _p(m), _p(v), p.numel(), float(lr), float(b1), float(b2),
          float(eps), int(step), _s(stream))


def lbm_nn_cast_weights(w, c, cout, wt, wd, stream=None):
    _call("lbm_nn_cast_weights", _p(w), c, cout, _p(wt), _p(wd), _s(stream))


def lbm_nn_cast_bf16(x, y, stream=None):
    _call("lbm_nn_cast_bf16", _p(x), x.numel(), _p(y), _s(stream))
