"""Python binding of the upscaler kernels (the C ABI in include/splotch_nn.h).

Argument marshalling only: each function checks shapes, dtypes and devices
of torch tensors and calls one library entry point on the current stream.
bf16 tensors are ``torch.bfloat16``; activations are NHWC.
"""
from __future__ import annotations

import ctypes as C

from . import splotch

class NNWeights(C.Structure):
    _fields_ = [("w", C.c_void_p * 6), ("b", C.c_void_p * 6)]


_SIGS = {
    "splotch_nn_upscale_workspace_size": [C.c_int32, C.c_int32, C.c_int32,
                                          C.POINTER(C.c_size_t)],
    "splotch_nn_upscale": [C.POINTER(NNWeights), C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                           C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                           C.c_void_p],
    "splotch_nn_conv3x3_fwd": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               C.c_int32, C.c_int32, C.c_void_p],
    "splotch_nn_flip_weights": [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p],
    "splotch_nn_conv3x3_bwd_weight": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_int32, C.c_void_p],
    "splotch_nn_pack_input": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                              C.c_int32, C.c_void_p],
    "splotch_nn_head": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                        C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p],
    "splotch_nn_adam": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float,
                        C.c_float, C.c_float, C.c_float, C.c_int32, C.c_void_p],
    "splotch_nn_to_bf16": [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p],
    "splotch_nn_consistency": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                               C.c_int32, C.c_void_p],
    "splotch_nn_region_check": [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
}
_lib = None


def lib():
    global _lib
    if _lib is None:
        L = splotch.load()
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = C.c_int32
            fn.argtypes = args
        _lib = L
    return _lib


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != splotch.OK:
        msg = lib().splotch_status_string(st).decode()
        raise splotch.SplotchError(st, f"{name}: {msg}")


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _s(stream=None):
    return splotch._stream_ptr(stream)


def _need(t, dtype, shape, name):
    import torch
    if t is None:
        return
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def conv3x3_fwd(x, w, bias=None, mask=None, relu=True, out_f32=False, out=None, stream=None):
    """y = conv3x3(x * [mask > 0], w) + bias (ReLU if relu).  x: bf16
    [n, h, w, cin]; w: bf16 [cout, 3, 3, cin]; returns y [n, h, w, cout]."""
    import torch
    n, h, wd, cin = x.shape
    cout = w.shape[0]
    _need(x, torch.bfloat16, None, "x")
    _need(w, torch.bfloat16, (cout, 3, 3, cin), "w")
    _need(bias, torch.float32, (cout,), "bias")
    _need(mask, torch.bfloat16, x.shape, "mask")
    dt = torch.float32 if out_f32 else torch.bfloat16
    if out is None:
        out = torch.empty((n, h, wd, cout), dtype=dt, device=x.device)
    _need(out, dt, (n, h, wd, cout), "out")
    _call("splotch_nn_conv3x3_fwd", _p(x), _p(w), _p(bias), _p(mask), _p(out), n, h, wd, cin,
          cout, int(relu), int(out_f32), _s(stream))
    return out


def flip_weights(w, out=None, stream=None):
    """[cout, 3, 3, cin] -> [cin, 3, 3, cout] with the taps reversed."""
    import torch
    cout, _, _, cin = w.shape
    _need(w, torch.bfloat16, None, "w")
    if out is None:
        out = torch.empty((cin, 3, 3, cout), dtype=torch.bfloat16, device=w.device)
    _need(out, torch.bfloat16, (cin, 3, 3, cout), "out")
    _call("splotch_nn_flip_weights", _p(w), _p(out), cin, cout, _s(stream))
    return out


def conv3x3_bwd_weight(x, dy, dw, db=None, mask=None, stream=None):
    """dw += dW, db += db of conv3x3 (dy masked by [mask > 0])."""
    import torch
    n, h, wd, cin = x.shape
    cout = dy.shape[3]
    _need(x, torch.bfloat16, None, "x")
    _need(dy, torch.bfloat16, (n, h, wd, cout), "dy")
    _need(mask, torch.bfloat16, (n, h, wd, cout), "mask")
    _need(dw, torch.float32, (cout, 3, 3, cin), "dw")
    _need(db, torch.float32, (cout,), "db")
    _call("splotch_nn_conv3x3_bwd_weight", _p(x), _p(dy), _p(mask), _p(dw), _p(db), n, h, wd,
          cin, cout, _s(stream))


def pack_input(log_accum, center_count, out=None, stream=None):
    """[n, h, w, 3] float + [n, h, w] int32 -> bf16 [n, h, w, 4]."""
    import torch
    n, h, wd, _ = log_accum.shape
    _need(log_accum, torch.float32, (n, h, wd, 3), "log_accum")
    _need(center_count, torch.int32, (n, h, wd), "center_count")
    if out is None:
        out = torch.empty((n, h, wd, 4), dtype=torch.bfloat16, device=log_accum.device)
    _need(out, torch.bfloat16, (n, h, wd, 4), "out")
    _call("splotch_nn_pack_input", _p(log_accum), _p(center_count), _p(out), n, h, wd,
          _s(stream))
    return out


def head(conv6, L_low, rgb=None, L_full=None, target=None, loss_sum=None, dconv6=None,
         stream=None):
    """Shuffle + bilinear residual + resolve (and the MSE loss/gradient)."""
    import torch
    n, h, wd, _ = conv6.shape
    full = (n, 4 * h, 4 * wd, 3)
    _need(conv6, torch.float32, (n, h, wd, 48), "conv6")
    _need(L_low, torch.float32, (n, h, wd, 3), "L_low")
    if rgb is None:
        rgb = torch.empty(full, dtype=torch.float32, device=conv6.device)
    _need(rgb, torch.float32, full, "rgb")
    _need(L_full, torch.float32, full, "L_full")
    _need(target, torch.float32, full, "target")
    _need(loss_sum, torch.float32, (1,), "loss_sum")
    _need(dconv6, torch.bfloat16, (n, h, wd, 48), "dconv6")
    _call("splotch_nn_head", _p(conv6), _p(L_low), _p(rgb), _p(L_full), _p(target),
          _p(loss_sum), _p(dconv6), n, h, wd, _s(stream))
    return rgb


def adam(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    import torch
    for t, nm in ((p, "p"), (g, "g"), (m, "m"), (v, "v")):
        _need(t, torch.float32, p.shape, nm)
    _call("splotch_nn_adam", _p(p), _p(g), _p(m), _p(v), int(p.numel()), float(lr),
          float(beta1), float(beta2), float(eps), int(step), _s(stream))


def to_bf16(src, out=None, stream=None):
    import torch
    _need(src, torch.float32, None, "src")
    if out is None:
        out = torch.empty(src.shape, dtype=torch.bfloat16, device=src.device)
    _need(out, torch.bfloat16, src.shape, "out")
    _call("splotch_nn_to_bf16", _p(src), _p(out), int(src.numel()), _s(stream))
    return out


def consistency(L_full, L_low, sum_sq, stream=None):
    """sum_sq (float [1], accumulated) += the consistency sum of squares."""
    import torch
    n, h, wd, _ = L_low.shape
    _need(L_low, torch.float32, (n, h, wd, 3), "L_low")
    _need(L_full, torch.float32, (n, 4 * h, 4 * wd, 3), "L_full")
    _need(sum_sq, torch.float32, (1,), "sum_sq")
    _call("splotch_nn_consistency", _p(L_full), _p(L_low), _p(sum_sq), n, h, wd, _s(stream))


def region_check(L_full, L_low, region, theta, mask, n_marked, metric=None, stream=None):
    """Per-region consistency of one image: mask (uint8, one per region) =
    metric > theta; n_marked (int32 [1], accumulated) += marked regions."""
    import torch
    _, h, wd, _ = L_low.shape
    _need(L_low, torch.float32, (1, h, wd, 3), "L_low")
    _need(L_full, torch.float32, (1, 4 * h, 4 * wd, 3), "L_full")
    q = int(region) // 4
    nreg = (-(-h // q)) * (-(-wd // q))
    _need(mask, torch.uint8, (nreg,), "mask")
    _need(n_marked, torch.int32, (1,), "n_marked")
    _need(metric, torch.float32, (nreg,), "metric")
    _call("splotch_nn_region_check", _p(L_full), _p(L_low), h, wd, int(region), float(theta),
          _p(metric), _p(mask), _p(n_marked), _s(stream))
    return mask


def upscale_workspace_size(n, h, w) -> int:
    out = C.c_size_t()
    _call("splotch_nn_upscale_workspace_size", n, h, w, C.byref(out))
    return int(out.value)


def upscale(weights: NNWeights, log_accum, center_count, rgb, L_full=None, check=None,
            workspace=None, stream=None):
    """The whole network in one call (pack, six convolutions, head and, with
    ``check`` given, the consistency sum of squares written to check[0])."""
    import torch
    n, h, wd, _ = log_accum.shape
    full = (n, 4 * h, 4 * wd, 3)
    _need(log_accum, torch.float32, (n, h, wd, 3), "log_accum")
    _need(center_count, torch.int32, (n, h, wd), "center_count")
    _need(rgb, torch.float32, full, "rgb")
    _need(L_full, torch.float32, full, "L_full")
    _need(check, torch.float32, (1,), "check")
    need = upscale_workspace_size(n, h, wd)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=log_accum.device)
    _call("splotch_nn_upscale", C.byref(weights), _p(log_accum), _p(center_count), n, h, wd,
          _p(rgb), _p(L_full), _p(check), _p(workspace),
          C.c_size_t(workspace.numel() * workspace.element_size()), _s(stream))
    return rgb
