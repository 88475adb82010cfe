"""Thin ctypes binding of the denoiser and gamma-index ABI
(``include/pmc_unet.h``).  Function names match the C entry points; this
module only marshals arguments (torch tensors provide device memory and
streams).  Every computation runs in ``libpmc.so``."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import pmc

# every symbol include/pmc_unet.h declares
EXPORTS = ("pmc_unet_create", "pmc_unet_destroy", "pmc_unet_last_error", "pmc_unet_param_count",
           "pmc_unet_get_params", "pmc_unet_set_params", "pmc_unet_forward", "pmc_unet_backward",
           "pmc_unet_forward_region",
           "pmc_unet_get_grads", "pmc_unet_zero_grads", "pmc_unet_adam_step", "pmc_unet_grad_norm",
           "pmc_nn_conv3d_forward", "pmc_nn_conv3d_backward_data", "pmc_nn_conv3d_backward_weight",
           "pmc_nn_conv3d_backward_data_noalloc", "pmc_nn_mfma_probe",
           "pmc_gamma_index", "pmc_denoise_disagreement")

_ready = False
# element count of one network input, per handle (the C calls take bare
# pointers sized at creation)
_shape = {}
_numel = {}


def lib():
    global _ready
    L = pmc.lib()
    if not _ready:
        vp, i32, f32 = C.c_void_p, C.c_int, C.c_float
        L.pmc_unet_create.argtypes = [C.POINTER(vp), i32, i32, i32, i32, i32, C.c_uint64]
        L.pmc_unet_destroy.argtypes = [vp]
        L.pmc_unet_last_error.argtypes = [vp]
        L.pmc_unet_last_error.restype = C.c_char_p
        L.pmc_unet_param_count.argtypes = [vp, C.POINTER(C.c_int64)]
        L.pmc_unet_get_params.argtypes = [vp, vp]
        L.pmc_unet_set_params.argtypes = [vp, vp]
        L.pmc_unet_forward.argtypes = [vp, vp, vp, vp, vp]
        L.pmc_unet_forward_region.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, vp, vp]
        L.pmc_unet_backward.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double), vp]
        L.pmc_unet_get_grads.argtypes = [vp, vp]
        L.pmc_unet_zero_grads.argtypes = [vp, vp]
        L.pmc_unet_adam_step.argtypes = [vp, f32, f32, vp]
        L.pmc_unet_grad_norm.argtypes = [vp, C.POINTER(C.c_double), vp]
        L.pmc_nn_conv3d_forward.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, i32, vp]
        L.pmc_nn_conv3d_backward_data.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, i32, vp]
        L.pmc_nn_conv3d_backward_data_noalloc.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, i32, vp]
        L.pmc_nn_mfma_probe.argtypes = [i32, vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.pmc_nn_conv3d_backward_weight.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, i32, vp]
        L.pmc_gamma_index.argtypes = [vp, vp, i32, i32, i32, f32, f32, f32, f32, f32, f32, f32, f32,
                                      vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), vp]
        L.pmc_denoise_disagreement.argtypes = [vp, vp, vp, C.c_int64, f32, f32, C.POINTER(C.c_double),
                                               C.POINTER(C.c_int64), vp]
        for name in EXPORTS:
            if name != "pmc_unet_last_error":
                getattr(L, name).restype = C.c_int
        _ready = True
    return L


def _check(u, status):
    if status != pmc.PMC_OK:
        msg = lib().pmc_unet_last_error(u).decode() if u else ""
        raise pmc.PMCError(status, msg)


def _dev(t, dtype, name):
    import torch
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s device tensor" % (name, dtype))
    return C.c_void_p(t.data_ptr())


def _stream(stream, device=0):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)


def pmc_unet_create(device, n, d, h, w, seed):
    u = C.c_void_p()
    _check(None, lib().pmc_unet_create(C.byref(u), int(device), n, d, h, w, int(seed)))
    _numel[u.value] = n * d * h * w
    _shape[u.value] = (n, d, h, w)
    return u


def pmc_unet_destroy(u):
    _numel.pop(u.value, None)
    _shape.pop(u.value, None)
    _check(None, lib().pmc_unet_destroy(u))


def _sized(u, *tensors):
    want = _numel.get(u.value)
    for t in tensors:
        if want is None or t.numel() != want:
            raise ValueError("tensor has %d elements, the network takes %s" % (t.numel(), want))


def pmc_unet_param_count(u) -> int:
    c = C.c_int64()
    _check(u, lib().pmc_unet_param_count(u, C.byref(c)))
    return c.value


def pmc_unet_get_params(u) -> np.ndarray:
    p = np.zeros(pmc_unet_param_count(u), np.float32)
    _check(u, lib().pmc_unet_get_params(u, C.c_void_p(p.ctypes.data)))
    return p


def pmc_unet_set_params(u, params):
    p = np.ascontiguousarray(params, np.float32)
    if p.size != pmc_unet_param_count(u):
        raise ValueError("parameter vector has the wrong length")
    _check(u, lib().pmc_unet_set_params(u, C.c_void_p(p.ctypes.data)))


def pmc_unet_get_grads(u) -> np.ndarray:
    g = np.zeros(pmc_unet_param_count(u), np.float32)
    _check(u, lib().pmc_unet_get_grads(u, C.c_void_p(g.ctypes.data)))
    return g


def pmc_unet_zero_grads(u, stream=None):
    _check(u, lib().pmc_unet_zero_grads(u, _stream(stream)))


def pmc_unet_forward(u, dose, density, out, stream=None):
    import torch
    _sized(u, dose, density, out)
    f = torch.float32
    _check(u, lib().pmc_unet_forward(u, _dev(dose, f, "dose"), _dev(density, f, "density"),
                                     _dev(out, f, "out"), _stream(stream, dose.device)))


def pmc_unet_forward_region(u, dose, density, out, stream=None):
    """Denoise a [d][h][w] grid no larger than the network's shape (zero
    outside it); dose, density and out are tensors of that shape."""
    import torch
    shp = _shape.get(u.value)
    if shp is None or dose.dim() != 3 or tuple(density.shape) != tuple(dose.shape) or \
            tuple(out.shape) != tuple(dose.shape):
        raise ValueError("dose, density and out must be [d][h][w] tensors of one shape")
    d, h, w = (int(v) for v in dose.shape)
    if shp[0] != 1 or d > shp[1] or h > shp[2] or w > shp[3]:
        raise ValueError("grid %s does not fit the network's shape %s" % ((d, h, w), shp))
    f = torch.float32
    _check(u, lib().pmc_unet_forward_region(u, _dev(dose, f, "dose"), _dev(density, f, "density"), d, h, w,
                                            _dev(out, f, "out"), _stream(stream, dose.device)))


def pmc_unet_backward(u, dose, density, target, stream=None) -> float:
    import torch
    _sized(u, dose, density, target)
    f = torch.float32
    loss = C.c_double()
    _check(u, lib().pmc_unet_backward(u, _dev(dose, f, "dose"), _dev(density, f, "density"),
                                      _dev(target, f, "target"), C.byref(loss),
                                      _stream(stream, dose.device)))
    return loss.value


def pmc_unet_adam_step(u, lr, grad_scale=1.0, stream=None):
    _check(u, lib().pmc_unet_adam_step(u, float(lr), float(grad_scale), _stream(stream)))


def pmc_unet_grad_norm(u, stream=None):
    out = C.c_double(0.0)
    _check(u, lib().pmc_unet_grad_norm(u, C.byref(out), _stream(stream)))
    return out.value


def _bf16(t, name):
    import torch
    if t.dtype not in (torch.bfloat16, torch.int16) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous bfloat16 device tensor" % name)
    return C.c_void_p(t.data_ptr())


def kp(cin: int) -> int:
    """Row length of a convolution weight matrix: 27*cin rounded up to 32."""
    return (27 * cin + 31) // 32 * 32


def pmc_nn_conv3d_forward(x, w, bias, y, relu=False, stream=None):
    """x [n,d,h,w,cin] bf16, w [cout, Kp] bf16, bias [cout] f32 or None, y
    [n,d,h,w,cout] bf16."""
    import torch
    n, d, h, wd, cin = x.shape
    cout = y.shape[-1]
    b = _dev(bias, torch.float32, "bias") if bias is not None else None
    _check(None, lib().pmc_nn_conv3d_forward(_bf16(x, "x"), _bf16(w, "w"), b, _bf16(y, "y"), n, d, h,
                                             wd, cin, cout, int(bool(relu)),
                                             _stream(stream, x.device)))


def pmc_nn_conv3d_backward_data(dy, w, dx, stream=None):
    n, d, h, wd, cout = dy.shape
    cin = dx.shape[-1]
    _check(None, lib().pmc_nn_conv3d_backward_data(_bf16(dy, "dy"), _bf16(w, "w"), _bf16(dx, "dx"),
                                                   n, d, h, wd, cin, cout,
                                                   _stream(stream, dy.device)))


def pmc_nn_conv3d_backward_data_noalloc(dy, w, dx, stream=None):
    """As pmc_nn_conv3d_backward_data, with the library's device-resident
    workspace (no allocation; stream-ordered, no synchronisation)."""
    n, d, h, wd, cout = dy.shape
    cin = dx.shape[-1]
    _check(None, lib().pmc_nn_conv3d_backward_data_noalloc(_bf16(dy, "dy"), _bf16(w, "w"), _bf16(dx, "dx"),
                                                           n, d, h, wd, cin, cout,
                                                           _stream(stream, dy.device)))


def pmc_nn_mfma_probe(iters=20000, stream=None):
    """(best launch ms, FLOP per launch) of the matrix-core throughput probe."""
    ms, flop = C.c_double(), C.c_double()
    h = None
    if stream is not None:
        h = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)
    _check(None, lib().pmc_nn_mfma_probe(int(iters), h, C.byref(ms), C.byref(flop)))
    return ms.value, flop.value


def pmc_nn_conv3d_backward_weight(x, dy, dw, stream=None):
    import torch
    n, d, h, wd, cin = x.shape
    cout = dy.shape[-1]
    _check(None, lib().pmc_nn_conv3d_backward_weight(_bf16(x, "x"), _bf16(dy, "dy"),
                                                     _dev(dw, torch.float32, "dw"), n, d, h, wd,
                                                     cin, cout, _stream(stream, x.device)))


def pmc_gamma_index(ref, ev, voxel_cm, dose_frac=0.02, dta_cm=0.2, cutoff_frac=0.1,
                    search_cm=0.6, step_cm=0.05, gamma=None, stream=None):
    """Gamma pass rate of ``ev`` against ``ref`` ([nz,ny,nx] float64 device
    tensors); returns (pass_rate, n_eval)."""
    import torch
    nz, ny, nx = ref.shape
    if tuple(ev.shape) != tuple(ref.shape):
        raise ValueError("ref and eval must have the same shape")
    rate = C.c_double()
    n = C.c_int64()
    g = _dev(gamma, torch.float32, "gamma") if gamma is not None else None
    _check(None, lib().pmc_gamma_index(_dev(ref, torch.float64, "ref"), _dev(ev, torch.float64, "eval"),
                                       nx, ny, nz, voxel_cm[0], voxel_cm[1], voxel_cm[2], dose_frac,
                                       dta_cm, cutoff_frac, search_cm, step_cm, g, C.byref(rate),
                                       C.byref(n), _stream(stream, ref.device)))
    return rate.value, n.value


def pmc_denoise_disagreement(den, mc, var_mc, cutoff_frac=0.1, k_sigma=4.0, stream=None):
    """Fraction of voxels above cutoff_frac * max(mc) where the denoised
    dose (float32 tensor) departs from the Monte Carlo dose (float64) by more
    than k_sigma standard errors; returns (fraction, count above cutoff)."""
    import torch
    if den.numel() != mc.numel() or var_mc.numel() != mc.numel():
        raise ValueError("tensors must have the same number of elements")
    frac = C.c_double()
    n = C.c_int64()
    _check(None, lib().pmc_denoise_disagreement(_dev(den, torch.float32, "den"), _dev(mc, torch.float64, "mc"),
                                                _dev(var_mc, torch.float64, "var_mc"), mc.numel(),
                                                cutoff_frac, k_sigma, C.byref(frac), C.byref(n),
                                                _stream(stream, mc.device)))
    return frac.value, n.value


class UNet:
    """Owns one network; convenience wrapper over the functions above."""

    def __init__(self, shape, seed=0, device=0):
        n, d, h, w = shape
        self.shape = shape
        self.u = pmc_unet_create(device, n, d, h, w, seed)

    def close(self):
        if self.u:
            pmc_unet_destroy(self.u)
            self.u = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        return pmc_unet_get_params(self.u)

    def set_params(self, p):
        pmc_unet_set_params(self.u, p)

    def grads(self):
        return pmc_unet_get_grads(self.u)

    def zero_grads(self, stream=None):
        pmc_unet_zero_grads(self.u, stream)

    def forward(self, dose, density, out, stream=None):
        pmc_unet_forward(self.u, dose, density, out, stream)

    def forward_region(self, dose, density, out, stream=None):
        pmc_unet_forward_region(self.u, dose, density, out, stream)

    def backward(self, dose, density, target, stream=None):
        return pmc_unet_backward(self.u, dose, density, target, stream)

    def adam_step(self, lr, grad_scale=1.0, stream=None):
        pmc_unet_adam_step(self.u, lr, grad_scale, stream)

    def grad_norm(self, stream=None):
        return pmc_unet_grad_norm(self.u, stream)
