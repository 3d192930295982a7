"""FP64 CPU reference of dense membrane-CNN inference (arXiv 1612.02120, Section 2.2).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the GPU library. See emcnn_oracle.c for
the definitions; this module marshals numpy arrays into the C reference and adds
its own copy of the receptive-field arithmetic.

Pins (tests/test_oracle_*.py): pure-Python brute force on tiny inputs (bitwise),
torch float64 conv2d, delta-kernel identity, constant-input closed form, exact
translation equivariance, monotone-quantisation commutation, exhaustive bf16 /
e4m3fn encoder checks against torch casts, central finite differences for the
student gradient and the Adam step-one closed form.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_KIND = {"conv": 0, "pool": 1, "pool2": 2, "sub2": 3}
_ACT = {"none": 0, "relu": 1, "sigmoid": 2, "maxout": 3, "softmax": 4, "softmax0": 5}
QMODES = {"exact": 0, "bf16": 1, "fp8": 2}


class _Layer(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32), ("cin", ctypes.c_int32),
                ("cout", ctypes.c_int32), ("act", ctypes.c_int32)]


_lib = None
_native = None


def lib():
    global _lib
    if _lib is None:
        _lib = _bind(ctypes.CDLL(_build.build(force=False)))
    return _lib


def native_lib():
    """The -O3 -march=native timing build of the same source (bitwise the same
    results), compiled for this host on first use."""
    global _native
    if _native is None:
        _native = _bind(ctypes.CDLL(_build.build_native()))
    return _native


def _bind(L):
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_forward.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    L.orc_trace.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                            ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_void_p]
    L.orc_conv_layer.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_student_loss_grad.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_void_p, dp, ctypes.c_void_p]
    L.orc_adam.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, ctypes.c_double]
    L.orc_bf16_array.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    L.orc_e4m3_array.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    L.orc_sigmoid.argtypes = [ctypes.c_double]
    L.orc_sigmoid.restype = ctypes.c_double
    L.orc_radius.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_patch.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                            ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp, dp]
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_forward_maps.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    L.orc_patch_maps.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                 ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_double)]
    L.orc_watershed.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                ctypes.c_void_p]
    L.orc_out_dims.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.orc_forward_full.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    return L


def _layers(net):
    arr = (_Layer * len(net))()
    for i, L in enumerate(net):
        if L["kind"] == "conv":
            arr[i] = _Layer(0, L["k"], L["cin"], L["cout"], _ACT[L["act"]])
        else:
            arr[i] = _Layer(_KIND[L["kind"]], 2, 0, 0, 0)
    return arr


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def radius(net) -> int:
    """Receptive radius R (FoV = R + 1): r += (k - 1) j and j *= stride over the
    layers, a 2x2 pool counting as k = 2 ("pool2" has stride 2, "pool" 1) and a
    subsample ("sub2") as k = 1 with stride 2."""
    R, j = 0, 1
    for L in net:
        R += (L["k"] - 1 if L["kind"] == "conv" else 0 if L["kind"] == "sub2" else 1) * j
        if L["kind"] in ("pool2", "sub2"):
            j *= 2
    return R


def out_dims(net, H, W, full=False):
    """Dense output dims (Ho, Wo) of an H x W slice: H - R without subsampling;
    with a subsample, the pruned form's half-resolution map (full: every position)."""
    Ho, Wo = ctypes.c_int(0), ctypes.c_int(0)
    if lib().orc_out_dims(_layers(net), len(net), int(H), int(W), 1 if full else 0, ctypes.byref(Ho),
                          ctypes.byref(Wo)):
        raise ValueError("net does not fit %d x %d" % (H, W))
    return Ho.value, Wo.value


def patch(img, net, params, y, x):
    """Patch form at (y, x): the net on the (R+1)^2 window of one slice with
    plain stride-1 convs and stride-2 pools. Returns (probability, logit)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    params = np.ascontiguousarray(params, dtype=np.float64)
    out, lg = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().orc_patch(_ptr(img), H, W, _layers(net), len(net), _ptr(params), int(y), int(x),
                         ctypes.byref(out), ctypes.byref(lg))
    if rc:
        raise ValueError("oracle patch failed (%d)" % rc)
    return out.value, lg.value


def forward(vol, net, params, qmode="exact", act_scales=None, threads=0, logits=False, native=False):
    """Dense output of ``net`` on every slice of ``vol`` (Z x H x W uint8).

    Returns float64 Z x (H-R) x (W-R) probabilities, or pre-sigmoid logits of
    the last layer when ``logits`` is true. ``act_scales`` (FP8 mode): one input
    scale per conv layer (ignored where the layer is not FP8).
    """
    vol = np.ascontiguousarray(vol, dtype=np.uint8)
    if vol.ndim == 2:
        vol = vol[None]
    Z, H, W = vol.shape
    Ho, Wo = out_dims(net, H, W)
    params = np.ascontiguousarray(params, dtype=np.float64)
    n_conv = sum(1 for L in net if L["kind"] == "conv")
    sc = np.zeros(n_conv) if act_scales is None else np.array(
        [0.0 if s is None else s for s in act_scales], dtype=np.float64)
    out = np.empty((Z, Ho, Wo), dtype=np.float64)
    lay = _layers(net)
    L = native_lib() if native else lib()
    rc = L.orc_forward(_ptr(vol), Z, H, W, lay, len(net), _ptr(params), QMODES[qmode],
                           _ptr(sc), None if logits else _ptr(out),
                           _ptr(out) if logits else None, int(threads))
    if rc:
        raise ValueError("oracle forward failed (%d)" % rc)
    return out


def forward_full(vol, net, params, threads=0):
    """The full dense form (exact FP64): a subsampling layer keeps every position
    and doubles the spacing of the later layers, so output (z, Y, X) is the net
    on the window at input (Y, X); Z x (H - R) x (W - R)."""
    vol = np.ascontiguousarray(vol, dtype=np.uint8)
    if vol.ndim == 2:
        vol = vol[None]
    Z, H, W = vol.shape
    Ho, Wo = out_dims(net, H, W, full=True)
    params = np.ascontiguousarray(params, dtype=np.float64)
    out = np.empty((Z, Ho, Wo), dtype=np.float64)
    rc = lib().orc_forward_full(_ptr(vol), Z, H, W, _layers(net), len(net), _ptr(params), _ptr(out), int(threads))
    if rc:
        raise ValueError("oracle forward_full failed (%d)" % rc)
    return out


def trace(img, net, params, qmode="exact", act_scales=None):
    """Every layer's output (C x h x w float64) for one slice. In a fake-quant
    mode a conv's output is its FP64 value before the next layer rounds it."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    lay = _layers(net)
    dims = np.zeros(3 * len(net), dtype=np.int32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    n_conv = sum(1 for L in net if L["kind"] == "conv")
    sc = np.zeros(n_conv) if act_scales is None else np.array(
        [0.0 if s is None else s for s in act_scales], dtype=np.float64)
    # first pass for dims: run with bufs == NULL
    rc = lib().orc_trace(_ptr(img), H, W, lay, len(net), _ptr(params), QMODES[qmode], _ptr(sc), _ptr(dims), None)
    if rc:
        raise ValueError("oracle trace failed (%d)" % rc)
    bufs = [np.empty(tuple(dims[3 * l:3 * l + 3]), dtype=np.float64) for l in range(len(net))]
    ptrs = (ctypes.c_void_p * len(net))(*[b.ctypes.data for b in bufs])
    rc = lib().orc_trace(_ptr(img), H, W, lay, len(net), _ptr(params), QMODES[qmode], _ptr(sc), _ptr(dims), ptrs)
    if rc:
        raise ValueError("oracle trace failed (%d)" % rc)
    return bufs


def conv_layer(a, weights, bias, k, pool=False, qmode="exact", in_scale=0.0):
    """One inner conv (optionally after the 2x2 stride-1 max filter) on a given
    C x H x W map in a fake-quant mode's number format; returns (out, absum):
    the conv output before its activation and the scaled sum of |products|."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    C, H, W = a.shape
    wt = np.ascontiguousarray(weights, dtype=np.float64)
    bs = np.ascontiguousarray(bias, dtype=np.float64)
    Co = bs.size
    assert wt.size == Co * C * k * k
    Ho, Wo = H - (1 if pool else 0) - (k - 1), W - (1 if pool else 0) - (k - 1)
    out = np.empty((Co, Ho, Wo))
    absum = np.empty((Co, Ho, Wo))
    rc = lib().orc_conv_layer(_ptr(a), C, H, W, 1 if pool else 0, _ptr(wt), _ptr(bs), int(k), Co, QMODES[qmode],
                              float(in_scale), _ptr(out), _ptr(absum))
    if rc:
        raise ValueError("oracle conv_layer failed (%d)" % rc)
    return out, absum


def student_loss_grad(patches, teacher, net, params):
    """(mean BCE-with-logits, gradient) for a batch; see emcnn_oracle.c."""
    patches = np.ascontiguousarray(patches, dtype=np.uint8)
    teacher = np.ascontiguousarray(teacher, dtype=np.float64)
    params = np.ascontiguousarray(params, dtype=np.float64)
    B, P, _ = patches.shape
    grad = np.zeros_like(params)
    loss = ctypes.c_double(0.0)
    rc = lib().orc_student_loss_grad(_ptr(patches), B, P, _ptr(teacher), _layers(net), len(net),
                                     _ptr(params), ctypes.byref(loss), _ptr(grad))
    if rc:
        raise ValueError("oracle student_loss_grad failed (%d)" % rc)
    return loss.value, grad


def adam(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (theta, m, v, g):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(_ptr(theta), _ptr(m), _ptr(v), _ptr(g), theta.size, int(t), lr, b1, b2, eps)


def bf16_round(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_bf16_array(_ptr(x), _ptr(out), x.size)
    return out


def e4m3_round(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_e4m3_array(_ptr(x), _ptr(out), x.size)
    return out


def sigmoid(t: float) -> float:
    return lib().orc_sigmoid(float(t))


def num_threads() -> int:
    return lib().orc_num_threads()


def watershed(prob, t_seed):
    """3-D watershed by steepest descent with seeded minima (see emcnn_oracle.c):
    int32 labels of a Z x H x W float32 probability map."""
    p = np.ascontiguousarray(prob, dtype=np.float32)
    if p.ndim == 2:
        p = p[None]
    Z, H, W = p.shape
    lab = np.empty((Z, H, W), dtype=np.int32)
    rc = lib().orc_watershed(_ptr(p), Z, H, W, float(np.float32(t_seed)), _ptr(lab))
    if rc:
        raise ValueError("oracle watershed failed (%d)" % rc)
    return lab


def forward_maps(maps, net, params, threads=0):
    """Dense output of a multi-channel net on real-valued maps (Z x C x H x W,
    planar), exact FP64: Z x Ho x Wo."""
    m = np.ascontiguousarray(maps, dtype=np.float64)
    Z, C, H, W = m.shape
    Ho, Wo = out_dims(net, H, W)
    params = np.ascontiguousarray(params, dtype=np.float64)
    out = np.empty((Z, Ho, Wo), dtype=np.float64)
    rc = lib().orc_forward_maps(_ptr(m), Z, C, H, W, _layers(net), len(net), _ptr(params), _ptr(out), int(threads))
    if rc:
        raise ValueError("oracle forward_maps failed (%d)" % rc)
    return out


def patch_maps(maps, net, params, y, x):
    """Patch form of a multi-channel net on one window of C x H x W maps."""
    m = np.ascontiguousarray(maps, dtype=np.float64)
    C, H, W = m.shape
    out = ctypes.c_double(0.0)
    rc = lib().orc_patch_maps(_ptr(m), C, H, W, _layers(net), len(net),
                              _ptr(np.ascontiguousarray(params, dtype=np.float64)), int(y), int(x), ctypes.byref(out))
    if rc:
        raise ValueError("oracle patch_maps failed (%d)" % rc)
    return out.value
