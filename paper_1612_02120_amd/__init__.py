"""Python binding of libemcnn (include/emcnn.h): dense membrane-probability
inference of a uint8 EM stack on an MI355X (arXiv 1612.02120, Section 2.2).

The functions keep the C names and only marshal arguments: torch CUDA tensors
provide device memory and streams, numpy arrays provide host weights. All
computation happens in the library's HIP kernels. If the library is not built
the import fails; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libemcnn.so")

CNN_OK, CNN_EINVAL, CNN_ENOMEM, CNN_EHIP, CNN_EUNSUPPORTED = 0, -1, -2, -3, -4
PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2}
_ACT = {"none": 0, "relu": 1, "sigmoid": 2, "maxout": 3, "softmax": 4, "softmax0": 5}
_POOL_KIND = {"pool": 1, "pool2": 2, "sub2": 3}  # 2x2 window, stride 1 / stride 2; 2x subsample


class CnnError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__("%s failed (%d): %s" % (fn, code, msg))
        self.code = code


class _Layer(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32), ("cin", ctypes.c_int32),
                ("cout", ctypes.c_int32), ("act", ctypes.c_int32), ("act_scale", ctypes.c_float)]


class _Spec(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("layers", ctypes.POINTER(_Layer)),
                ("precision", ctypes.c_int32)]


class _Tile(ctypes.Structure):
    _fields_ = [("inp", ctypes.c_void_p), ("z", ctypes.c_int64), ("h", ctypes.c_int64),
                ("w", ctypes.c_int64), ("halo", ctypes.c_int32), ("out", ctypes.c_void_p)]


class _PatchSrc(ctypes.Structure):
    _fields_ = [("volume", ctypes.c_void_p), ("teacher", ctypes.c_void_p), ("Z", ctypes.c_int64),
                ("H", ctypes.c_int64), ("W", ctypes.c_int64), ("z", ctypes.c_int32), ("y", ctypes.c_int32),
                ("x", ctypes.c_int32)]


class _Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


EXPORTS = [
    "cnn_create", "cnn_destroy", "cnn_geometry", "cnn_infer", "cnn_infer_batch", "cnn_autotune",
    "cnn_describe", "cnn_set_batch_graph", "cnn_set_workspace_limit", "student_create",
    "student_destroy", "student_get_state", "student_set_state", "student_grad",
    "student_train_step", "student_infer", "student_infer_with_fallback", "cnn_last_error",
    "cnn_profile", "cnn_profile_read", "cnn_variant_name", "cnn_set_variant",
    "cnn_infer_noalloc", "student_gather", "cnn_read_activation", "cnn_mfma_probe", "cnn_mfma_bench",
    "cnn_output_dims", "watershed_3d", "cnn_infer_maps", "cnn_autotune_batch",
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libemcnn.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    sig = {
        "cnn_create": [vp, i64, vp, vp],
        "cnn_destroy": [vp],
        "cnn_geometry": [vp, vp, vp],
        "cnn_output_dims": [vp, i64, i64, vp, vp],
        "watershed_3d": [vp, vp, f32, vp, vp, vp],
        "cnn_infer": [vp, vp, vp, vp, vp],
        "cnn_infer_noalloc": [vp, vp, vp, vp, vp],
        "cnn_infer_maps": [vp, vp, vp, vp, vp],
        "cnn_read_activation": [vp, i32, vp, i64, vp, vp],
        "cnn_mfma_probe": [i32, vp, vp, vp, i32, i32, vp],
        "cnn_mfma_bench": [i32, i32, i32, vp, vp, vp, vp],
        "cnn_infer_batch": [vp, vp, i32, vp],
        "cnn_autotune": [vp, i64, i64, ctypes.c_char_p, vp],
        "cnn_autotune_batch": [vp, vp, i32, vp],
        "cnn_describe": [vp, ctypes.c_char_p, i32],
        "cnn_set_batch_graph": [vp, i32],
        "cnn_set_workspace_limit": [vp, i64],
        "cnn_profile": [vp, i32],
        "cnn_variant_name": [vp, i32, i32, ctypes.c_char_p, i32],
        "cnn_set_variant": [vp, i32, ctypes.c_char_p],
        "cnn_profile_read": [vp, vp, vp, i32],
        "student_create": [vp, i64, i32, vp],
        "student_destroy": [vp],
        "student_get_state": [vp, vp, vp, vp, vp],
        "student_set_state": [vp, vp, vp, vp, i64],
        "student_grad": [vp, vp, vp, i32, i32, vp, vp, vp],
        "student_train_step": [vp, vp, vp, i32, i32, vp, vp, vp, vp],
        "student_gather": [vp, i32, i32, i32, vp, vp, vp],
        "student_infer": [vp, vp, vp, vp, vp],
        "student_infer_with_fallback": [vp, vp, vp, vp, vp, f32, i32, i32, ctypes.c_uint64, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.cnn_last_error.argtypes = []
    L.cnn_last_error.restype = ctypes.c_char_p
    return L


_lib = _load()


def cnn_last_error() -> str:
    return _lib.cnn_last_error().decode()


def _check(rc, fn):
    if rc != CNN_OK:
        raise CnnError(rc, fn, cnn_last_error())


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dims(t):
    return (ctypes.c_int64 * 3)(*[int(s) for s in t.shape])


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_buf(t, dtype, name, shape=None, min_numel=None):
    """Host-side checks of a caller buffer before its pointer reaches the
    library: tensor, dtype, shape (or at least min_numel elements), contiguity."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(int(v) for v in shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError("%s needs at least %d elements, got %d" % (name, min_numel, t.numel()))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _on_device(**bufs):
    """Every buffer passed to the library lives in device memory (checked after
    the host-side checks of all buffers)."""
    for name, t in bufs.items():
        if t is not None and not t.is_cuda:
            raise TypeError("%s must be a CUDA (HIP) tensor" % name)


def _require_cuda(t, dtype, name, shape=None, min_numel=None):
    _check_buf(t, dtype, name, shape, min_numel)
    _on_device(**{name: t})


def radius_of(net) -> int:
    """Receptive radius of a layer list: r += (k - 1) j over the layers, where j
    (the input spacing) doubles after every stride-2 layer; a 2x2 pool has
    k = 2, a subsample k = 1."""
    R, j = 0, 1
    for L in net:
        R += (L["k"] - 1 if L["kind"] == "conv" else 0 if L["kind"] == "sub2" else 1) * j
        if L["kind"] in ("pool2", "sub2"):
            j *= 2
    return R


class Net:
    """Owning handle of a cnn_net."""

    def __init__(self, ptr, R, precision=0):
        self.ptr = ptr
        self.R = R
        self.precision = precision

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.cnn_destroy(self.ptr)
            self.ptr = None

    def close(self):
        self.__del__()

    def out_dims(self, H, W):
        """(Ho, Wo) of an H x W slice (cnn_output_dims); (0, 0) below the field of view."""
        if H < self.R + 1 or W < self.R + 1:
            return 0, 0
        Ho, Wo = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.cnn_output_dims(self.ptr, int(H), int(W), ctypes.byref(Ho), ctypes.byref(Wo)),
               "cnn_output_dims")
        return Ho.value, Wo.value


def cnn_create(weights, net, precision="fp32", act_scales=None) -> Net:
    """weights: float64 vector (per conv W[cout][cin][k][k] then b[cout]);
    net: list of layer dicts; act_scales: per-conv FP8 input scales (None allowed)."""
    w = np.ascontiguousarray(weights, dtype=np.float64)
    arr = (_Layer * len(net))()
    ci = 0
    for i, L in enumerate(net):
        if L["kind"] == "conv":
            s = 0.0
            if act_scales is not None and act_scales[ci] is not None:
                s = float(act_scales[ci])
            arr[i] = _Layer(0, L["k"], L["cin"], L["cout"], _ACT[L["act"]], s)
            ci += 1
        else:
            arr[i] = _Layer(_POOL_KIND[L["kind"]], 1 if L["kind"] == "sub2" else 2, 0, 0, 0, 0.0)
    spec = _Spec(len(net), arr, PRECISIONS[precision])
    out = ctypes.c_void_p()
    _check(_lib.cnn_create(w.ctypes.data_as(ctypes.c_void_p), w.size, ctypes.byref(spec),
                           ctypes.byref(out)), "cnn_create")
    R = ctypes.c_int32()
    _check(_lib.cnn_geometry(out, ctypes.byref(R), None), "cnn_geometry")
    return Net(out, R.value, PRECISIONS[precision])


def cnn_destroy(net: Net):
    net.close()


def cnn_geometry(net: Net):
    R, fov = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.cnn_geometry(net.ptr, ctypes.byref(R), ctypes.byref(fov)), "cnn_geometry")
    return R.value, fov.value


def cnn_infer(net: Net, volume, out=None, stream=None):
    """volume: CUDA uint8 Z x H x W; returns (or fills) CUDA float32 Z x (H-R) x (W-R)."""
    import torch
    Z, H, W = _volume_dims(volume)
    Ho, Wo = net.out_dims(H, W) if net.ptr else (H - net.R, W - net.R)
    if out is None:
        out = torch.empty((Z, max(Ho, 0), max(Wo, 0)), dtype=torch.float32, device=volume.device)
    _check_buf(out, torch.float32, "out", shape=(Z, Ho, Wo))
    _on_device(volume=volume, out=out)
    _check(_lib.cnn_infer(net.ptr, _ptr(volume), _dims(volume), _ptr(out), _stream(stream)),
           "cnn_infer")
    return out


def cnn_infer_maps(net: Net, maps, out=None, stream=None):
    """maps: CUDA float32 Z x H x W x C (the net's first-conv input maps);
    returns (or fills) CUDA float32 Z x (H-R) x (W-R)."""
    import torch
    if not isinstance(maps, torch.Tensor) or maps.dim() != 4:
        raise ValueError("maps must be a Z x H x W x C tensor")
    _check_buf(maps, torch.float32, "maps")
    Z, H, W, C = (int(v) for v in maps.shape)
    Ho, Wo = net.out_dims(H, W) if net.ptr else (H - net.R, W - net.R)
    if out is None:
        out = torch.empty((Z, max(Ho, 0), max(Wo, 0)), dtype=torch.float32, device=maps.device)
    _check_buf(out, torch.float32, "out", shape=(Z, Ho, Wo))
    _on_device(maps=maps, out=out)
    dims = (ctypes.c_int64 * 4)(Z, H, W, C)
    _check(_lib.cnn_infer_maps(net.ptr, _ptr(maps), dims, _ptr(out), _stream(stream)), "cnn_infer_maps")
    return out


NOALLOC_SCRATCH_BYTES = 128 << 20  # CNN_NOALLOC_SCRATCH_BYTES of include/emcnn.h


def cnn_infer_noalloc(net: Net, volume, out, stream=None):
    """cnn_infer without any allocation: `out` (CUDA float32 Z x (H-R) x (W-R))
    is required, and the library works in its static device scratch."""
    import torch
    Z, H, W = _volume_dims(volume)
    Ho, Wo = net.out_dims(H, W) if net.ptr else (H - net.R, W - net.R)
    _check_buf(out, torch.float32, "out", shape=(Z, Ho, Wo))
    _on_device(volume=volume, out=out)
    _check(_lib.cnn_infer_noalloc(net.ptr, _ptr(volume), _dims(volume), _ptr(out), _stream(stream)),
           "cnn_infer_noalloc")
    return out


def _tile_array(tiles):
    import torch
    arr = (_Tile * len(tiles))()
    for i, (inp, halo, out) in enumerate(tiles):
        _require_cuda(inp, torch.uint8, "tile input")
        _require_cuda(out, torch.float32, "tile output")
        z, h, w = inp.shape
        if tuple(out.shape) != (z, h - 2 * halo, w - 2 * halo):
            raise ValueError("tile %d: output must be z x (h-2 halo) x (w-2 halo)" % i)
        arr[i] = _Tile(inp.data_ptr(), z, h, w, int(halo), out.data_ptr())
    return arr


def cnn_infer_batch(net: Net, tiles, stream=None):
    """tiles: list of (input uint8 CUDA tensor z x h x w, halo, output float32 CUDA tensor
    z x (h-2 halo) x (w-2 halo))."""
    arr = _tile_array(tiles)
    _check(_lib.cnn_infer_batch(net.ptr, arr, len(tiles), _stream(stream)), "cnn_infer_batch")


def cnn_autotune(net: Net, H: int, W: int, cache_path=None, stream=None):
    _check(_lib.cnn_autotune(net.ptr, int(H), int(W),
                             None if cache_path is None else str(cache_path).encode(),
                             _stream(stream)), "cnn_autotune")


def cnn_autotune_batch(net: Net, tiles, stream=None):
    """Per tile class tile shapes for cnn_infer_batch, tuned on these tiles
    (as cnn_infer_batch takes them; their outputs are overwritten)."""
    arr = _tile_array(tiles)
    _check(_lib.cnn_autotune_batch(net.ptr, arr, len(tiles), _stream(stream)), "cnn_autotune_batch")


def cnn_describe(net: Net) -> str:
    buf = ctypes.create_string_buffer(4096)
    _check(_lib.cnn_describe(net.ptr, buf, 4096), "cnn_describe")
    return buf.value.decode()


def cnn_set_batch_graph(net: Net, enable: bool):
    _check(_lib.cnn_set_batch_graph(net.ptr, 1 if enable else 0), "cnn_set_batch_graph")


def cnn_set_workspace_limit(net: Net, nbytes: int):
    _check(_lib.cnn_set_workspace_limit(net.ptr, int(nbytes)), "cnn_set_workspace_limit")


def cnn_read_activation(net: Net, layer: int, stream=None):
    """Stored output map of executed layer `layer` from the last cnn_infer, as a
    CUDA tensor in the stored layout (FP32: Z x h x w x C float32; BF16 / FP8:
    Z x C/16 x h x w x 16 bfloat16 / uint8 e4m3fn codes) and its (Z, C, h, w)."""
    import torch
    dt = {0: torch.float32, 1: torch.bfloat16, 2: torch.uint8}
    shape = (ctypes.c_int64 * 4)()
    # first call with a one-byte buffer only reports the shape (and fails on size)
    probe = torch.empty(1, dtype=torch.uint8, device="cuda")
    _lib.cnn_read_activation(net.ptr, int(layer), _ptr(probe), 0, shape, _stream(stream))
    Z, C, h, w = (int(v) for v in shape)
    if Z == 0:
        _check(_lib.cnn_read_activation(net.ptr, int(layer), _ptr(probe), 0, shape, _stream(stream)),
               "cnn_read_activation")
    prec = net.precision
    out = torch.empty((Z, h, w, C) if prec == 0 else (Z, C // 16, h, w, 16), dtype=dt[prec], device="cuda")
    _check(_lib.cnn_read_activation(net.ptr, int(layer), _ptr(out), out.numel() * out.element_size(), shape,
                                    _stream(stream)), "cnn_read_activation")
    return out, (Z, C, h, w)


def cnn_mfma_probe(precision, a, b, chain=1, stream=None):
    """D of ntiles 16 x 16 MFMA tiles, each accumulated over `chain` operand
    tiles (include/emcnn.h, cnn_mfma_probe): a, b are uint8 CUDA tensors
    (ntiles * chain) x 64 x 16 (FP8: x 32) holding each lane's operand bytes;
    returns float32 ntiles x 64 x 4 (lane (g, n): D[4g + k][n])."""
    import torch
    ch = 32 if precision == "fp8" else 16
    n = a.shape[0]
    if n % chain:
        raise ValueError("the operand tiles must be a multiple of chain")
    _check_buf(a, torch.uint8, "a", shape=(n, 64, ch))
    _check_buf(b, torch.uint8, "b", shape=(n, 64, ch))
    d = torch.empty((n // chain, 64, 4), dtype=torch.float32, device=a.device)
    _on_device(a=a, b=b)
    _check(_lib.cnn_mfma_probe(PRECISIONS[precision], _ptr(a), _ptr(b), _ptr(d), n // chain, int(chain),
                               _stream(stream)), "cnn_mfma_probe")
    return d


def cnn_mfma_bench(precision, ops, blocks=2048, iters=4096, stream=None):
    """(TFLOP/s, shader MHz) of the precision's MFMA on register operands from ops."""
    import torch
    _check_buf(ops, torch.uint8, "ops", min_numel=256 * 2 * 64 * 32)
    _on_device(ops=ops)
    tf, mhz = ctypes.c_double(), ctypes.c_double()
    _check(_lib.cnn_mfma_bench(PRECISIONS[precision], int(blocks), int(iters), _ptr(ops), ctypes.byref(tf),
                               ctypes.byref(mhz), _stream(stream)), "cnn_mfma_bench")
    return tf.value, mhz.value


def cnn_variant_names(net: Net, layer: int):
    """Names of the compiled candidates of executed layer `layer`."""
    out, buf = [], ctypes.create_string_buffer(512)
    while _lib.cnn_variant_name(net.ptr, layer, len(out), buf, 512) == CNN_OK:
        out.append(buf.value.decode())
    return out


def cnn_set_variant(net: Net, layer: int, name: str):
    _check(_lib.cnn_set_variant(net.ptr, int(layer), name.encode()), "cnn_set_variant")


def cnn_profile(net: Net, enable: bool):
    _check(_lib.cnn_profile(net.ptr, 1 if enable else 0), "cnn_profile")


def cnn_profile_read(net: Net, max_layers: int = 8):
    """Summed milliseconds and launch counts per executed layer since the last read."""
    ms = (ctypes.c_double * max_layers)()
    n = (ctypes.c_int32 * max_layers)()
    _check(_lib.cnn_profile_read(net.ptr, ms, n, max_layers), "cnn_profile_read")
    return list(ms), list(n)


# ---------------------------------------------------------------- student

STUDENT_R = 6
STUDENT_PARAMS = 801


class Student:
    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.student_destroy(self.ptr)
            self.ptr = None

    def close(self):
        self.__del__()


def student_create(w_init, precision="bf16") -> Student:
    w = np.ascontiguousarray(w_init, dtype=np.float64)
    out = ctypes.c_void_p()
    _check(_lib.student_create(w.ctypes.data_as(ctypes.c_void_p), w.size, PRECISIONS[precision],
                               ctypes.byref(out)), "student_create")
    return Student(out)


def student_destroy(s: Student):
    s.close()


def student_get_state(s: Student):
    w, m, v = (np.zeros(STUDENT_PARAMS) for _ in range(3))
    t = ctypes.c_int64()
    _check(_lib.student_get_state(s.ptr, w.ctypes.data_as(ctypes.c_void_p),
                                  m.ctypes.data_as(ctypes.c_void_p),
                                  v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t)),
           "student_get_state")
    return w, m, v, t.value


def student_set_state(s: Student, w, m, v, step: int):
    w, m, v = (np.ascontiguousarray(a, dtype=np.float64) for a in (w, m, v))
    _check(_lib.student_set_state(s.ptr, w.ctypes.data_as(ctypes.c_void_p),
                                  m.ctypes.data_as(ctypes.c_void_p),
                                  v.ctypes.data_as(ctypes.c_void_p), int(step)),
           "student_set_state")


def _check_patches(patches, teacher):
    import torch
    if not isinstance(patches, torch.Tensor) or patches.dim() != 3 or patches.shape[1] != patches.shape[2]:
        raise ValueError("patches must be a B x P x P tensor")
    B, P, _ = patches.shape
    _check_buf(patches, torch.uint8, "patches")
    _check_buf(teacher, torch.float32, "teacher_prob", shape=(B, P - STUDENT_R, P - STUDENT_R))
    return B, P


def student_grad(s: Student, patches, teacher, grad_out=None, loss_out=None, stream=None):
    import torch
    B, P = _check_patches(patches, teacher)
    dev = patches.device
    if grad_out is None:
        grad_out = torch.empty(STUDENT_PARAMS, dtype=torch.float32, device=dev)
    if loss_out is None:
        loss_out = torch.empty(1, dtype=torch.float64, device=dev)
    _check_buf(grad_out, torch.float32, "grad_out", shape=(STUDENT_PARAMS,))
    _check_buf(loss_out, torch.float64, "loss_out", min_numel=1)
    _on_device(patches=patches, teacher_prob=teacher, grad_out=grad_out, loss_out=loss_out)
    _check(_lib.student_grad(s.ptr, _ptr(patches), _ptr(teacher), B, P, _ptr(grad_out),
                             _ptr(loss_out), _stream(stream)), "student_grad")
    return grad_out, loss_out


def student_gather(sources, patch, teacher_R, patches_out, teacher_out, stream=None):
    """Gather a training batch on the device. sources: list of (volume uint8
    Z x H x W, teacher map float32 Z x (H-R) x (W-R), z, y, x); fills
    patches_out (B x P x P uint8) and teacher_out (B x (P-6) x (P-6) float32)."""
    import torch
    B = len(sources)
    _check_buf(patches_out, torch.uint8, "patches_out", shape=(B, patch, patch))
    _check_buf(teacher_out, torch.float32, "teacher_out", shape=(B, patch - STUDENT_R, patch - STUDENT_R))
    arr = (_PatchSrc * max(B, 1))()
    for i, (vol, tmap, z, y, x) in enumerate(sources):
        Z, H, W = _volume_dims(vol)
        _check_buf(tmap, torch.float32, "teacher map", shape=(Z, H - teacher_R, W - teacher_R))
        _on_device(volume=vol, teacher_map=tmap)
        arr[i] = _PatchSrc(vol.data_ptr(), tmap.data_ptr(), Z, H, W, int(z), int(y), int(x))
    _on_device(patches_out=patches_out, teacher_out=teacher_out)
    _check(_lib.student_gather(arr, B, int(patch), int(teacher_R), _ptr(patches_out), _ptr(teacher_out),
                               _stream(stream)), "student_gather")
    return patches_out, teacher_out


def student_train_step(s: Student, patches, teacher, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                       loss_out=None, gnorm_out=None, stream=None):
    import torch
    B, P = _check_patches(patches, teacher)
    dev = patches.device
    if loss_out is None:
        loss_out = torch.empty(1, dtype=torch.float64, device=dev)
    if gnorm_out is None:
        gnorm_out = torch.empty(1, dtype=torch.float64, device=dev)
    _check_buf(loss_out, torch.float64, "loss_out", min_numel=1)
    _check_buf(gnorm_out, torch.float64, "gnorm_out", min_numel=1)
    _on_device(patches=patches, teacher_prob=teacher, loss_out=loss_out, gnorm_out=gnorm_out)
    hp = _Adam(lr, beta1, beta2, eps)
    _check(_lib.student_train_step(s.ptr, _ptr(patches), _ptr(teacher), B, P, ctypes.byref(hp),
                                   _ptr(loss_out), _ptr(gnorm_out), _stream(stream)),
           "student_train_step")
    return loss_out, gnorm_out


def _volume_dims(volume):
    import torch
    if not isinstance(volume, torch.Tensor) or volume.dim() != 3:
        raise ValueError("volume must be a Z x H x W tensor")
    _check_buf(volume, torch.uint8, "volume")
    return (int(v) for v in volume.shape)


def student_infer(s: Student, volume, out=None, stream=None):
    import torch
    Z, H, W = _volume_dims(volume)
    if out is None:
        out = torch.empty((Z, max(H - STUDENT_R, 0), max(W - STUDENT_R, 0)), dtype=torch.float32,
                          device=volume.device)
    _check_buf(out, torch.float32, "out", shape=(Z, H - STUDENT_R, W - STUDENT_R))
    _on_device(volume=volume, out=out)
    _check(_lib.student_infer(s.ptr, _ptr(volume), _dims(volume), _ptr(out), _stream(stream)),
           "student_infer")
    return out


def fallback_tiles(shape_out, tile):
    """(ty, tx): fallback tiles per slice along y and x for an output of shape Z x Ho x Wo."""
    _, Ho, Wo = shape_out
    return (Ho + tile - 1) // tile, (Wo + tile - 1) // tile


def student_infer_with_fallback(s: Student, teacher: Net, volume, tau=0.01, tile=512, n_samples=4,
                                seed=0, out=None, stats=None, flags=None, stream=None):
    """Returns (out, stats); with flags (an int32 CUDA tensor of Z * ty * tx
    elements, see fallback_tiles) the per-tile decisions are written there too."""
    import torch
    Z, H, W = _volume_dims(volume)
    R = teacher.R
    if out is None:
        out = torch.empty((Z, max(H - R, 0), max(W - R, 0)), dtype=torch.float32, device=volume.device)
    if stats is None:
        stats = torch.zeros(2, dtype=torch.int32, device=volume.device)
    _check_buf(out, torch.float32, "out", shape=(Z, H - R, W - R))
    _check_buf(stats, torch.int32, "stats", shape=(2,))
    if flags is not None:
        ty, tx = fallback_tiles((Z, H - R, W - R), max(int(tile), 1))
        _check_buf(flags, torch.int32, "flags", shape=(Z * ty * tx,))
    _on_device(volume=volume, out=out, stats=stats, flags=flags)
    _check(_lib.student_infer_with_fallback(s.ptr, teacher.ptr, _ptr(volume), _dims(volume),
                                            _ptr(out), float(tau), int(tile), int(n_samples),
                                            int(seed), _ptr(stats),
                                            None if flags is None else _ptr(flags),
                                            _stream(stream)),
           "student_infer_with_fallback")
    return out, stats


# ---------------------------------------------------------------- watershed


def watershed_3d(prob, seed_threshold, labels=None, work=None, stream=None):
    """3-D watershed of a float32 CUDA map Z x H x W (include/emcnn.h); returns
    int32 labels of the same shape."""
    import torch
    if not isinstance(prob, torch.Tensor) or prob.dim() != 3:
        raise ValueError("prob must be a Z x H x W tensor")
    _check_buf(prob, torch.float32, "prob")
    if labels is None:
        labels = torch.empty(prob.shape, dtype=torch.int32, device=prob.device)
    if work is None:
        work = torch.empty(prob.numel() + 1, dtype=torch.int32, device=prob.device)
    _check_buf(labels, torch.int32, "labels", shape=tuple(prob.shape))
    _check_buf(work, torch.int32, "work", min_numel=prob.numel() + 1)
    _on_device(prob=prob, labels=labels, work=work)
    _check(_lib.watershed_3d(_ptr(prob), _dims(prob), float(seed_threshold), _ptr(labels), _ptr(work),
                             _stream(stream)), "watershed_3d")
    return labels
