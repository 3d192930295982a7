"""The C-ABI library loads without a GPU, exports every entry point declared in
include/emcnn.h, and rejects bad network specs before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "emcnn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("cnn_create", "cnn_infer", "cnn_infer_batch", "student_train_step",
              "student_infer_with_fallback", "cnn_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1612_02120_amd as m
    lib = ctypes.CDLL(m.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) <= set(m.EXPORTS)


def test_library_is_a_gfx950_code_object_build():
    import paper_1612_02120_amd as m
    data = open(m.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def _spec(m, net, prec="fp32"):
    arr = (m._Layer * len(net))()
    for i, L in enumerate(net):
        if L["kind"] == "conv":
            arr[i] = m._Layer(0, L["k"], L["cin"], L["cout"], m._ACT[L["act"]], 0.0)
        else:
            arr[i] = m._Layer(m._POOL_KIND[L["kind"]], 2, 0, 0, 0, 0.0)
    return m._Spec(len(net), arr, m.PRECISIONS[prec]), arr


def _create_rc(m, w, net, prec="fp32", n=None):
    spec, keep = _spec(m, net, prec)
    out = ctypes.c_void_p()
    w = np.ascontiguousarray(w, dtype=np.float64)
    rc = m._lib.cnn_create(w.ctypes.data_as(ctypes.c_void_p), w.size if n is None else n,
                           ctypes.byref(spec), ctypes.byref(out))
    return rc, out


def test_create_validates_before_device_use():
    import paper_1612_02120_amd as m
    from synth.nets import NET_B, he_normal_params
    w = he_normal_params(NET_B, 200)
    rc, _ = _create_rc(m, w, NET_B, n=w.size - 1)
    assert rc == m.CNN_EINVAL and "n_weights" in m.cnn_last_error()
    bad = [dict(NET_B[1])] + NET_B  # pool first
    rc, _ = _create_rc(m, w, bad)
    assert rc == m.CNN_EINVAL
    chan = [dict(L) for L in NET_B]
    chan[2]["cin"] = 47  # channel mismatch
    rc, _ = _create_rc(m, w, chan)
    assert rc == m.CNN_EINVAL
    pool_head = NET_B[:5] + [NET_B[1], NET_B[5]]  # pooling right before the head
    rc, _ = _create_rc(m, np.zeros(w.size), pool_head)
    assert rc == m.CNN_EUNSUPPORTED
    sig = [dict(L) for L in NET_B]
    sig[-1]["act"] = "none"
    rc, _ = _create_rc(m, w, sig)
    assert rc == m.CNN_EUNSUPPORTED
    assert m._lib.cnn_create(None, 0, None, None) == m.CNN_EINVAL


def test_create_validates_fastmemb_specs_before_device_use():
    import paper_1612_02120_amd as m
    from synth.nets import NET_FM, he_normal_params
    w = he_normal_params(NET_FM, 400)
    assert m.radius_of(NET_FM) == 52  # field of view 53 (Section 2.2)
    rc, _ = _create_rc(m, w, NET_FM, n=w.size + 1)
    assert rc == m.CNN_EINVAL and "n_weights" in m.cnn_last_error()
    rc, _ = _create_rc(m, w, NET_FM, prec="fp8")
    assert rc == m.CNN_EUNSUPPORTED and "FP32 or BF16" in m.cnn_last_error()
    odd = [dict(L) for L in NET_FM]
    odd[0]["cout"] = 63  # max-out pairs channels
    rc, _ = _create_rc(m, w, odd)
    assert rc == m.CNN_EINVAL and "even" in m.cnn_last_error()
    three = [dict(L) for L in NET_FM]
    three[-1]["cout"] = 3  # the softmax output has two classes
    rc, _ = _create_rc(m, np.zeros(w.size + 32 * 16 + 1), three)
    assert rc == m.CNN_EINVAL and "two classes" in m.cnn_last_error()


def test_null_handles_are_rejected():
    import paper_1612_02120_amd as m
    assert m._lib.cnn_infer(None, None, None, None, None) == m.CNN_EINVAL
    assert m._lib.cnn_infer_batch(None, None, 0, None) == m.CNN_EINVAL
    assert m._lib.cnn_destroy(None) == m.CNN_OK
    assert m._lib.student_train_step(None, None, None, 1, 128, None, None, None, None) == m.CNN_EINVAL
    assert m._lib.cnn_geometry(None, None, None) == m.CNN_EINVAL
    assert m._lib.cnn_autotune_batch(None, None, 0, None) == m.CNN_EINVAL


def test_binding_checks_caller_buffers_before_the_library():
    """Caller buffers with a wrong dtype, shape or size are rejected by the
    binding before their pointers reach the library (an undersized or
    mistyped buffer would otherwise receive out-of-bounds device writes).
    CPU tensors stand in here: the device check comes last, so a buffer that
    passes the host-side checks fails only on being a CPU tensor."""
    torch = pytest.importorskip("torch")
    import paper_1612_02120_amd as m
    s = m.Student(None)
    net = m.Net(None, 12)
    vol = torch.zeros((2, 40, 50), dtype=torch.uint8)
    pt = torch.zeros((3, 20, 20), dtype=torch.uint8)
    tt = torch.zeros((3, 14, 14), dtype=torch.float32)

    def raises(exc, fn, *a, **k):
        with pytest.raises(exc) as e:
            fn(*a, **k)
        return str(e.value)

    # inference outputs: shape and dtype
    assert "shape" in raises(ValueError, m.cnn_infer, net, vol, out=torch.zeros((2, 28, 37)))
    assert "float32" in raises(TypeError, m.cnn_infer, net, vol, out=torch.zeros((2, 28, 38), dtype=torch.float64))
    assert "shape" in raises(ValueError, m.student_infer, s, vol, out=torch.zeros((2, 34, 43)))
    assert "CUDA" in raises(TypeError, m.student_infer, s, vol, out=torch.zeros((2, 34, 44)))
    # fallback: out in the teacher frame, stats int32[2], flags int32[tiles]
    good_out = torch.zeros((2, 28, 38))
    assert "shape" in raises(ValueError, m.student_infer_with_fallback, s, net, vol, out=torch.zeros((2, 34, 44)))
    assert "shape" in raises(ValueError, m.student_infer_with_fallback, s, net, vol, out=good_out,
                             stats=torch.zeros(1, dtype=torch.int32))
    assert "int32" in raises(TypeError, m.student_infer_with_fallback, s, net, vol, out=good_out,
                             stats=torch.zeros(2, dtype=torch.int64))
    assert "shape" in raises(ValueError, m.student_infer_with_fallback, s, net, vol, out=good_out,
                             stats=torch.zeros(2, dtype=torch.int32), tile=16,
                             flags=torch.zeros(2 * 2 * 3 - 1, dtype=torch.int32))
    assert "CUDA" in raises(TypeError, m.student_infer_with_fallback, s, net, vol, out=good_out,
                            stats=torch.zeros(2, dtype=torch.int32), tile=16,
                            flags=torch.zeros(2 * 2 * 3, dtype=torch.int32))
    # training: targets, gradient, FP64 scalars
    assert "shape" in raises(ValueError, m.student_grad, s, pt, torch.zeros((3, 14, 13)))
    assert "shape" in raises(ValueError, m.student_grad, s, pt, tt, grad_out=torch.zeros(800))
    assert "float32" in raises(TypeError, m.student_grad, s, pt, tt, grad_out=torch.zeros(801, dtype=torch.float64))
    assert "float64" in raises(TypeError, m.student_grad, s, pt, tt, grad_out=torch.zeros(801),
                               loss_out=torch.zeros(1, dtype=torch.float32))
    assert "float64" in raises(TypeError, m.student_train_step, s, pt, tt,
                               loss_out=torch.zeros(1, dtype=torch.float64), gnorm_out=torch.zeros(1))
    assert "at least" in raises(ValueError, m.student_train_step, s, pt, tt,
                                loss_out=torch.zeros(0, dtype=torch.float64), gnorm_out=torch.zeros(1, dtype=torch.float64))
    assert "CUDA" in raises(TypeError, m.student_train_step, s, pt, tt,
                            loss_out=torch.zeros(1, dtype=torch.float64), gnorm_out=torch.zeros(1, dtype=torch.float64))
