"""Layer-by-layer, element-wise pins of the BF16 and FP8 forms of net B.

Each stored inter-layer map of the GPU (read back with cnn_read_activation)
is checked against the oracle's single-layer reference evaluated on the GPU's
own input map of that layer, so every layer is judged on its own arithmetic:

* a stored code (e4m3fn, or bf16 value) must lie between the codes of the
  oracle's FP64 value moved down and up by the layer's accumulation-error
  bound (rounding is monotone, so any sum within the bound rounds into that
  range); the bound is FP8_ACC_REL (FP8 matrix instructions, measured by
  tests/test_gpu_mfma.py) or FP32 accumulation for BF16, times the oracle's
  sum of |products|, plus the FP32 epilogue roundings;
* the last body conv with the fused head and sigmoid: the probability must be
  within 1/4 of the logit bound (the sigmoid's largest slope) of the
  oracle's, whose input is the GPU's last stored map.

The share of stored values that differ from the oracle's nominal rounding is
printed: only values next to a rounding boundary may differ.
"""
import numpy as np
import pytest

import oracle
from synth import em_volume
from synth.nets import NET_B, calibrated_params, fp8_act_scales, random_bias_params
from tests.bounds import BF16_ACC_REL, FP8_ACC_REL, U32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def emcnn():
    import paper_1612_02120_amd as m
    assert torch.cuda.is_available()
    return m


def _convs(p):
    """(W, b, k) of every conv of net B, from the flat parameter vector."""
    out, o = [], 0
    for L in NET_B:
        if L["kind"] == "conv":
            nw = L["cout"] * L["cin"] * L["k"] ** 2
            out.append((p[o:o + nw], p[o + nw:o + nw + L["cout"]], L["k"]))
            o += nw + L["cout"]
    return out


def _decode(t, prec):
    """Stored channel-blocked map (Z x C/16 x h x w x 16) -> float64 Z x C x h x w."""
    if prec == "fp8":
        v = t.cpu().view(torch.float8_e4m3fn).to(torch.float64)
    else:
        v = t.cpu().to(torch.float64)
    Z, CB, h, w, _ = v.shape
    return v.permute(0, 1, 4, 2, 3).reshape(Z, CB * 16, h, w).numpy()


def _round(x, prec):
    return oracle.e4m3_round(x) if prec == "fp8" else oracle.bf16_round(x)


def _check_stored(got, val, eps, scale, prec, what):
    """got: stored values in units of the code (a / scale for FP8, a for BF16);
    val: oracle FP64 conv output before ReLU; eps: its error bound."""
    inv = 1.0 / scale
    lo = _round(np.maximum(val - eps, 0.0) * inv * (1 - 4 * U32), prec)
    hi = _round(np.maximum(val + eps, 0.0) * inv * (1 + 4 * U32), prec)
    nominal = _round(np.maximum(val, 0.0) * inv, prec)
    bad = (got < lo) | (got > hi)
    print("%s: %d values, %d off the nominal rounding (%.2e), %d outside the bound"
          % (what, got.size, int((got != nominal).sum()), (got != nominal).mean(), int(bad.sum())))
    assert not bad.any(), np.argwhere(bad)[:5]
    return (got != nominal).mean()


@pytest.mark.parametrize("prec,params", [("fp8", "calibrated"), ("fp8", "random"), ("bf16", "calibrated")])
def test_layers_elementwise(emcnn, prec, params):
    vol = em_volume(81, 2, 70, 90)
    p = calibrated_params("B") if params == "calibrated" else random_bias_params(NET_B, 200, 83, sigma=0.1)
    sc = fp8_act_scales("B") if prec == "fp8" else [None, 1.0, 1.0, None]
    h = emcnn.cnn_create(p, NET_B, prec, act_scales=sc if prec == "fp8" else None)
    prob = emcnn.cnn_infer(h, torch.from_numpy(vol).cuda())
    a0, sh0 = emcnn.cnn_read_activation(h, 0)
    a1, sh1 = emcnn.cnn_read_activation(h, 1)
    torch.cuda.synchronize()
    g0, g1 = _decode(a0, prec), _decode(a1, prec)
    P = prob.cpu().numpy().astype(np.float64)
    (w1, b1, k1), (w2, b2, k2), (w3, b3, k3), (wh, bh, _) = _convs(p)
    acc = FP8_ACC_REL if prec == "fp8" else BF16_ACC_REL
    for z in range(vol.shape[0]):
        # layer 0: bf16(w / 255) against the raw uint8 input, FP32 accumulation
        w1q = oracle.bf16_round(w1 / 255.0)
        v0, m0 = oracle.conv_layer(vol[z][None].astype(np.float64), w1q, b1, k1)
        e0 = BF16_ACC_REL * m0 + 2 * U32 * (np.abs(v0) + np.abs(b1)[:, None, None])
        _check_stored(g0[z], v0, e0, sc[1] if prec == "fp8" else 1.0, prec, "%s layer 0, slice %d" % (prec, z))
        # layer 1: max filter, then conv2 on the GPU's stored layer-0 values
        a_in = g0[z] * (sc[1] if prec == "fp8" else 1.0)
        v1, m1 = oracle.conv_layer(a_in, w2, b2, k2, pool=True, qmode=prec, in_scale=sc[1] if prec == "fp8" else 0.0)
        e1 = acc * m1 + 3 * U32 * (np.abs(v1) + np.abs(b2)[:, None, None])
        _check_stored(g1[z], v1, e1, sc[2] if prec == "fp8" else 1.0, prec, "%s layer 1, slice %d" % (prec, z))
        # last body conv + 1x1 head + sigmoid on the GPU's stored layer-1 values
        a_in = g1[z] * (sc[2] if prec == "fp8" else 1.0)
        v2, m2 = oracle.conv_layer(a_in, w3, b3, k3, pool=True, qmode=prec, in_scale=sc[2] if prec == "fp8" else 0.0)
        e2 = acc * m2 + 3 * U32 * (np.abs(v2) + np.abs(b3)[:, None, None])
        hrelu = np.maximum(v2, 0.0)
        logit = bh[0] + np.tensordot(wh, hrelu, axes=(0, 0))
        elog = np.tensordot(np.abs(wh), e2, axes=(0, 0)) + 50 * U32 * (np.tensordot(np.abs(wh), hrelu, axes=(0, 0))
                                                                       + abs(bh[0]))
        ref = 1.0 / (1.0 + np.exp(-logit))
        err = np.abs(P[z] - ref)
        bound = 0.25 * elog + 1e-6
        print("%s head, slice %d: max |p - ref| %.3g, max bound %.3g, max err / bound %.3g"
              % (prec, z, err.max(), bound.max(), (err / bound).max()))
        assert (err <= bound).all()
