"""Pins of the FP64 CPU reference for FastMemb, the paper's own net (Section 2.2).

FastMemb alternates 4x4 convolutions (32 features, max-out over channel pairs)
with 2x2 stride-2 max-pools and ends in a two-class softmax. Its dense output is
what a sliding-window classifier gives at every position. The paper computes it
by splitting each k-stride operation into k^2 fragments and interleaving them;
the reference computes it with max filters and spaced (dilated) convolutions.
The pins below check that reference against facts that do not come from it.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import em_volume
from synth.nets import NET_FM, calibrated_params, conv_layers, param_count


def test_field_of_view_and_parameter_count():
    # Section 2.2: 4x4 kernels and three 2x2/s2 pools give a 53 x 53 field of
    # view; the reading 1->64, 32->64, 32->64 (max-out to 32), 32->2 has
    # 67,778 parameters, the paper's "70k".
    assert oracle.radius(NET_FM) + 1 == 53
    assert oracle.lib().orc_radius(oracle._layers(NET_FM), len(NET_FM)) == 52
    assert param_count(NET_FM) == 67778


def _split(params):
    out, off = [], 0
    for L in conv_layers(NET_FM):
        n = L["cout"] * L["cin"] * L["k"] ** 2
        out.append((params[off:off + n].reshape(L["cout"], L["cin"], L["k"], L["k"]),
                    params[off + n:off + n + L["cout"]]))
        off += n + L["cout"]
    return out


def _fragments_interleaved(img, params):
    """The paper's fragment scheme, written with torch float64 primitives: the
    strided net (stride-1 convs, stride-2 pools) runs on every one of the 8 x 8
    input offsets; output (r, c) of fragment (fy, fx) is the dense output at
    (fy + 8r, fx + 8c). Interleaving the fragments gives the dense map."""
    H, W = img.shape
    R = 52
    Ho, Wo = H - R, W - R
    dense = np.full((Ho, Wo), np.nan)
    layers = _split(params)
    for fy in range(8):
        for fx in range(8):
            x = torch.from_numpy(img[fy:, fx:].astype(np.float64) / 255.0)[None, None]
            for li, (w, b) in enumerate(layers):
                x = torch.nn.functional.conv2d(x, torch.from_numpy(w), torch.from_numpy(b))
                if li < 3:
                    x = torch.maximum(x[:, 0::2], x[:, 1::2])  # max-out over channel pairs
                    x = torch.nn.functional.max_pool2d(x, 2, stride=2)
            p = torch.softmax(x, dim=1)[0, 1].numpy()
            for r in range(p.shape[0]):
                for c in range(p.shape[1]):
                    y, xx = fy + 8 * r, fx + 8 * c
                    if y < Ho and xx < Wo:
                        dense[y, xx] = p[r, c]
    return dense


def test_dense_equals_interleaved_fragments():
    img = em_volume(11, 1, 77, 70)[0]
    p = calibrated_params("FM")
    got = oracle.forward(img, NET_FM, p)[0]
    ref = _fragments_interleaved(img, p)
    assert not np.isnan(ref).any()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_dense_equals_patch_form_everywhere():
    # the sliding-window definition, one field-of-view window per output
    img = em_volume(12, 1, 61, 66)[0]
    p = calibrated_params("FM")
    got = oracle.forward(img, NET_FM, p)[0]
    for y in range(got.shape[0]):
        for x in range(got.shape[1]):
            assert oracle.patch(img, NET_FM, p, y, x)[0] == got[y, x]


def test_constant_input_closed_form():
    # On a constant image every map is spatially constant: a conv maps channel
    # values v to b + (sum of each kernel) . v, max-out takes pair maxima,
    # pooling is the identity, and the output is the class-1 softmax.
    rng = np.random.default_rng(5)
    p = calibrated_params("FM") + rng.normal(0, 0.05, size=param_count(NET_FM))
    for val in (0, 77, 255):
        v = np.array([val / 255.0])
        for li, (w, b) in enumerate(_split(p)):
            v = b + w.sum(axis=(2, 3)) @ v
            if li < 3:
                v = np.maximum(v[0::2], v[1::2])
        want = np.exp(v[1]) / (np.exp(v[0]) + np.exp(v[1]))
        img = np.full((1, 56, 57), val, dtype=np.uint8)
        got = oracle.forward(img, NET_FM, p)[0]
        assert got.shape == (4, 5)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_translation_equivariance_bitwise():
    vol = em_volume(13, 1, 70, 72)[0]
    p = calibrated_params("FM")
    a = oracle.forward(vol, NET_FM, p)[0]
    b = oracle.forward(vol[3:, 5:], NET_FM, p)[0]
    assert np.array_equal(a[3:, 5:], b)


def test_softmax_logit_is_class_difference():
    vol = em_volume(14, 1, 60, 60)[0]
    p = calibrated_params("FM")
    prob = oracle.forward(vol, NET_FM, p)[0]
    lg = oracle.forward(vol, NET_FM, p, logits=True)[0]
    np.testing.assert_allclose(prob, 1.0 / (1.0 + np.exp(-lg)), rtol=0, atol=1e-15)


def test_strided_nets_reject_quantised_modes():
    vol = em_volume(15, 1, 60, 60)
    with pytest.raises(ValueError):
        oracle.forward(vol, NET_FM, calibrated_params("FM"), qmode="bf16")
