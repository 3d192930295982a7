"""Pins of the FP64 CPU reference for MaskExtend (Section 3, "MaskExtend: sparse
segmentation via CNN"), under the reading in the design notes: twelve input
maps; 4x4 convs with max-out to 32, 40, 48, 56 features, each followed by a
2x2 stride-2 pool; a fifth 4x4 conv with max-out to 64; a 1x1 conv to three
classes and a softmax, the map holding the object class. Computed densely like
FastMemb (pools as max filters, spacing doubled after each).

* field of view 109 (the paper's figure) by the receptive-field recursion;
* the dense map equals the patch form (the net on each 109 x 109 window);
* it equals the paper's fragment scheme written with torch float64 primitives
  on all 16 x 16 offsets;
* constant input maps give the scalar recursion's value;
* the three-class softmax sums to one and matches its closed form.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import maskextend_maps
from synth.nets import NET_ME, conv_layers, he_normal_params, param_count


def _params(seed=500, sigma=0.05):
    p = he_normal_params(NET_ME, seed)
    rng = np.random.default_rng(seed + 1)
    off = 0
    for L in conv_layers(NET_ME):
        n = L["cout"] * L["cin"] * L["k"] ** 2
        p[off + n:off + n + L["cout"]] = rng.normal(0, sigma, L["cout"])
        off += n + L["cout"]
    return p


def _split(params):
    out, off = [], 0
    for L in conv_layers(NET_ME):
        n = L["cout"] * L["cin"] * L["k"] ** 2
        out.append((params[off:off + n].reshape(L["cout"], L["cin"], L["k"], L["k"]),
                    params[off + n:off + n + L["cout"]]))
        off += n + L["cout"]
    return out


def _planar(maps):
    return np.ascontiguousarray(np.transpose(maps, (0, 3, 1, 2)), dtype=np.float64)


def test_field_of_view_and_parameters():
    assert oracle.radius(NET_ME) + 1 == 109
    assert param_count(NET_ME) == (64 * 12 * 16 + 64) + (80 * 32 * 16 + 80) + (96 * 40 * 16 + 96) + \
        (112 * 48 * 16 + 112) + (128 * 56 * 16 + 128) + (3 * 64 + 3) == 316067


def test_dense_equals_patch_form():
    m = _planar(maskextend_maps(31, 1, 118, 115))
    p = _params()
    dense = oracle.forward_maps(m, NET_ME, p)[0]
    assert dense.shape == (10, 7)
    for y in range(dense.shape[0]):
        for x in range(dense.shape[1]):
            assert oracle.patch_maps(m[0], NET_ME, p, y, x) == dense[y, x]


def _fragments(maps, params):
    layers = _split(params)
    C, H, W = maps.shape
    Ho, Wo = H - 108, W - 108
    dense = np.full((Ho, Wo), np.nan)
    for fy in range(16):
        for fx in range(16):
            x = torch.from_numpy(maps[:, fy:, fx:])[None]
            for li, (w, b) in enumerate(layers):
                x = torch.nn.functional.conv2d(x, torch.from_numpy(w), torch.from_numpy(b))
                if li < 5:
                    x = torch.maximum(x[:, 0::2], x[:, 1::2])
                if li < 4:
                    x = torch.nn.functional.max_pool2d(x, 2, stride=2)
            pr = torch.softmax(x, dim=1)[0, 0].numpy()
            for r in range(pr.shape[0]):
                for c in range(pr.shape[1]):
                    if fy + 16 * r < Ho and fx + 16 * c < Wo:
                        dense[fy + 16 * r, fx + 16 * c] = pr[r, c]
    return dense


def test_dense_equals_interleaved_fragments():
    m = _planar(maskextend_maps(32, 1, 140, 131))
    p = _params()
    got = oracle.forward_maps(m, NET_ME, p)[0]
    ref = _fragments(m[0], p)
    assert not np.isnan(ref).any()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_constant_maps_closed_form():
    p = _params(501, 0.1)
    rng = np.random.default_rng(3)
    for _ in range(3):
        c = rng.uniform(0, 1, 12)
        v = c.copy()
        for li, (w, b) in enumerate(_split(p)):
            v = b + w.sum(axis=(2, 3)) @ v
            if li < 5:
                v = np.maximum(v[0::2], v[1::2])
        want = np.exp(v[0] - v.max()) / np.exp(v - v.max()).sum()
        m = np.broadcast_to(c[None, :, None, None], (1, 12, 111, 112)).copy()
        got = oracle.forward_maps(m, NET_ME, p)[0]
        assert got.shape == (3, 4)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_class0_softmax_matches_definition():
    # a 1-layer net: the 1x1 three-class softmax alone
    net = [{"kind": "conv", "k": 1, "cin": 12, "cout": 3, "act": "softmax0"}]
    rng = np.random.default_rng(4)
    p = rng.normal(0, 1, 3 * 12 + 3)
    m = rng.uniform(0, 1, (1, 12, 5, 6))
    got = oracle.forward_maps(m, net, p)[0]
    z = np.einsum("oc,chw->ohw", p[:36].reshape(3, 12), m[0]) + p[36:][:, None, None]
    np.testing.assert_allclose(got, np.exp(z[0]) / np.exp(z).sum(axis=0), rtol=1e-14, atol=1e-15)
