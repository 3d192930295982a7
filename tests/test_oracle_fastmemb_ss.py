"""Pins of the FP64 CPU reference for FastMemb_ss (Section 2.2, "A subsampling
CNN for 3 nm data"), under the reading stated in the design notes: FastMemb_3nm
is FastMemb plus one more {stride-2 pool, conv(4, 32 -> 64, max-out)} pair, and
FastMemb_ss replaces its first, highest-resolution stride-2 pool by a 2x
subsample, so that 3 nm input yields a map at 6 nm. The reference's dense form
prunes the recursion to the one fragment the subsample keeps; these pins tie it
to things that do not come from that code path:

* the pruned map equals every second sample, in each direction, of the full
  dense map (the subsample keeping every position, like a pool without max);
* both equal the patch form (the net on one field-of-view window);
* both equal the paper's fragment scheme written with torch primitives;
* constant input gives the scalar recursion's value;
* the field of view (108 at 3 nm) and the cost ratios follow in closed form.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import em_volume
from synth.nets import NET_FM, NET_FM3, NET_FMSS, conv_layers, he_normal_params, param_count


def _params(seed=410, bias_sigma=0.05):
    p = he_normal_params(NET_FMSS, seed)
    rng = np.random.default_rng(seed + 1)
    off = 0
    for L in conv_layers(NET_FMSS):
        n = L["cout"] * L["cin"] * L["k"] ** 2
        p[off + n:off + n + L["cout"]] = rng.normal(0, bias_sigma, L["cout"])
        off += n + L["cout"]
    return p


def _split(params):
    out, off = [], 0
    for L in conv_layers(NET_FMSS):
        n = L["cout"] * L["cin"] * L["k"] ** 2
        out.append((params[off:off + n].reshape(L["cout"], L["cin"], L["k"], L["k"]),
                    params[off + n:off + n + L["cout"]]))
        off += n + L["cout"]
    return out


def test_field_of_view_and_output_dims():
    # r += (k - 1) j, j doubled by each stride-2 layer; a subsample has a
    # one-pixel window: 3 + 2*3 + 2 + 4*3 + 4 + 8*3 + 8 + 16*3 = 107
    assert oracle.radius(NET_FMSS) == 107
    assert oracle.radius(NET_FM3) == 108
    assert param_count(NET_FMSS) == param_count(NET_FM3) == 67778 + 32 * 64 * 16 + 64
    for H, W in ((108, 108), (109, 140), (200, 211)):
        assert oracle.out_dims(NET_FMSS, H, W) == ((H - 108) // 2 + 1, (W - 108) // 2 + 1)
        assert oracle.out_dims(NET_FMSS, H, W, full=True) == (H - 107, W - 107)


def test_pruned_equals_every_second_sample_of_full_dense_map():
    img = em_volume(21, 2, 131, 124)
    p = _params()
    pruned = oracle.forward(img, NET_FMSS, p)
    full = oracle.forward_full(img, NET_FMSS, p)
    assert pruned.shape == (2, 12, 9) and full.shape == (2, 24, 17)
    assert np.array_equal(pruned, full[:, ::2, ::2])


def test_full_dense_equals_patch_form_everywhere():
    img = em_volume(22, 1, 115, 113)[0]
    p = _params()
    full = oracle.forward_full(img, NET_FMSS, p)[0]
    for y in range(full.shape[0]):
        for x in range(full.shape[1]):
            assert oracle.patch(img, NET_FMSS, p, y, x)[0] == full[y, x]


def _fragments(img, params):
    """The paper's scheme with torch float64 primitives: the 1 -> 64 conv and
    max-out on the 3 nm image, the 2x subsample, then the strided net (stride-1
    convs, stride-2 pools) on each of the 8 x 8 offsets of the subsampled map;
    fragment (fy, fx), output (r, c) is the map at (fy + 8r, fx + 8c)."""
    layers = _split(params)
    x = torch.from_numpy(img.astype(np.float64) / 255.0)[None, None]
    w, b = layers[0]
    x = torch.nn.functional.conv2d(x, torch.from_numpy(w), torch.from_numpy(b))
    x = torch.maximum(x[:, 0::2], x[:, 1::2])[:, :, ::2, ::2]
    hs, ws = x.shape[2], x.shape[3]
    Ho, Wo = hs - 52, ws - 52
    dense = np.full((Ho, Wo), np.nan)
    for fy in range(8):
        for fx in range(8):
            y = x[:, :, fy:, fx:]
            for li, (w, b) in enumerate(layers[1:]):
                y = torch.nn.functional.conv2d(y, torch.from_numpy(w), torch.from_numpy(b))
                if li < 3:
                    y = torch.maximum(y[:, 0::2], y[:, 1::2])
                    y = torch.nn.functional.max_pool2d(y, 2, stride=2)
            pr = torch.softmax(y, dim=1)[0, 1].numpy()
            for r in range(pr.shape[0]):
                for c in range(pr.shape[1]):
                    if fy + 8 * r < Ho and fx + 8 * c < Wo:
                        dense[fy + 8 * r, fx + 8 * c] = pr[r, c]
    return dense


def test_pruned_equals_interleaved_fragments():
    img = em_volume(23, 1, 140, 126)[0]
    p = _params()
    got = oracle.forward(img, NET_FMSS, p)[0]
    ref = _fragments(img, p)
    assert got.shape == ref.shape == (17, 10) and not np.isnan(ref).any()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_constant_input_closed_form():
    p = _params(seed=411, bias_sigma=0.1)
    for val in (0, 90, 255):
        v = np.array([val / 255.0])
        for li, (w, b) in enumerate(_split(p)):
            v = b + w.sum(axis=(2, 3)) @ v
            if li < 4:
                v = np.maximum(v[0::2], v[1::2])
        want = np.exp(v[1]) / (np.exp(v[0]) + np.exp(v[1]))
        got = oracle.forward(np.full((1, 112, 113), val, np.uint8), NET_FMSS, p)[0]
        assert got.shape == (3, 3)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def _macs_per_output(net, pruned=True):
    """Multiply-adds per output pixel of the dense form: each conv's
    cin * cout * k^2 per position it is evaluated at, relative to the output
    grid. Layers before a subsample run at 4x the output's pixel count when the
    subsample keeps every position; the pruned form evaluates them only where
    the subsample keeps them."""
    total, scale = 0, 1
    sub_seen = False
    for L in reversed(net):
        if L["kind"] == "sub2":
            sub_seen = True
            scale = 1 if pruned else 4
        elif L["kind"] == "conv":
            total += scale * L["cin"] * L["cout"] * L["k"] ** 2
    return total


def test_cost_ratios_closed_form():
    # FastMemb_6nm per 6 nm output: 16 (1*64 + 2*32*64 + 32*2) = 67,584 MAC.
    fm = _macs_per_output(NET_FM)
    assert fm == 16 * (64 + 2 * 2048 + 64) == 67584
    # FastMemb_ss per 6 nm output: one more 32 -> 64 conv; the 1 -> 64 conv is
    # needed only at the positions the subsample keeps (pruned form).
    ss = _macs_per_output(NET_FMSS)
    assert ss == 16 * (64 + 3 * 2048 + 64) == 100352
    assert ss / fm == pytest.approx(6272 / 4224)  # 1.485x (the paper prints 1.17x)
    # the full dense form of the same net (every 3 nm position) and FastMemb_3nm
    # (4x the pixels of the 6 nm map, one extra pair): 5.94x (the paper: 5.68x / 5.86x)
    assert _macs_per_output(NET_FM3) * 4 / fm == pytest.approx(4 * 6272 / 4224)
    assert _macs_per_output(NET_FMSS, pruned=False) == 4 * 16 * 64 + 16 * 3 * 2048 + 16 * 64


def _patch_macs(net, fov):
    """Multiply-adds of the patch form (the net on one fov x fov window)."""
    h, c, total = fov, 1, 0
    for L in net:
        if L["kind"] == "conv":
            h -= L["k"] - 1
            total += h * h * L["cin"] * L["cout"] * L["k"] ** 2
        elif L["kind"] in ("pool2", "sub2"):
            h = (h + 1) // 2 if L["kind"] == "sub2" else h // 2
    return total


def test_patch_versus_dense_multiplication_ratio():
    # Section 2.2 credits dense computation of FastMemb with about 284x fewer
    # multiplications than sliding-window patches. With the 1 -> 64, 32 -> 64,
    # 32 -> 64, 32 -> 2 reading: patch 50^2*64*16 + 22^2*2048*16 + 8^2*2048*16
    # + 1*64*16 = 20,517,888 MAC against 67,584 per dense output: 303.6x.
    patch = _patch_macs(NET_FM, 53)
    assert patch == 50 * 50 * 64 * 16 + 22 * 22 * 2048 * 16 + 8 * 8 * 2048 * 16 + 64 * 16 == 20517888
    assert patch / _macs_per_output(NET_FM) == pytest.approx(303.6, abs=0.05)


def test_subsample_rejects_quantised_modes_and_late_placement():
    vol = em_volume(24, 1, 120, 120)
    with pytest.raises(ValueError):
        oracle.forward(vol, NET_FMSS, _params(), qmode="bf16")
    late = NET_FM[:2] + [{"kind": "sub2"}] + NET_FM[2:]  # a subsample after a stride-2 pool
    with pytest.raises(ValueError):
        oracle.out_dims(late, 200, 200)
