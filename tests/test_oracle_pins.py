"""Pins of the FP64 CPU reference against facts that do not come from itself.

Each test names the property of the method (Section 2.2: dense valid
convolution, stride-1 max filtering, two-class softmax output) or of the number
format that it checks.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from synth import em_slice, em_volume
from synth.nets import NET_A, NET_B, NET_S, he_normal_params, random_bias_params, param_count
from tests import bruteforce


def _conv(k, cin, cout, act):
    return {"kind": "conv", "k": k, "cin": cin, "cout": cout, "act": act}


POOL = {"kind": "pool"}
TINY_NET = [_conv(3, 1, 3, "relu"), POOL, _conv(3, 3, 3, "relu"), POOL, _conv(2, 3, 2, "relu"),
            _conv(1, 2, 1, "sigmoid")]


def test_param_counts_and_radius():
    # Net geometry: R = sum(k-1) over convs + 1 per 2x2/s1 filter; FoV = R + 1.
    assert param_count(NET_A) == 6849 and oracle.radius(NET_A) == 8
    assert param_count(NET_B) == 79729 and oracle.radius(NET_B) == 12
    assert param_count(NET_S) == 801 and oracle.radius(NET_S) == 6


def test_bruteforce_bitwise_tiny():
    rng = np.random.default_rng(7)
    vol = rng.integers(0, 256, size=(2, 13, 11), dtype=np.uint8)
    p = random_bias_params(TINY_NET, 11, 12, sigma=0.3)
    got = oracle.forward(vol, TINY_NET, p)
    for z in range(2):
        ref = np.array(bruteforce.forward_slice(vol[z].tolist(), TINY_NET, p.tolist()))
        assert got[z].shape == ref.shape
        assert np.array_equal(got[z], ref), np.abs(got[z] - ref).max()


def test_bruteforce_bitwise_net_a_window():
    img = em_slice(1, 0, 14, 12)
    p = random_bias_params(NET_A, 100, 5)
    got = oracle.forward(img[None], NET_A, p)[0]
    ref = np.array(bruteforce.forward_slice(img.tolist(), NET_A, p.tolist()))
    assert np.array_equal(got, ref)


def _torch_forward(vol, net, params):
    x = torch.from_numpy(vol.astype(np.float64) / 255.0)[:, None]
    off = 0
    outs = []
    for L in net:
        if L["kind"] == "pool":
            x = torch.nn.functional.max_pool2d(x, 2, stride=1)
            outs.append(x.numpy())
            continue
        k, ci, co = L["k"], L["cin"], L["cout"]
        nw = co * ci * k * k
        w = torch.from_numpy(params[off:off + nw].reshape(co, ci, k, k))
        b = torch.from_numpy(params[off + nw:off + nw + co])
        off += nw + co
        x = torch.nn.functional.conv2d(x, w, b)
        if L["act"] == "relu":
            x = torch.relu(x)
        elif L["act"] == "sigmoid":
            x = torch.sigmoid(x)
    return x[:, 0].numpy()


@pytest.mark.parametrize("name,net", [("A", NET_A), ("B", NET_B), ("S", NET_S)])
def test_torch_conv2d_float64(name, net):
    vol = em_volume(3, 2, 41, 37)
    p = random_bias_params(net, 1 + len(name), 9)
    got = oracle.forward(vol, net, p)
    ref = _torch_forward(vol, net, p)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-12


@pytest.mark.parametrize("p,q", [(0, 0), (1, 3), (4, 2), (3, 4)])
def test_delta_kernel_identity(p, q):
    # A delta at (p, q) copies in[y+p][x+q]: pins cross-correlation orientation
    # and the position of the valid output window.
    net = [_conv(5, 1, 1, "none")]
    w = np.zeros(26)
    w[p * 5 + q] = 1.0
    img = em_slice(5, 0, 19, 23)
    got = oracle.forward(img[None], net, w)[0]
    assert np.array_equal(got, img[p:p + 15, q:q + 19] / 255.0)


def test_constant_input_closed_form():
    # Constant input c: every layer's map is constant per channel, obtained by the
    # scalar recursion v'[co] = b[co] + sum_ci v[ci] * sum_ij W[co][ci]; pools keep it.
    net = NET_B
    p = random_bias_params(net, 200, 3, sigma=0.2)
    for c in (0, 17, 200, 255):
        vol = np.full((1, 30, 27), c, dtype=np.uint8)
        got = oracle.forward(vol, net, p)[0]
        v = np.array([c / 255.0])
        off = 0
        for L in net:
            if L["kind"] == "pool":
                continue
            k, ci, co = L["k"], L["cin"], L["cout"]
            nw = co * ci * k * k
            w = p[off:off + nw].reshape(co, ci, k * k).sum(axis=2)
            b = p[off + nw:off + nw + co]
            off += nw + co
            v = b + w @ v
            if L["act"] == "relu":
                v = np.maximum(v, 0.0)
            else:
                v = 1.0 / (1.0 + np.exp(-v))
        assert got.shape == (18, 15)
        assert np.allclose(got, v[0], rtol=1e-12, atol=0)
        assert np.ptp(got) == 0.0


def test_translation_equivariance_bitwise():
    # Dense valid computation has no dependence on absolute position.
    vol = em_volume(8, 1, 50, 47)
    p = random_bias_params(NET_B, 200, 4)
    full = oracle.forward(vol, NET_B, p)
    for dy, dx in [(1, 0), (0, 3), (5, 7)]:
        sh = oracle.forward(vol[:, dy:, dx:], NET_B, p)
        assert np.array_equal(sh, full[:, dy:, dx:])


def test_slice_independence():
    vol = em_volume(9, 3, 33, 30)
    p = he_normal_params(NET_A, 100)
    full = oracle.forward(vol, NET_A, p)
    for z in range(3):
        assert np.array_equal(oracle.forward(vol[z:z + 1], NET_A, p)[0], full[z])


def test_thread_count_does_not_change_result():
    vol = em_volume(10, 1, 40, 40)
    p = random_bias_params(NET_B, 200, 6)
    a = oracle.forward(vol, NET_B, p, threads=1)
    b = oracle.forward(vol, NET_B, p, threads=4)
    assert np.array_equal(a, b)


def test_sigmoid_special_values():
    # Sigmoid equals the two-class softmax; symmetric, 1/2 at 0, no overflow.
    assert oracle.sigmoid(0.0) == 0.5
    for t in (1e-3, 0.5, 3.0, 20.0, 700.0, 1000.0):
        a, b = oracle.sigmoid(t), oracle.sigmoid(-t)
        assert abs((a + b) - 1.0) <= 2.3e-16
        assert a == pytest.approx(1.0 / (1.0 + math.exp(-t)), rel=1e-15)
        sm = math.exp(t / 2) / (math.exp(t / 2) + math.exp(-t / 2)) if t < 700 else 1.0
        assert a == pytest.approx(sm, rel=1e-14)


def test_relu_pool_commute():
    # ReLU then 2x2 max equals 2x2 max then ReLU (max is monotone): lets a fused
    # kernel pool either before or after the activation, bitwise.
    rng = np.random.default_rng(3)
    a = torch.from_numpy(rng.normal(size=(4, 20, 17)))
    r1 = torch.nn.functional.max_pool2d(torch.relu(a)[None], 2, stride=1)
    r2 = torch.relu(torch.nn.functional.max_pool2d(a[None], 2, stride=1))
    assert torch.equal(r1, r2)


def test_bf16_encoder_exhaustive():
    # Every bf16 value round-trips; random float32 values match torch's RNE cast.
    bits = np.arange(0, 1 << 16, dtype=np.uint32) << 16
    vals = bits.view(np.float32).astype(np.float64)
    fin = np.isfinite(vals)
    assert np.array_equal(oracle.bf16_round(vals[fin]), vals[fin])
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=200000) * 10.0 ** rng.integers(-30, 30, size=200000),
                        (bits[fin[: len(bits)]].view(np.float32).astype(np.float64) * (1 + 2.0 ** -8))[:50000]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = oracle.bf16_round(x32.astype(np.float64))
    ok = np.isfinite(ref)
    assert np.array_equal(got[ok], ref[ok])


def test_e4m3_encoder_against_torch():
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    fin = np.isfinite(codes)
    assert fin.sum() == 254  # 0x7f and 0xff are NaN
    assert np.array_equal(oracle.e4m3_round(codes[fin]), codes[fin])
    assert np.nanmax(codes) == 448.0
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(-464, 464, 100000), rng.normal(size=100000) * 2.0 ** -7,
                        rng.normal(size=100000)])
    # midpoints between neighbouring codes: ties go to the even code
    fc = np.sort(codes[fin & (codes >= 0)])
    mids = (fc[1:] + fc[:-1]) / 2
    x = np.concatenate([x, mids, -mids])
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = oracle.e4m3_round(x)
    assert np.array_equal(got, ref)
    # saturation beyond the largest finite value
    big = np.array([465.0, 1000.0, 1e30, -500.0])
    assert np.array_equal(oracle.e4m3_round(big), np.array([448.0, 448.0, 448.0, -448.0]))


def _fake_quant_reference(vol, net, p, mode, scales, layers=False):
    """The declared fake-quant forms composed from library primitives (torch
    float64 conv2d) and the separately pinned encoders. layers: also return
    every layer's output (Z x C x h x w)."""
    x = torch.from_numpy(vol.astype(np.float64))[:, None]  # raw uint8 values
    off, first, ci_idx = 0, True, 0
    nconv = sum(1 for L in net if L["kind"] == "conv")
    outs = []
    for L in net:
        if L["kind"] == "pool":
            x = torch.nn.functional.max_pool2d(x, 2, stride=1)
            outs.append(x.numpy())
            continue
        k, ci, co = L["k"], L["cin"], L["cout"]
        nw = co * ci * k * k
        w = p[off:off + nw].reshape(co, ci, k, k)
        b = torch.from_numpy(p[off + nw:off + nw + co])
        off += nw + co
        head = ci_idx == nconv - 1 and k == 1 and co == 1
        if first:
            wq = torch.from_numpy(oracle.bf16_round(w / 255.0))
            y = torch.nn.functional.conv2d(x, wq, b)
        elif head:
            y = torch.nn.functional.conv2d(x, torch.from_numpy(w), b)
        elif mode == "bf16":
            xq = torch.from_numpy(oracle.bf16_round(x.numpy()))
            y = torch.nn.functional.conv2d(xq, torch.from_numpy(oracle.bf16_round(w)), b)
        else:
            s = scales[ci_idx]
            sw = np.abs(w).reshape(co, -1).max(axis=1) / 448.0
            wq = oracle.e4m3_round(w / sw[:, None, None, None])
            xq = torch.from_numpy(oracle.e4m3_round(x.numpy() / s))
            y = torch.nn.functional.conv2d(xq, torch.from_numpy(wq))
            y = b[None, :, None, None] + torch.from_numpy(s * sw)[None, :, None, None] * y
        first = False
        ci_idx += 1
        if L["act"] == "relu":
            y = torch.relu(y)
        elif L["act"] == "sigmoid":
            y = torch.sigmoid(y)
        x = y
        outs.append(x.numpy())
    if layers:
        return x[:, 0].numpy(), outs
    return x[:, 0].numpy()


@pytest.mark.parametrize("mode", ["bf16", "fp8"])
def test_fake_quant_composition(mode):
    vol = em_volume(12, 2, 36, 33)
    p = random_bias_params(NET_B, 200, 13)
    scales = [None, 0.0049, 0.0053, None]
    got = oracle.forward(vol, NET_B, p, qmode=mode, act_scales=scales)
    ref = _fake_quant_reference(vol, NET_B, p, mode, scales)
    assert np.abs(got - ref).max() <= 1e-12
    exact = oracle.forward(vol, NET_B, p)
    # the quantised forms stay close to the exact one (sanity, not a pin)
    assert np.abs(got - exact).max() < (0.02 if mode == "bf16" else 0.08)


def test_fp8_weight_scale_maps_max_to_448():
    w = np.array([[0.3, -1.7, 0.2], [0.05, 0.01, -0.02]])
    sw = np.abs(w).max(axis=1) / 448.0
    q = oracle.e4m3_round(w / sw[:, None])
    assert q[0, 1] == -448.0 and q[1, 0] == 448.0


@pytest.mark.parametrize("mode", ["exact", "bf16", "fp8"])
def test_fake_quant_trace_and_single_layer(mode):
    """The per-layer trace in each number format equals the torch composition
    layer by layer; the single-layer reference (conv_layer) applied to a traced
    map reproduces the next traced conv; its |product| sums are checked by
    brute force at sampled outputs."""
    vol = em_volume(12, 1, 36, 33)
    p = random_bias_params(NET_B, 200, 13)
    scales = [None, 0.0049, 0.0053, None]
    tr = oracle.trace(vol[0], NET_B, p, qmode=mode, act_scales=None if mode == "exact" else scales)
    if mode == "exact":
        ref = [a[0] for a in _torch_layers(vol, NET_B, p)]
    else:
        ref = [a[0] for a in _fake_quant_reference(vol, NET_B, p, mode, scales, layers=True)[1]]
    assert len(tr) == len(ref) == len(NET_B)
    for l, (a, b) in enumerate(zip(tr, ref)):
        assert a.shape == b.shape, l
        assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max()), l
    offs, o = [], 0
    for L in NET_B:
        if L["kind"] == "conv":
            offs.append(o)
            o += L["cout"] * L["cin"] * L["k"] ** 2 + L["cout"]
    for ci, (lin, lout) in ((1, (0, 2)), (2, (2, 4))):
        L = NET_B[lout]
        nw = L["cout"] * L["cin"] * L["k"] ** 2
        w, b = p[offs[ci]:offs[ci] + nw], p[offs[ci] + nw:offs[ci] + nw + L["cout"]]
        out, absum = oracle.conv_layer(tr[lin], w, b, L["k"], pool=True, qmode=mode,
                                       in_scale=0.0 if mode == "exact" else scales[ci])
        assert np.abs(np.maximum(out, 0) - tr[lout]).max() <= 1e-12 * max(1.0, np.abs(tr[lout]).max())
        assert (absum + 1e-12 >= np.abs(out - b[:, None, None])).all()
        # brute force of the scaled |product| sum at a few outputs
        a = torch.nn.functional.max_pool2d(torch.from_numpy(tr[lin])[None], 2, stride=1)[0].numpy()
        W = w.reshape(L["cout"], L["cin"], L["k"], L["k"])
        if mode == "fp8":
            sw = np.abs(W).reshape(L["cout"], -1).max(axis=1) / 448.0
            Wq, aq, osc = oracle.e4m3_round(W / sw[:, None, None, None]), oracle.e4m3_round(a / scales[ci]), scales[ci] * sw
        elif mode == "bf16":
            Wq, aq, osc = oracle.bf16_round(W), oracle.bf16_round(a), np.ones(L["cout"])
        else:
            Wq, aq, osc = W, a, np.ones(L["cout"])
        rng = np.random.default_rng(5)
        for _ in range(6):
            co = int(rng.integers(0, L["cout"]))
            y = int(rng.integers(0, out.shape[1]))
            x = int(rng.integers(0, out.shape[2]))
            win = aq[:, y:y + L["k"], x:x + L["k"]]
            assert absum[co, y, x] == pytest.approx(osc[co] * np.abs(Wq[co] * win).sum(), rel=1e-12)
            assert out[co, y, x] == pytest.approx(b[co] + osc[co] * (Wq[co] * win).sum(), rel=1e-12, abs=1e-12)


def _torch_layers(vol, net, params):
    """Every layer's output of the exact net, composed from torch float64 ops."""
    x = torch.from_numpy(vol.astype(np.float64) / 255.0)[:, None]
    off, outs = 0, []
    for L in net:
        if L["kind"] == "pool":
            x = torch.nn.functional.max_pool2d(x, 2, stride=1)
        else:
            k, ci, co = L["k"], L["cin"], L["cout"]
            nw = co * ci * k * k
            w = torch.from_numpy(params[off:off + nw].reshape(co, ci, k, k))
            b = torch.from_numpy(params[off + nw:off + nw + co])
            off += nw + co
            x = torch.nn.functional.conv2d(x, w, b)
            x = torch.relu(x) if L["act"] == "relu" else torch.sigmoid(x)
        outs.append(x.numpy())
    return outs
