"""Layer specifications and seeded weights of the three membrane nets.

The paper's FastMemb alternates convolutions with max-pooling, and computes the
dense output by replacing pooling with stride-1 max-filtering (Section 2.2,
"Accelerating dense computation"). The nets below are that shape of network:

* NET_A - tiny: conv5x5 1->16 ReLU, conv5x5 16->16 ReLU, conv1x1 16->1 sigmoid.
* NET_B - teacher: conv5x5 1->48 ReLU, maxpool 2x2/s1, conv5x5 48->48 ReLU,
  maxpool 2x2/s1, conv3x3 48->48 ReLU, conv1x1 48->1 sigmoid.
* NET_S - student: conv5x5 1->8 ReLU, conv3x3 8->8 ReLU, conv1x1 8->1 sigmoid.
* NET_FM - FastMemb as the paper describes it (Section 2.2): three pairs of a
  4x4 conv with 32 features (max-out over channel pairs of a 64-channel conv)
  and a 2x2 stride-2 max-pool, then a 4x4 conv to two classes and a softmax;
  no other transfer function. Field of view 53, 67,778 parameters. Computed
  densely, each stride-2 pool becomes a max filter and doubles the spacing of
  every later layer.

A layer is a dict: ``{"kind": "conv", "k", "cin", "cout", "act"}`` with act in
{"none", "relu", "sigmoid", "maxout", "softmax", "softmax0"}, or ``{"kind": "pool"}``
(2x2 window, stride 1), ``{"kind": "pool2"}`` (2x2 window, stride 2) or
``{"kind": "sub2"}`` (keep every second pixel in each direction).

Parameter vectors are float64, conv layers in order, each as W[cout][cin][k][k]
(C order) followed by b[cout].

Weights: He-normal, W ~ N(0, 2/(cin k^2)), drawn with numpy ``default_rng(seed)``
layer by layer in the order above; hidden biases are 0. The head bias of A and B
is set from a stored calibration (``calibration.json``), the negated median of
the head pre-activation on a calibration slice (seed 99), so that the 0.5
threshold splits the output map roughly in half. The same file stores the
per-layer FP8 activation scales of net B. The file is written by a committed
script of the CPU reference and is plain data here.
"""
from __future__ import annotations

import json
import os

import numpy as np


def _conv(k, cin, cout, act):
    return {"kind": "conv", "k": k, "cin": cin, "cout": cout, "act": act}


POOL = {"kind": "pool"}
POOL2 = {"kind": "pool2"}

NET_A = [_conv(5, 1, 16, "relu"), _conv(5, 16, 16, "relu"), _conv(1, 16, 1, "sigmoid")]
NET_B = [_conv(5, 1, 48, "relu"), POOL, _conv(5, 48, 48, "relu"), POOL,
         _conv(3, 48, 48, "relu"), _conv(1, 48, 1, "sigmoid")]
NET_S = [_conv(5, 1, 8, "relu"), _conv(3, 8, 8, "relu"), _conv(1, 8, 1, "sigmoid")]
NET_FM = [_conv(4, 1, 64, "maxout"), POOL2, _conv(4, 32, 64, "maxout"), POOL2,
          _conv(4, 32, 64, "maxout"), POOL2, _conv(4, 32, 2, "softmax")]

# FastMemb_ss (Section 2.2, "A subsampling CNN for 3 nm data"), under the
# reading stated in the design notes: FastMemb_3nm is FastMemb with one more
# {stride-2 pool, conv(4, 32 -> 64, max-out)} pair, and FastMemb_ss replaces its
# first (highest-resolution) stride-2 pool by a 2x subsample, so that 3 nm input
# gives a 6 nm map. Field of view 108 at 3 nm.
SUB2 = {"kind": "sub2"}
NET_FM3 = [_conv(4, 1, 64, "maxout"), POOL2, _conv(4, 32, 64, "maxout"), POOL2, _conv(4, 32, 64, "maxout"),
           POOL2, _conv(4, 32, 64, "maxout"), POOL2, _conv(4, 32, 2, "softmax")]
NET_FMSS = [_conv(4, 1, 64, "maxout"), SUB2, _conv(4, 32, 64, "maxout"), POOL2, _conv(4, 32, 64, "maxout"),
            POOL2, _conv(4, 32, 64, "maxout"), POOL2, _conv(4, 32, 2, "softmax")]

# MaskExtend (Section 3, "MaskExtend: sparse segmentation via CNN"), under the
# reading stated in the design notes: twelve input maps; four pairs of a 4x4
# conv with max-out to 32, 40, 48, 56 features and a 2x2 stride-2 pool, a fifth
# 4x4 conv with max-out to 64 features, and a 1x1 conv to the three classes
# (object, other neurons, membrane) with a softmax; the map is the object
# class's probability. Field of view 109.
NET_ME = [_conv(4, 12, 64, "maxout"), POOL2, _conv(4, 32, 80, "maxout"), POOL2, _conv(4, 40, 96, "maxout"),
          POOL2, _conv(4, 48, 112, "maxout"), POOL2, _conv(4, 56, 128, "maxout"), _conv(1, 64, 3, "softmax0")]

NETS = {"A": NET_A, "B": NET_B, "S": NET_S, "FM": NET_FM, "FMSS": NET_FMSS, "FM3": NET_FM3, "ME": NET_ME}
WEIGHT_SEEDS = {"A": 100, "B": 200, "S": 300, "FM": 400, "FMSS": 410, "FM3": 420, "ME": 500}
CALIBRATION_SEED = 99
CALIBRATION_SHAPE = (1, 256, 256)

_CALIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "calibration.json")


def conv_layers(net):
    return [L for L in net if L["kind"] == "conv"]


def param_count(net) -> int:
    return sum(L["cout"] * L["cin"] * L["k"] * L["k"] + L["cout"] for L in conv_layers(net))


def he_normal_params(net, seed: int) -> np.ndarray:
    """He-normal weights, zero biases, as one float64 vector."""
    rng = np.random.default_rng(int(seed))
    parts = []
    for L in conv_layers(net):
        fan_in = L["cin"] * L["k"] * L["k"]
        w = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(L["cout"], L["cin"], L["k"], L["k"]))
        parts.append(w.ravel())
        parts.append(np.zeros(L["cout"]))
    return np.concatenate(parts).astype(np.float64)


def bias_slices(net):
    """(start, stop) of each conv layer's bias inside the parameter vector."""
    out, off = [], 0
    for L in conv_layers(net):
        off += L["cout"] * L["cin"] * L["k"] * L["k"]
        out.append((off, off + L["cout"]))
        off += L["cout"]
    return out


def random_bias_params(net, seed: int, bias_seed: int, sigma: float = 0.1) -> np.ndarray:
    """He-normal weights with every bias drawn from N(0, sigma^2) (own generator)."""
    p = he_normal_params(net, seed)
    rng = np.random.default_rng(int(bias_seed))
    for a, b in bias_slices(net):
        p[a:b] = rng.normal(0.0, sigma, size=b - a)
    return p


def load_calibration():
    if not os.path.exists(_CALIB_PATH):
        return {}
    with open(_CALIB_PATH) as f:
        return json.load(f)


def calibrated_params(name: str) -> np.ndarray:
    """Seeded He-normal weights of net ``name`` with the stored head bias applied."""
    net = NETS[name]
    p = he_normal_params(net, WEIGHT_SEEDS[name])
    cal = load_calibration().get(name)
    if cal is not None:
        a, b = bias_slices(net)[-1]
        p[a:b] = cal["head_bias"]
    return p


def fp8_act_scales(name: str = "B"):
    """Per conv layer input scale for the FP8 form (None where the layer is not FP8)."""
    cal = load_calibration().get(name)
    if cal is None or "act_scales" not in cal:
        raise RuntimeError("calibration.json lacks FP8 activation scales for net " + name)
    return list(cal["act_scales"])
