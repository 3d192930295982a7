"""Write synth/calibration.json from the FP64 CPU reference (test infrastructure).

The paper does not state biases or number formats, so two constants of the
networks are fixed here once and stored as plain data:

* head bias of nets A and B: the negated median of the head pre-activation (with
  head bias 0) over the dense output of a calibration slice (generator seed 99,
  256 x 256); with it the 0.5 threshold splits the calibration map in half;
* FP8 input scales of net B's FP8 layers: max of that layer's input activation
  over the calibration slice, divided by 448 (the largest e4m3fn value).

Run ``python -m oracle.calibrate`` after changing the nets or the generator; a
CPU test checks that the stored file matches a fresh run.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from synth import em_slice  # noqa: E402
from synth.nets import (CALIBRATION_SEED, CALIBRATION_SHAPE, NETS, WEIGHT_SEEDS,  # noqa: E402
                        he_normal_params)

OUT = os.path.join(os.path.dirname(HERE), "synth", "calibration.json")


def calibration_slice():
    _, H, W = CALIBRATION_SHAPE
    return em_slice(CALIBRATION_SEED, 0, H, W)


def compute():
    img = calibration_slice()
    res = {}
    for name in ("A", "B"):
        net = NETS[name]
        p = he_normal_params(net, WEIGHT_SEEDS[name])
        logit = oracle.forward(img[None], net, p, logits=True)
        entry = {"weight_seed": WEIGHT_SEEDS[name], "head_bias": -float(np.median(logit))}
        if name == "B":
            tr = oracle.trace(img, net, p)
            scales, prev = [], None
            first = True
            for li, L in enumerate(net):
                if L["kind"] != "conv":
                    prev = li
                    continue
                is_head = li == len(net) - 1
                if first or is_head:
                    scales.append(None)
                else:
                    src = tr[li - 1]
                    scales.append(float(src.max()) / 448.0)
                first = False
                prev = li
            entry["act_scales"] = scales
        res[name] = entry
    return res


def main():
    res = compute()
    with open(OUT, "w") as f:
        json.dump(res, f, indent=2, sort_keys=True)
        f.write("\n")
    print(json.dumps(res, indent=2))


if __name__ == "__main__":
    main()
