"""GPU parity at the full workload sizes, in the launch configuration bench.py
times, checked on windows the FP64 reference computes one by one.

* plain:     net B FP32 over 32 x 1024 x 1024 (seed 2), three 64 x 64 output
             windows (first slice corner, last slice far corner, a seeded one),
             max abs error <= 1e-5; the whole map is finite and in [0, 1].
* precision: net B BF16 / FP8 over 128 x 2048 x 2048 (seed 3); error windows are
             slices 0-3, output [0,256)^2, plus three seeded 256^2 windows; max
             abs error <= 2e-2 (BF16), 6e-2 (FP8).
* batch:     512 tiles (side logU[64,1024], 1-8 slices, halo 8) in one graph
             submission, bitwise equal to per-tile launches, and three seeded
             64 x 64 windows within tiles against the reference.
"""
import numpy as np
import pytest

import oracle
from synth import batch_tiles, em_volume
from synth.nets import NET_B, calibrated_params, fp8_act_scales

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = 12


@pytest.fixture(scope="module")
def emcnn():
    import paper_1612_02120_amd as m
    assert torch.cuda.is_available()
    return m


def _window_ref(vol, z, y, x, h, w, prec, p):
    # output window [y, y+h) x [x, x+w) of slice z needs input [y, y+h+R) x [x, x+w+R)
    sub = np.ascontiguousarray(vol[z:z + 1, y:y + h + R, x:x + w + R])
    return oracle.forward(sub, NET_B, p)[0]


@pytest.mark.timeout(300)
def test_plain_fp32_full_volume(emcnn):
    vol = em_volume(2, 32, 1024, 1024)
    p = calibrated_params("B")
    h = emcnn.cnn_create(p, NET_B, "fp32")
    out = emcnn.cnn_infer(h, torch.from_numpy(vol).cuda())
    torch.cuda.synchronize()
    assert torch.isfinite(out).all() and out.min() >= 0 and out.max() <= 1
    rng = np.random.default_rng(12)
    wins = [(0, 0, 0), (31, 1012 - 64, 1012 - 64),
            (int(rng.integers(0, 32)), int(rng.integers(0, 1012 - 64)), int(rng.integers(0, 1012 - 64)))]
    for z, y, x in wins:
        got = out[z, y:y + 64, x:x + 64].cpu().numpy().astype(np.float64)
        ref = _window_ref(vol, z, y, x, 64, 64, "fp32", p)
        assert np.abs(got - ref).max() <= 1e-5, (z, y, x)


@pytest.fixture(scope="module")
def precision_volume():
    return em_volume(3, 128, 2048, 2048)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("prec,tol", [("bf16", 2e-2), ("fp8", 6e-2)])
def test_precision_full_volume(emcnn, precision_volume, prec, tol):
    vol = precision_volume
    p = calibrated_params("B")
    h = emcnn.cnn_create(p, NET_B, prec, act_scales=fp8_act_scales("B") if prec == "fp8" else None)
    out = emcnn.cnn_infer(h, torch.from_numpy(vol).cuda())
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()
    rng = np.random.default_rng(33)
    wins = [(z, 0, 0) for z in range(4)] + [
        (int(rng.integers(0, 128)), int(rng.integers(0, 2036 - 256)), int(rng.integers(0, 2036 - 256)))
        for _ in range(3)]
    errs = []
    for z, y, x in wins:
        got = out[z, y:y + 256, x:x + 256].cpu().numpy().astype(np.float64)
        ref = _window_ref(vol, z, y, x, 256, 256, prec, p)
        errs.append(np.abs(got - ref))
    e = np.concatenate([a.ravel() for a in errs])
    print("%s full volume: max abs %.4g, mean abs %.4g over %d voxels" % (prec, e.max(), e.mean(), e.size))
    assert e.max() <= tol


@pytest.mark.timeout(300)
def test_batch_512_tiles(emcnn):
    p = calibrated_params("B")
    h = emcnn.cnn_create(p, NET_B, "bf16")
    tl = batch_tiles()
    pool = em_volume(4, 8, 1040, 1040)
    rng = np.random.default_rng(44)
    tiles, src = [], []
    for t in tl:
        y = int(rng.integers(0, 1040 - t["h"] + 1))
        x = int(rng.integers(0, 1040 - t["w"] + 1))
        arr = np.ascontiguousarray(pool[:t["z"], y:y + t["h"], x:x + t["w"]])
        L = t["h"] - 2 * t["halo"]
        tiles.append((torch.from_numpy(arr).cuda(), t["halo"],
                      torch.empty((t["z"], L, L), dtype=torch.float32, device="cuda")))
        src.append(arr)
    for _ in range(2):  # capture, then replay
        emcnn.cnn_infer_batch(h, tiles)
    torch.cuda.synchronize()
    emcnn.cnn_set_batch_graph(h, False)
    for inp, halo, out in tiles:
        single = torch.empty_like(out)
        emcnn.cnn_infer_batch(h, [(inp, halo, single)])
        assert torch.equal(single, out)
    torch.cuda.synchronize()
    for k in (0, 255, 511):
        arr, (_, halo, out) = src[k], tiles[k]
        L = out.shape[1]
        w = min(64, L)
        e = halo - R // 2
        ref = _window_ref(arr[:, e:arr.shape[1] - e, e:arr.shape[2] - e], 0, 0, 0, w, w, "bf16", p)
        got = out[0, :w, :w].cpu().numpy().astype(np.float64)
        assert np.abs(got - ref).max() <= 2e-2
