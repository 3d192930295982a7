"""Batched form with per tile class tile shapes (cnn_autotune_batch, tuned on
the same tiles): tiles of every size class give bitwise the same
probabilities as with the handle's default shapes, graph-captured and with
direct launches, and an explicit cnn_set_variant drops the per-class choice. The default batch path itself is
checked against the reference in test_gpu_fullsize.py and test_gpu_parity.py."""
import numpy as np
import pytest

from synth import em_volume
from synth.nets import NET_B, calibrated_params, fp8_act_scales

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = 12


@pytest.fixture(scope="module")
def emcnn():
    import paper_1612_02120_amd as m
    assert torch.cuda.is_available()
    return m


def _tiles(seed):
    # output sides spanning the five classes (edges 91, 181, 362, 724), ragged
    # and non-square, 1-3 slices, halos 6 and 8
    pool = em_volume(seed, 3, 1060, 1060)
    rng = np.random.default_rng(seed)
    tiles = []
    for (ho, wo) in [(64, 64), (90, 130), (100, 77), (181, 200), (255, 300), (361, 362), (500, 420),
                     (723, 700), (800, 760), (1000, 1030)]:
        halo = int(rng.choice([6, 8]))
        z = int(rng.integers(1, 4))
        h, w = ho + 2 * halo, wo + 2 * halo
        y, x = int(rng.integers(0, 1060 - h + 1)), int(rng.integers(0, 1060 - w + 1))
        arr = np.ascontiguousarray(pool[:z, y:y + h, x:x + w])
        tiles.append((torch.from_numpy(arr).cuda(), halo,
                      torch.full((z, ho, wo), -1.0, dtype=torch.float32, device="cuda")))
    return tiles


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_class_tile_shapes_are_bitwise_equal(emcnn, prec):
    h = emcnn.cnn_create(calibrated_params("B"), NET_B, prec,
                         act_scales=fp8_act_scales("B") if prec == "fp8" else None)
    tiles = _tiles(61)
    emcnn.cnn_infer_batch(h, tiles)
    torch.cuda.synchronize()
    ref = [out.clone() for _, _, out in tiles]
    for r in ref:
        assert bool(((r >= 0) & (r <= 1)).all())
    emcnn.cnn_autotune_batch(h, tiles)
    assert "batch classes" in emcnn.cnn_describe(h)
    for graph in (True, False):
        emcnn.cnn_set_batch_graph(h, graph)
        for _, _, out in tiles:
            out.fill_(-1.0)
        for _ in range(2):  # capture, then replay
            emcnn.cnn_infer_batch(h, tiles)
        torch.cuda.synchronize()
        for r, (_, _, out) in zip(ref, tiles):
            assert torch.equal(r, out)
    # an explicit choice applies to batches again
    emcnn.cnn_set_variant(h, 0, emcnn.cnn_variant_names(h, 0)[0])
    for _, _, out in tiles:
        out.fill_(-1.0)
    emcnn.cnn_infer_batch(h, tiles)
    torch.cuda.synchronize()
    for r, (_, _, out) in zip(ref, tiles):
        assert torch.equal(r, out)
