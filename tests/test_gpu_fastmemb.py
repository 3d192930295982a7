"""GPU parity of FastMemb (Section 2.2) through the C ABI against the FP64 reference.

FastMemb's stride-2 pools are evaluated densely: each becomes a 2x2 max filter
at the current spacing and doubles the spacing of the later convs, whose d^2
phase sub-lattices the kernels tile separately. Tolerance (max abs on the
class-1 probability against the exact reference): FP32 1e-5; BF16 (bf16
weights and stored activations, FP32 accumulation) 2e-2. Shapes span several
tiles per phase at the largest spacing (8) and ragged tails in every direction.
"""
import numpy as np
import pytest

import oracle
from synth import em_volume
from synth.nets import NET_FM, calibrated_params, random_bias_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def emcnn():
    import paper_1612_02120_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(emcnn, h, vol):
    out = emcnn.cnn_infer(h, _dev(vol))
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def _params():
    # He-normal weights with non-zero biases, so that every bias term is exercised
    return random_bias_params(NET_FM, 400, 41, sigma=0.2)


# (54, 53), (57, 61), (64, 72): every fragment row / column count of the stored
# maps (ceil(h / D) per fragment) ragged against the phase tiles
@pytest.mark.parametrize("shape", [(2, 131, 157), (1, 53, 53), (1, 60, 301), (1, 620, 590), (1, 54, 53), (1, 57, 61),
                                   (3, 64, 72)])
def test_fastmemb_matches_reference(emcnn, shape):
    vol = em_volume(40 + shape[1], *shape)
    p = _params()
    h = emcnn.cnn_create(p, NET_FM, "fp32")
    assert h.R == 52
    got = _run(emcnn, h, vol)
    ref = oracle.forward(vol, NET_FM, p)
    assert got.shape == ref.shape == (shape[0], shape[1] - 52, shape[2] - 52)
    err = np.abs(got - ref).max()
    print("FastMemb fp32", shape, "max err", err)
    assert err <= TOL


def test_every_fastmemb_candidate_matches_reference(emcnn):
    vol = em_volume(77, 2, 161, 203)
    p = _params()
    h = emcnn.cnn_create(p, NET_FM, "fp32")
    ref = oracle.forward(vol, NET_FM, p)
    n_layers = 4
    defaults = [emcnn.cnn_variant_names(h, l)[0] for l in range(n_layers)]
    assert "conv_phase" in defaults[1] and defaults[3].startswith("head_strip<")
    heads = emcnn.cnn_variant_names(h, 3)
    # the VALU form and the padded MFMA form of the softmax layer
    assert any("head_phase" in n for n in heads) and any("conv_phase" in n for n in heads)
    for layer in range(n_layers):
        for name in emcnn.cnn_variant_names(h, layer):
            emcnn.cnn_set_variant(h, layer, name)
            err = np.abs(_run(emcnn, h, vol) - ref).max()
            assert err <= TOL, (layer, name, err)
        emcnn.cnn_set_variant(h, layer, defaults[layer])


@pytest.mark.parametrize("prec,tol", [("fp32", TOL), ("bf16", 2e-2)])
@pytest.mark.parametrize("graph", [0, 1])
def test_fastmemb_batch_matches_per_tile_and_reference(emcnn, graph, prec, tol):
    p = _params()
    h = emcnn.cnn_create(p, NET_FM, prec)
    emcnn.cnn_set_batch_graph(h, graph)
    rng = np.random.default_rng(9)
    tiles, vols = [], []
    for t in range(5):
        L = int(rng.integers(3, 90))
        z = int(rng.integers(1, 3))
        halo = int(rng.choice([26, 29]))  # R / 2 = 26; larger halos are cropped to it
        v = em_volume(600 + t, z, L + 2 * halo, L + 11 + 2 * halo)
        vols.append((v, halo))
        tiles.append((_dev(v), halo, torch.empty((z, L, L + 11), dtype=torch.float32, device="cuda")))
    for rep in range(3):  # replays of the captured graph
        for _, _, o in tiles:
            o.fill_(-1.0)
        emcnn.cnn_infer_batch(h, tiles)
        torch.cuda.synchronize()
        for (v, halo), (_, _, o) in zip(vols, tiles):
            e = halo - 26
            single = _run(emcnn, h, v[:, e:v.shape[1] - e, e:v.shape[2] - e])
            assert np.array_equal(o.cpu().numpy().astype(np.float64), single)
    v, halo = vols[1]
    e = halo - 26
    ref = oracle.forward(v[:, e:v.shape[1] - e, e:v.shape[2] - e], NET_FM, p)
    assert np.abs(tiles[1][2].cpu().numpy() - ref).max() <= tol


def test_fastmemb_full_size_sampled_windows(emcnn):
    # the benchmark's workload (32 x 1024 x 1024) in its launch configuration;
    # sampled outputs against the reference's patch form (one 53 x 53 window each)
    vol = em_volume(2, 32, 1024, 1024)
    p = calibrated_params("FM")
    h = emcnn.cnn_create(p, NET_FM, "fp32")
    got = emcnn.cnn_infer(h, _dev(vol))
    torch.cuda.synchronize()
    assert tuple(got.shape) == (32, 972, 972)
    assert torch.isfinite(got).all()
    rng = np.random.default_rng(3)
    pts = [(int(rng.integers(0, 32)), int(rng.integers(0, 972)), int(rng.integers(0, 972))) for _ in range(40)]
    pts += [(0, 0, 0), (31, 971, 971), (5, 0, 971), (9, 971, 0)]
    g = got.cpu().numpy()
    for z, y, x in pts:
        want = oracle.patch(vol[z], NET_FM, p, y, x)[0]
        assert abs(g[z, y, x] - want) <= TOL, (z, y, x, g[z, y, x], want)


@pytest.mark.parametrize("shape", [(2, 131, 157), (1, 53, 53), (1, 620, 590)])
def test_fastmemb_bf16_matches_reference(emcnn, shape):
    vol = em_volume(50 + shape[1], *shape)
    p = _params()
    h = emcnn.cnn_create(p, NET_FM, "bf16")
    got = _run(emcnn, h, vol)
    ref = oracle.forward(vol, NET_FM, p)
    err = np.abs(got - ref)
    print("FastMemb bf16", shape, "max err", err.max(), "mean", err.mean())
    assert err.max() <= 2e-2


def test_every_fastmemb_bf16_candidate_matches_reference(emcnn):
    vol = em_volume(78, 1, 161, 203)
    p = _params()
    h = emcnn.cnn_create(p, NET_FM, "bf16")
    ref = oracle.forward(vol, NET_FM, p)
    defaults = [emcnn.cnn_variant_names(h, l)[0] for l in range(4)]
    for layer in range(4):
        for name in emcnn.cnn_variant_names(h, layer):
            emcnn.cnn_set_variant(h, layer, name)
            err = np.abs(_run(emcnn, h, vol) - ref).max()
            assert err <= 2e-2, (layer, name, err)
        emcnn.cnn_set_variant(h, layer, defaults[layer])


@pytest.mark.parametrize("shape", [(2, 131, 157), (1, 53, 53), (1, 620, 590)])
def test_fastmemb_bf16_warp_specialised_equals_plain_staging(emcnn, shape):
    # the warp-specialised spaced conv (producer waves stage the next 16-channel
    # block while consumer waves run the MFMAs), per phase or per group of four
    # phases, and conv_phase staging the same 16-channel blocks issue the same
    # MFMAs in the same order: bitwise equal
    vol = em_volume(90 + shape[1], *shape)
    p = _params()
    h = emcnn.cnn_create(p, NET_FM, "bf16")
    plain16 = "conv_phase<BF16,32,64,4,8,64,4,1,16>"
    for layer in (1, 2):
        names = emcnn.cnn_variant_names(h, layer)
        assert plain16 in names and sum(n.startswith("conv_ws_phase<") for n in names) >= 2, names
        assert names[0].startswith("conv_ws_group<"), names
        emcnn.cnn_set_variant(h, layer, plain16)
    base = _run(emcnn, h, vol)
    for layer in (1, 2):
        for name in emcnn.cnn_variant_names(h, layer):
            if name.startswith(("conv_ws_phase<", "conv_ws_group<")):
                emcnn.cnn_set_variant(h, layer, name)
                assert np.array_equal(_run(emcnn, h, vol), base), (layer, name)
        emcnn.cnn_set_variant(h, layer, plain16)


def test_fastmemb_bf16_full_size_sampled_windows(emcnn):
    vol = em_volume(2, 32, 1024, 1024)
    p = calibrated_params("FM")
    h = emcnn.cnn_create(p, NET_FM, "bf16")
    got = emcnn.cnn_infer(h, _dev(vol))
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    rng = np.random.default_rng(4)
    pts = [(int(rng.integers(0, 32)), int(rng.integers(0, 972)), int(rng.integers(0, 972))) for _ in range(40)]
    pts += [(0, 0, 0), (31, 971, 971)]
    errs = [abs(g[z, y, x] - oracle.patch(vol[z], NET_FM, p, y, x)[0]) for z, y, x in pts]
    print("FastMemb bf16 full size sampled max err", max(errs))
    assert max(errs) <= 2e-2


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fastmemb_small_workspace_equals_unlimited(emcnn, prec):
    # a 1 MiB workspace budget: one slice per slab, and batch tiles split into
    # groups; the fragment-major maps between layers are laid out per group
    vol = _dev(em_volume(95, 3, 140, 171))
    p = _params()
    big = emcnn.cnn_create(p, NET_FM, prec)
    small = emcnn.cnn_create(p, NET_FM, prec)
    emcnn.cnn_set_workspace_limit(small, 1 << 20)
    a = emcnn.cnn_infer(big, vol)
    b = emcnn.cnn_infer(small, vol)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    tiles_a, tiles_b = [], []
    for t in range(5):
        v = _dev(em_volume(700 + t, 1 + t % 3, 60 + 9 * t, 73 + 4 * t))
        oa = torch.empty((v.shape[0], v.shape[1] - 52, v.shape[2] - 52), device="cuda")
        tiles_a.append((v, 26, oa))
        tiles_b.append((v, 26, torch.empty_like(oa)))
    emcnn.cnn_infer_batch(big, tiles_a)
    emcnn.cnn_infer_batch(small, tiles_b)
    torch.cuda.synchronize()
    for (_, _, x), (_, _, y) in zip(tiles_a, tiles_b):
        assert torch.equal(x, y)
