"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU reference.

Tolerances (max abs probability error): FP32 1e-5; BF16 2e-2 and FP8 6e-2
against the exact reference. Against the reference's fake-quant form of the same
number formats (exact accumulation of the rounded operands): BF16 2e-3 (rare
one-ulp flips of an intermediate rounding); FP8 1e-2, because the gfx950
16x16x128 f8f6f4 MFMA sums its 128 products with less precision than FP32
(tests/bounds.py, measured by tests/test_gpu_mfma.py), which moves a few
hundredths of a percent of the next layer's e4m3 codes across rounding
boundaries; each such code then moves the probability by up to a few 1e-3.
The element-wise, layer-by-layer pin of the FP8 and BF16 kernels is
tests/test_gpu_layers.py.
"""
import numpy as np
import pytest

import oracle
from synth import em_volume
from synth.nets import NET_A, NET_B, calibrated_params, fp8_act_scales, random_bias_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _scales():
    return fp8_act_scales("B")


def test_tiny_net_a_fp32_full_slice(emcnn):
    vol = em_volume(1, 1, 256, 256)
    p = calibrated_params("A")
    h = emcnn.cnn_create(p, NET_A, "fp32")
    got = _run(emcnn, h, vol)
    ref = oracle.forward(vol, NET_A, p)
    assert got.shape == (1, 248, 248)
    err = np.abs(got - ref).max()
    print("net A fp32 256^2 max err", err)
    assert err <= 1e-5


@pytest.mark.parametrize("shape", [(2, 75, 83), (1, 13, 13), (1, 40, 200), (3, 33, 47)])
def test_net_b_fp32_random_bias(emcnn, shape):
    vol = em_volume(20 + shape[1], *shape)
    p = random_bias_params(NET_B, 200, 21)
    h = emcnn.cnn_create(p, NET_B, "fp32")
    got = _run(emcnn, h, vol)
    ref = oracle.forward(vol, NET_B, p)
    err = np.abs(got - ref).max()
    print("net B fp32", shape, "max err", err)
    assert err <= 1e-5


@pytest.mark.parametrize("prec,tol_fq,tol_exact", [("bf16", 2e-3, 2e-2), ("fp8", 1e-2, 6e-2)])
def test_net_b_low_precision(emcnn, prec, tol_fq, tol_exact):
    vol = em_volume(31, 2, 70, 90)
    p = calibrated_params("B")
    sc = _scales() if prec == "fp8" else None
    h = emcnn.cnn_create(p, NET_B, prec, act_scales=sc)
    got = _run(emcnn, h, vol)
    fq = oracle.forward(vol, NET_B, p, qmode=prec, act_scales=sc)
    ex = oracle.forward(vol, NET_B, p)
    e_fq, e_ex = np.abs(got - fq).max(), np.abs(got - ex).max()
    print(prec, "max err vs fake-quant", e_fq, "vs exact", e_ex, "mean vs exact", np.abs(got - ex).mean())
    assert e_fq <= tol_fq
    assert e_ex <= tol_exact


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_translation_equivariance_bitwise(emcnn, prec):
    vol = em_volume(41, 1, 90, 100)
    p = calibrated_params("B")
    h = emcnn.cnn_create(p, NET_B, prec, act_scales=_scales() if prec == "fp8" else None)
    full = _run(emcnn, h, vol)
    for dy, dx in [(1, 0), (0, 5), (9, 17)]:
        sh = _run(emcnn, h, vol[:, dy:, dx:])
        assert np.array_equal(sh, full[:, dy:, dx:]), (prec, dy, dx)


def test_run_twice_deterministic(emcnn):
    vol = em_volume(42, 2, 120, 130)
    h = emcnn.cnn_create(calibrated_params("B"), NET_B, "bf16")
    a, b = _run(emcnn, h, vol), _run(emcnn, h, vol)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("graph", [True, False])
def test_batch_matches_per_tile_and_oracle(emcnn, graph):
    p = calibrated_params("B")
    h = emcnn.cnn_create(p, NET_B, "fp32")
    emcnn.cnn_set_batch_graph(h, graph)
    rng = np.random.default_rng(5)
    tiles, vols = [], []
    for t in range(7):
        L = int(rng.integers(5, 70))
        z = int(rng.integers(1, 4))
        halo = int(rng.choice([6, 8]))
        v = em_volume(500 + t, z, L + 2 * halo, L + 7 + 2 * halo)
        vols.append((v, halo))
        tiles.append((_dev(v), halo, torch.empty((z, L, L + 7), dtype=torch.float32, device="cuda")))
    for rep in range(3):  # replays of the captured graph
        for _, _, o in tiles:
            o.fill_(-1.0)
        emcnn.cnn_infer_batch(h, tiles)
        torch.cuda.synchronize()
        for (v, halo), (_, _, o) in zip(vols, tiles):
            e = halo - 6
            single = _run(emcnn, h, v[:, e:v.shape[1] - e, e:v.shape[2] - e])
            assert np.array_equal(o.cpu().numpy().astype(np.float64), single)
    v, halo = vols[0]
    e = halo - 6
    ref = oracle.forward(v[:, e:v.shape[1] - e, e:v.shape[2] - e], NET_B, p)
    assert np.abs(tiles[0][2].cpu().numpy() - ref).max() <= 1e-5


def test_invalid_arguments_leave_stream_untouched(emcnn):
    """Arguments are validated before anything is enqueued: with per-layer
    profiling on (every layer launch brackets itself with events), rejected
    calls record no launch, leave their sentinel outputs untouched, and the
    stream they were given is idle right after them."""
    import ctypes
    h = emcnn.cnn_create(calibrated_params("B"), NET_B, "fp32")
    emcnn.cnn_set_batch_graph(h, False)  # direct launches, which the profiler records
    emcnn.cnn_profile_read(h)
    emcnn.cnn_profile(h, True)
    st = torch.cuda.Stream()
    sp = st.cuda_stream
    small = _dev(np.zeros((1, 12, 40), np.uint8))  # H < field of view 13
    out = torch.full((1, 4, 28), 7.0, device="cuda")
    dims = (ctypes.c_int64 * 3)(1, 12, 40)
    lib = emcnn._lib
    codes = [
        lib.cnn_infer(h.ptr, emcnn._ptr(small), dims, emcnn._ptr(out), sp),
        lib.cnn_infer_noalloc(h.ptr, emcnn._ptr(small), dims, emcnn._ptr(out), sp),
    ]
    t = _dev(np.zeros((1, 30, 30), np.uint8))
    tout = torch.full((1, 20, 20), 7.0, device="cuda")
    with pytest.raises(emcnn.CnnError) as ei:
        emcnn.cnn_infer_batch(h, [(t, 5, tout)], stream=st)  # halo < R/2
    codes.append(ei.value.code)
    s = emcnn.student_create(np.zeros(801), "bf16")
    big = _dev(np.zeros((1, 60, 60), np.uint8))
    fout = torch.full((1, 48, 48), 7.0, device="cuda")
    stats = torch.full((2,), -5, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(emcnn.CnnError) as ei:  # tile < 16
        emcnn.student_infer_with_fallback(s, h, big, tau=0.1, tile=8, out=fout, stats=stats, stream=st)
    codes.append(ei.value.code)
    assert st.query()  # nothing pending on the caller's stream
    assert codes == [emcnn.CNN_EINVAL] * 4
    ms, n = emcnn.cnn_profile_read(h)
    assert sum(n) == 0, n
    torch.cuda.synchronize()
    assert (out == 7.0).all() and (tout == 7.0).all() and (fout == 7.0).all()
    assert stats.tolist() == [-5, -5]


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2), ("fp8", 6e-2)])
def test_every_candidate_variant_matches_reference(emcnn, prec, tol):
    # every compiled tile shape / K order the autotuner may pick, on a ragged volume
    vol = em_volume(77, 2, 61, 150)
    p = calibrated_params("B")
    sc = _scales() if prec == "fp8" else None
    h = emcnn.cnn_create(p, NET_B, prec, act_scales=sc)
    ref = oracle.forward(vol, NET_B, p)
    defaults = [emcnn.cnn_variant_names(h, l)[0] for l in range(3)]
    for layer in range(3):
        for name in emcnn.cnn_variant_names(h, layer):
            emcnn.cnn_set_variant(h, layer, name)
            got = _run(emcnn, h, vol)
            err = np.abs(got - ref).max()
            assert err <= tol, (layer, name, err)
        emcnn.cnn_set_variant(h, layer, defaults[layer])


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_fused_first_layer_bitwise_equals_unfused(emcnn, prec):
    """BF16 / FP8 net B's conv2 has candidates that compute the first layer in
    their producer waves (no layer-0 launch, no layer-0 output in HBM). Rounding
    and quantisation are monotone, so filtering before or after them is the
    same: every fused candidate equals the separate conv_first + conv2 path
    bitwise, on a ragged multi-slice volume, in direct and batched submission."""
    vol = em_volume(21, 3, 203, 331)
    h = emcnn.cnn_create(calibrated_params("B"), NET_B, prec,
                         act_scales=fp8_act_scales("B") if prec == "fp8" else None)
    names = emcnn.cnn_variant_names(h, 1)
    fused_names = [n for n in names if n.endswith(",5>")]
    assert fused_names and not names[0].endswith(",5>"), names
    ref = emcnn.cnn_infer(h, _dev(vol))
    torch.cuda.synchronize()
    assert "computed inside layer 1" not in emcnn.cnn_describe(h)
    tin = _dev(vol[:, 20:180, 40:300])
    tout_ref = torch.empty((3, 160 - 12, 260 - 12), dtype=torch.float32, device="cuda")
    emcnn.cnn_infer_batch(h, [(tin, 6, tout_ref)])
    for name in fused_names:
        emcnn.cnn_set_variant(h, 1, name)
        emcnn.cnn_profile(h, True)
        fused = emcnn.cnn_infer(h, _dev(vol))
        torch.cuda.synchronize()
        emcnn.cnn_profile(h, False)
        _, launches = emcnn.cnn_profile_read(h)
        assert launches[0] == 0 and launches[1] == 1 and launches[2] == 1
        assert "computed inside layer 1" in emcnn.cnn_describe(h)
        assert torch.equal(fused, ref), name
        tout = torch.empty_like(tout_ref)
        emcnn.cnn_infer_batch(h, [(tin, 6, tout)])
        torch.cuda.synchronize()
        assert torch.equal(tout, tout_ref), name
