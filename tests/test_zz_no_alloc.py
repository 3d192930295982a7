"""cnn_infer_noalloc (static device scratch, no allocation) against cnn_infer:
bitwise equal outputs on two calls in a row, the second with a smaller input,
for the slab path (whole slices fit the scratch) and the strip path (a slice
is split into row strips), plus the clear error for rows too wide."""
import numpy as np
import pytest

from synth import em_volume
from synth.nets import NET_B, NET_FM, calibrated_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def emcnn():
    import paper_1612_02120_amd as m
    assert torch.cuda.is_available()
    return m


def _both(emcnn, h, vol):
    v = torch.from_numpy(vol).cuda()
    ref = emcnn.cnn_infer(h, v)
    out = torch.full_like(ref, float("nan"))
    emcnn.cnn_infer_noalloc(h, v, out)
    torch.cuda.synchronize()
    return ref, out


@pytest.mark.parametrize("name,net,prec,big", [
    ("B", NET_B, "fp32", (2, 1100, 1060)),   # 2 x 1100 x 1060: strips of rows
    ("B", NET_B, "bf16", (1, 1500, 2100)),
    ("FM", NET_FM, "fp32", (1, 1100, 1090)),  # stride-2 pools: strips keep the phase parity
])
def test_noalloc_matches_cnn_infer(emcnn, name, net, prec, big):
    print("noalloc case", name, prec, big, flush=True)
    h = emcnn.cnn_create(calibrated_params(name), net, prec)
    for shape in (big, (3, 300, 260)):  # second call: smaller input (slab path)
        ref, out = _both(emcnn, h, em_volume(41, *shape))
        assert torch.equal(ref, out), (shape, (ref - out).abs().max().item())
    h.close()


def test_noalloc_rejects_rows_too_wide(emcnn):
    h = emcnn.cnn_create(calibrated_params("B"), NET_B, "fp32")
    v = torch.zeros((1, 30, 17000), dtype=torch.uint8, device="cuda")
    out = torch.full((1, 18, 17000 - 12), -1.0, device="cuda")
    with pytest.raises(emcnn.CnnError) as e:
        emcnn.cnn_infer_noalloc(h, v, out)
    assert e.value.code == emcnn.CNN_EINVAL and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert (out == -1.0).all()  # nothing was enqueued
    h.close()
