"""The matrix instructions of the conv kernels on given operands
(cnn_mfma_probe), against FP64 sums of the same products: FP32 and BF16 within
FP32 accumulation, FP8 (e4m3fn, 16x16x128 f8f6f4) within FP8_ACC_REL of the sum
of absolute products; exact on small integers. Also the measured throughput
ceiling of each instruction (cnn_mfma_bench) at the clock it ran."""
import numpy as np
import pytest

from tests.bounds import BF16_ACC_REL, FP32_ACC_REL, FP8_ACC_REL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def emcnn():
    import paper_1612_02120_amd as m
    assert torch.cuda.is_available()
    return m


def _operands(prec, nt, rng, kind):
    """uint8 operand bytes (nt x 64 x CH) and their float64 element values (nt x 64 x E)."""
    if prec == "fp8":
        if kind == "full":
            codes = rng.integers(0, 254, size=(nt, 64, 32))
            codes = np.where(codes >= 127, codes + 1, codes)  # skip 0x7f (NaN); 0xff is out of range
        elif kind == "positive":  # same sign, wide exponent range: no cancellation
            codes = rng.integers(1, 127, size=(nt, 64, 32))
        else:  # small integers 0..8 (exact)
            codes = np.array([0x00, 0x38, 0x40, 0x44, 0x48, 0x4A, 0x4C, 0x4E, 0x50])[rng.integers(0, 9, size=(nt, 64, 32))]
        b = codes.astype(np.uint8)
        vals = torch.from_numpy(b.copy()).view(torch.float8_e4m3fn).to(torch.float64).numpy()
        return b, vals
    if prec == "bf16":
        x = rng.standard_normal((nt, 64, 8)) * np.exp2(rng.integers(-20, 20, size=(nt, 64, 8)))
        if kind == "small":
            x = rng.integers(-8, 9, size=(nt, 64, 8)).astype(np.float64)
        t = torch.from_numpy(x).to(torch.bfloat16)
        return t.view(torch.uint8).numpy().reshape(nt, 64, 16), t.to(torch.float64).numpy()
    x = rng.standard_normal((nt, 64, 4)) * np.exp2(rng.integers(-20, 20, size=(nt, 64, 4)))
    if kind == "small":
        x = rng.integers(-8, 9, size=(nt, 64, 4)).astype(np.float64)
    t = torch.from_numpy(x).to(torch.float32)
    return t.view(torch.uint8).numpy().reshape(nt, 64, 16), t.to(torch.float64).numpy()


@pytest.mark.parametrize("chain", [1, 10])
@pytest.mark.parametrize("prec,bound", [("fp32", FP32_ACC_REL), ("bf16", BF16_ACC_REL), ("fp8", FP8_ACC_REL)])
def test_mfma_probe_accumulation(emcnn, prec, bound, chain):
    """chain 10: ten instructions accumulating onto each other, as the 10 K steps
    of the FP8 5x5 conv; the bound is on the sum of |products| of the whole chain."""
    rng = np.random.default_rng(17 + chain)
    for kind in ("full", "positive", "small"):
        nt = 1024 // chain * chain
        ab, av = _operands(prec, nt, rng, kind)
        bb, bv = _operands(prec, nt, rng, kind)
        d = emcnn.cnn_mfma_probe(prec, torch.from_numpy(ab).cuda(), torch.from_numpy(bb).cuda(), chain=chain)
        torch.cuda.synchronize()
        E = av.shape[2]
        A = av.reshape(nt // chain, chain, 4, 16, E)
        B = bv.reshape(nt // chain, chain, 4, 16, E)
        exact = np.einsum("tcgme,tcgne->tmn", A, B)
        mag = np.einsum("tcgme,tcgne->tmn", np.abs(A), np.abs(B))
        nt = nt // chain
        got = d.cpu().numpy().astype(np.float64).reshape(nt, 4, 16, 4).transpose(0, 1, 3, 2).reshape(nt, 16, 16)
        err = np.abs(got - exact)
        ratio = (err / np.where(mag > 0, mag, 1.0)).max()
        big = np.einsum("tcgme,tcgne->tcgmne", np.abs(A), np.abs(B)).max(axis=(1, 2, 5)) if E <= 32 else None
        rmax = (err / np.where(big > 0, big, 1.0)).max() if big is not None else float("nan")
        print("%s %s chain %d: max |D - exact| / sum|ab| = %.3g (bound %.3g); / max|ab| = %.3g"
              % (prec, kind, chain, ratio, bound, rmax))
        if kind == "small":
            assert np.array_equal(got, exact)
        else:
            assert ratio <= bound


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_mfma_bench_runs(emcnn, prec):
    rng = np.random.default_rng(3)
    if prec == "fp8":
        ops, _ = _operands("fp8", 512, rng, "full")
    else:
        ops = rng.integers(0, 256, size=(512, 64, 32)).astype(np.uint8)
        if prec == "bf16":  # finite bf16 values: clear the top exponent bit
            ops[..., 1::2] &= 0xBF
        else:
            ops[..., 3::4] &= 0xBF
    tf, mhz = emcnn.cnn_mfma_bench(prec, torch.from_numpy(ops.reshape(-1)).cuda(), blocks=1024, iters=512)
    peak = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}[prec]
    print("%s MFMA loop: %.1f TFLOP/s = %.1f%% of %.1f at %.0f MHz" % (prec, tf, 100 * tf / peak, peak, mhz))
    assert 0.05 * peak < tf < 1.05 * peak
    assert 500 < mhz < 2600
