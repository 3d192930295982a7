"""The learned part: a student distilled on the GPU from the plain FP32 net's maps,
and what it gains over the plain net alone.

The teacher is net B with seeded He-normal weights; its maps are indecisive
(about a third of all voxels lie within 0.01 of the 0.5 threshold), so the
thresholded agreement of any approximation is limited: even the BF16 form of
the teacher agrees with the FP32 form on only about 99 %. The student (FoV 7
against the teacher's 13) reaches about 80 % raw agreement. What it gains:

* raw agreement far above the untrained student (chance level, 50 %);
* ~10x the plain FP32 net's throughput where it is trusted;
* per-tile fallback that fires on the tiles where it is worse: on a volume
  whose tiles come from two generators (default, and a harder one with noise
  sigma 24 and cell spacing 16), with tau set between the two per-tile flip
  rates measured on a separate calibration volume, the hard tiles fall back
  and most default tiles keep the student's output, and the output agrees with
  the teacher more than the raw student does.

Training-outcome numbers are stochastic: parity unpinned; the test pins the
mechanism (seeded, reproducible).
"""
import numpy as np
import pytest

from synth import em_volume, mixed_difficulty_volume
from synth.nets import NET_B, NET_S, calibrated_params, he_normal_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def emcnn():
    import paper_1612_02120_amd as m
    assert torch.cuda.is_available()
    return m


def _tile_flip_rates(st_map, te_map, tile=512):
    f = ((st_map >= 0.5) != (te_map >= 0.5)).float()
    Z, H, W = te_map.shape
    return np.array([f[z, a:a + tile, b:b + tile].mean().item()
                     for z in range(Z) for a in range(0, H, tile) for b in range(0, W, tile)])


@pytest.mark.timeout(600)
def test_distilled_student_gain(emcnn):
    from paper_1612_02120_amd import distill
    teacher = emcnn.cnn_create(calibrated_params("B"), NET_B, "fp32")
    vols = [torch.from_numpy(em_volume(5000 + i, 16, 512, 512)).cuda() for i in range(16)]
    maps = distill.teacher_maps(teacher, vols)
    p0 = he_normal_params(NET_S, 300)
    student = emcnn.student_create(p0, "bf16")
    untrained = emcnn.student_create(p0, "bf16")
    losses, _ = distill.train(student, vols, maps, teacher.R, steps=4000, seed=11)
    torch.cuda.synchronize()
    assert torch.isfinite(losses).all()
    assert losses[-500:].mean().item() < losses[:50].mean().item()

    ev = torch.from_numpy(em_volume(7777, 4, 1024, 1024)).cuda()
    evm = emcnn.cnn_infer(teacher, ev)
    r_t, _, _ = distill.evaluate(student, teacher, ev, evm, tau=1.0)
    r_u, _, _ = distill.evaluate(untrained, teacher, ev, evm, tau=1.0)
    print("raw agreement trained %.4f untrained %.4f" % (r_t["raw_agreement"], r_u["raw_agreement"]))
    assert r_t["raw_agreement"] >= r_u["raw_agreement"] + 0.2
    assert r_t["fallback_rate"] == 0.0 and r_t["agreement"] == r_t["raw_agreement"]

    # tau between the per-tile flip rates of default and hard tiles, from a calibration volume
    cv, chard = mixed_difficulty_volume(8801, 8, 1024, 1024, tile=512, hard_frac=0.3)
    cvd = torch.from_numpy(cv).cuda()
    cm = emcnn.cnn_infer(teacher, cvd)
    fl = _tile_flip_rates(emcnn.student_infer(student, cvd)[:, 3:3 + 1012, 3:3 + 1012], cm)
    h = chard.reshape(-1)
    assert h.any() and (~h).any()
    tau = float((fl[~h].max() + fl[h].min()) / 2)
    print("calibration flip rates: default max %.4f, hard min %.4f -> tau %.4f" % (fl[~h].max(), fl[h].min(), tau))
    assert fl[h].min() > fl[~h].max()

    tv, thard = mixed_difficulty_volume(8802, 8, 1024, 1024, tile=512, hard_frac=0.3)
    tvd = torch.from_numpy(tv).cuda()
    tm = emcnn.cnn_infer(teacher, tvd)
    r, out, st = distill.evaluate(student, teacher, tvd, tm, tau=tau, tile=512, n_samples=16, seed=5)
    th = thard.reshape(-1)
    # which tiles fell back: there the output equals the teacher's map exactly
    fell = np.array([torch.equal(out[z, a:a + 512, b:b + 512], tm[z, a:a + 512, b:b + 512])
                     for z in range(8) for a in range(0, 1012, 512) for b in range(0, 1012, 512)])
    print("mixed volume: %s; hard tiles %d, fell back: hard %d default %d" % (
        r, th.sum(), (fell & th).sum(), (fell & ~th).sum()))
    assert fell.sum() == r["fallback_tiles"]
    assert (fell & th).sum() >= 0.75 * th.sum()
    assert (fell & ~th).sum() <= 0.5 * (~th).sum()
    assert r["agreement"] > r["raw_agreement"] + 0.01
