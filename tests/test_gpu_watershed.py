"""GPU 3-D watershed (watershed_3d, through the C ABI) against the exact CPU
reference, label for label: the labelling is unique (a total order, no
flooding order), so the bar is bitwise equality. Cases: tiny volumes with many
exact ties, ragged sizes, every seed / no seed / one voxel, a synthetic 3-D
Voronoi map, and the membrane map of net B over an EM-like stack at full
headline size (32 x 1012 x 1012)."""
import numpy as np
import pytest
from scipy import ndimage  # noqa: E402

import oracle
from synth import em_volume
from synth.nets import NET_B, calibrated_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def emcnn():
    import paper_1612_02120_amd as m
    assert torch.cuda.is_available()
    return m


def _gpu(emcnn, p, t):
    lab = emcnn.watershed_3d(torch.from_numpy(np.ascontiguousarray(p)).cuda(), t)
    torch.cuda.synchronize()
    return lab.cpu().numpy()


@pytest.mark.parametrize("shape,levels,t,seed", [((3, 5, 6), 0, 0.2, 0), ((2, 7, 4), 4, 0.3, 1),
                                                 ((5, 37, 41), 6, 0.25, 2), ((1, 1, 1), 0, 0.5, 3),
                                                 ((4, 33, 65), 0, 2.0, 4), ((3, 40, 29), 3, -1.0, 5),
                                                 ((2, 64, 64), 1, 0.5, 6)])
def test_watershed_random_with_ties(emcnn, shape, levels, t, seed):
    print("watershed case", shape, levels, t, flush=True)
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, shape)
    if levels:
        p = np.floor(p * levels) / levels
    p = p.astype(np.float32)
    assert np.array_equal(_gpu(emcnn, p, t), oracle.watershed(p, t))


@pytest.mark.parametrize("shape,frac,seed", [((3, 9, 600), 0.85, 7), ((2, 5, 1030), 0.97, 8), ((2, 3, 700), 1.0, 9),
                                              ((4, 6, 257), 0.6, 10)])
def test_watershed_long_seed_runs(emcnn, shape, frac, seed):
    """Seed runs along x that cross the 256-column chunks of a row (the
    first-seed scan carries between chunks), rows that are all seeds, and
    exact ties among the seeds and the rest."""
    print("watershed runs case", shape, frac, flush=True)
    rng = np.random.default_rng(seed)
    p = np.floor(rng.uniform(0, 1, shape) * 5) / 5 + 0.2
    p = np.where(rng.uniform(0, 1, shape) < frac, 0.1, p).astype(np.float32)
    t = 0.15
    assert np.array_equal(_gpu(emcnn, p, t), oracle.watershed(p, t))


@pytest.mark.parametrize("sigma,q", [(1.0, 0.1), (2.5, 0.3)])
def test_watershed_smooth_maps(emcnn, sigma, q):
    rng = np.random.default_rng(11)
    p = ndimage.gaussian_filter(rng.uniform(0, 1, (9, 130, 117)), sigma).astype(np.float32)
    t = float(np.quantile(p, q))
    assert np.array_equal(_gpu(emcnn, p, t), oracle.watershed(p, t))


def test_watershed_on_net_b_map_full_size(emcnn):
    """The over-segmentation stage on the plain net's output over the headline
    volume (32 x 1024^2 in, 32 x 1012^2 map)."""
    h = emcnn.cnn_create(calibrated_params("B"), NET_B, "fp32")
    vol = torch.from_numpy(em_volume(2, 32, 1024, 1024)).cuda()
    pm = emcnn.cnn_infer(h, vol)
    t = float(torch.quantile(pm[0].flatten()[::97].float(), 0.25).item())
    lab = emcnn.watershed_3d(pm, t)
    torch.cuda.synchronize()
    P = pm.cpu().numpy()
    ref = oracle.watershed(P, t)
    got = lab.cpu().numpy()
    print("net B map %s, t %.4f: %d basins" % (P.shape, t, len(np.unique(ref))))
    assert np.array_equal(got, ref)
