"""Pins of the exact CPU reference of the 3-D watershed (Section 2.1: a 3-D
watershed over the membrane probability map gives an over-segmentation).
Reading: watershed by steepest descent with seeded minima, ties broken by
voxel index (emcnn_oracle.c states it in full).

* brute force: the definition written again in pure Python with other
  algorithms (seed components by repeated min-relaxation, descent by plain
  iteration), on tiny volumes with many ties;
* ground truth: on a synthetic 3-D Voronoi map (cell interiors low, 1.5-voxel
  shells high) the seeded basins are the cells;
* invariants: every basin is 6-connected, a voxel carries the label of its
  descent successor, special cases (all seeds, no seeds, constant map).
"""
import numpy as np
import pytest
from scipy import ndimage
from scipy.spatial import cKDTree

import oracle


def _brute(p, t):
    Z, H, W = p.shape
    N = p.size
    flat = p.ravel()

    def nbrs(v):
        z, y, x = v // (H * W), (v // W) % H, v % W
        out = []
        for dz, dy, dx in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
            zz, yy, xx = z + dz, y + dy, x + dx
            if 0 <= zz < Z and 0 <= yy < H and 0 <= xx < W:
                out.append((zz * H + yy) * W + xx)
        return out

    seed = [bool(flat[v] < np.float32(t)) for v in range(N)]
    comp = [v if seed[v] else -1 for v in range(N)]
    changed = True
    while changed:  # each seed takes the least index among its seed neighbours until stable
        changed = False
        for v in range(N):
            if seed[v]:
                m = min([comp[v]] + [comp[u] for u in nbrs(v) if seed[u]])
                if m < comp[v]:
                    comp[v], changed = m, True

    def nxt(v):
        if seed[v]:
            return v
        return min([v] + nbrs(v), key=lambda u: (flat[u], u))

    lab = np.zeros(N, dtype=np.int64)
    for v in range(N):
        r = v
        while nxt(r) != r:
            r = nxt(r)
        lab[v] = comp[r] + 1 if seed[r] else r + 1
    return lab.reshape(p.shape)


@pytest.mark.parametrize("shape,levels,t,seed", [((3, 5, 6), 0, 0.2, 0), ((2, 7, 4), 4, 0.3, 1),
                                                 ((4, 4, 4), 3, 0.0, 2), ((1, 9, 11), 5, 0.45, 3),
                                                 ((5, 3, 2), 2, 0.6, 4)])
def test_brute_force(shape, levels, t, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, shape)
    if levels:
        p = np.floor(p * levels) / levels  # plateaus: many exact ties
    p = p.astype(np.float32)
    got = oracle.watershed(p, t)
    assert np.array_equal(got, _brute(p, t))


def _voronoi_map(shape, ncells, seed, shell=1.5):
    rng = np.random.default_rng(seed)
    Z, H, W = shape
    pts = rng.uniform((0, 0, 0), shape, size=(ncells, 3))
    g = np.stack(np.meshgrid(np.arange(Z) + 0.5, np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij"),
                 axis=-1).reshape(-1, 3)
    d, idx = cKDTree(pts).query(g, k=2)
    cell = idx[:, 0].reshape(shape)
    ridge = ((d[:, 1] - d[:, 0]) < shell).reshape(shape)
    p = np.where(ridge, 0.9, 0.1) + rng.uniform(0, 0.05, size=shape)
    return p.astype(np.float32), cell, ridge


def test_voronoi_cells_are_recovered():
    p, cell, ridge = _voronoi_map((12, 40, 44), 25, 7)
    lab = oracle.watershed(p, 0.5)
    inside = ~ridge
    checked = 0
    for c in np.unique(cell):
        m = inside & (cell == c)
        if not m.any():
            continue
        _, ncomp = ndimage.label(m)
        if ncomp != 1:
            continue  # a thin cell whose interior breaks apart on the grid
        labs = np.unique(lab[m])
        assert labs.size == 1  # one basin per cell interior
        # no other cell's interior has that basin
        assert not (inside & (cell != c) & (lab == labs[0])).any()
        checked += 1
    assert checked >= 15
    # every shell voxel drains into one of its cells' basins or a shell minimum
    assert (lab > 0).all()


def test_basins_connected_and_descent_consistent():
    rng = np.random.default_rng(9)
    p = ndimage.gaussian_filter(rng.uniform(0, 1, (6, 30, 33)), 1.5).astype(np.float32)
    t = float(np.quantile(p, 0.2))
    lab = oracle.watershed(p, t)
    for l in np.unique(lab):
        _, n = ndimage.label(lab == l)
        assert n == 1
    # label(v) == label(next(v)) for non-seed voxels
    Z, H, W = p.shape
    flat, lf = p.ravel(), lab.ravel()
    for v in rng.integers(0, p.size, size=400):
        if flat[v] < np.float32(t):
            continue
        z, y, x = v // (H * W), (v // W) % H, v % W
        cand = [v]
        for dz, dy, dx in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
            zz, yy, xx = z + dz, y + dy, x + dx
            if 0 <= zz < Z and 0 <= yy < H and 0 <= xx < W:
                cand.append((zz * H + yy) * W + xx)
        u = min(cand, key=lambda q: (flat[q], q))
        assert lf[u] == lf[v]


def test_special_cases():
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 1, (3, 8, 9)).astype(np.float32)
    assert (oracle.watershed(p, 2.0) == 1).all()  # every voxel a seed: one component
    const = np.full((2, 5, 6), 0.7, np.float32)
    assert (oracle.watershed(const, 0.5) == 1).all()  # one plateau drains to index 0
    lab = oracle.watershed(p, -1.0)  # no seeds: one basin per local minimum of the order
    mins = [v for v in range(p.size) if lab.ravel()[v] == v + 1]
    assert len(np.unique(lab)) == len(mins)
    one = oracle.watershed(np.zeros((1, 1, 1), np.float32), 0.5)
    assert one.tolist() == [[[1]]]
