"""Pins of the host reference for the fallback decisions (tests/fallback_ref.py).

* splitmix64: the first outputs of the generator seeded with 1234567, as
  published with the generator's reference implementation (Vigna), are
  reproduced by iterating the state and applying the output mix.
* Window placement: every window lies inside its tile, has min(16, tile side)
  extent, and tiles cover the output exactly once (ragged edges included).
* Decision: flips > tau * count (strict), brute-forced on a tiny map.
"""
import numpy as np

from tests import fallback_ref as ref


def test_splitmix64_published_sequence():
    g, s, out = 0x9E3779B97F4A7C15, 1234567, []
    for _ in range(5):
        out.append(ref.mix64(s))
        s = (s + g) & ((1 << 64) - 1)
    assert out == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_windows_inside_tiles_and_cover():
    Z, Ho, Wo, tile = 2, 70, 45, 32
    wins = ref.tile_windows(Z, Ho, Wo, tile, 5, 9)
    ty, tx = 3, 2
    assert len(wins) == Z * ty * tx
    cover = np.zeros((Z, Ho, Wo), dtype=int)
    for t, ws in enumerate(wins):
        z, a, b = t // (ty * tx), (t // tx) % ty, t % tx
        y0, x0 = a * tile, b * tile
        th, tw = min(tile, Ho - y0), min(tile, Wo - x0)
        cover[z, y0:y0 + th, x0:x0 + tw] += 1
        assert len(ws) == 5
        for (zz, y, x, h, w) in ws:
            assert zz == z and h == min(16, th) and w == min(16, tw)
            assert y0 <= y and y + h <= y0 + th and x0 <= x and x + w <= x0 + tw
    assert (cover == 1).all()


def test_decision_is_strict_and_counts_brute_force():
    rng = np.random.default_rng(0)
    S = rng.uniform(0, 1, size=(1, 40, 40))
    T = rng.uniform(0, 1, size=(1, 40, 40))
    wins = ref.tile_windows(1, 40, 40, 20, 3, 1)
    flips, counts = ref.flips_and_counts(S, T, wins)
    for t, ws in enumerate(wins):
        f = c = 0
        for (z, y, x, h, w) in ws:
            for i in range(h):
                for j in range(w):
                    f += (S[z, y + i, x + j] >= 0.5) != (T[z, y + i, x + j] >= 0.5)
                    c += 1
        assert (f, c) == (flips[t], counts[t])
    tau = float(flips[0]) / float(counts[0])
    assert ref.decide(flips, counts, tau)[0] == 0 or np.float32(tau) * np.float32(counts[0]) < flips[0]
    assert ref.decide(np.array([5]), np.array([10]), 0.5)[0] == 0
    assert ref.decide(np.array([6]), np.array([10]), 0.5)[0] == 1
    assert ref.decide(np.array([0]), np.array([10]), -1.0)[0] == 1
    assert ref.decide(np.array([10]), np.array([10]), 1.0)[0] == 0
