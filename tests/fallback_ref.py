"""Host reference of the student fallback decisions (multi-pass scheme, paper
Section 1: a fast pass everywhere, extra effort only where errors are likely).

Given the student map in the teacher's output frame and the teacher map, it
places the sample windows by the rule the C header documents (splitmix64 output
mix, Steele, Lea and Flood 2014), counts the voxels whose 0.5-threshold
decisions differ, and flags a tile when flips > tau * count in float32. It is
written from that documented rule and shares no code with the library.
"""
import numpy as np

_M64 = (1 << 64) - 1


def mix64(x: int) -> int:
    """splitmix64 output function applied to x + golden-ratio increment (mod 2^64)."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def tile_windows(Z, Ho, Wo, tile, n_samples, seed):
    """For every tile t (numbered (z * ty + a) * tx + b): list of windows (z, y, x, h, w)."""
    ty, tx = -(-Ho // tile), -(-Wo // tile)
    out = []
    for z in range(Z):
        for a in range(ty):
            for b in range(tx):
                t = (z * ty + a) * tx + b
                y0, x0 = a * tile, b * tile
                th, tw = min(tile, Ho - y0), min(tile, Wo - x0)
                wh, ww = min(16, th), min(16, tw)
                wins = []
                for k in range(n_samples):
                    r = mix64(seed ^ mix64(t * 64 + k))
                    oy = r % (th - wh + 1)
                    ox = (r >> 32) % (tw - ww + 1)
                    wins.append((z, y0 + oy, x0 + ox, wh, ww))
                out.append(wins)
    return out


def flips_and_counts(student, teacher, windows):
    """Per tile: (flips, sampled-voxel count) of the 0.5-threshold decisions."""
    dis = (student >= 0.5) != (teacher >= 0.5)
    flips = np.zeros(len(windows), dtype=np.int64)
    counts = np.zeros(len(windows), dtype=np.int64)
    for t, wins in enumerate(windows):
        for (z, y, x, h, w) in wins:
            flips[t] += int(dis[z, y:y + h, x:x + w].sum())
            counts[t] += h * w
    return flips, counts


def decide(flips, counts, tau):
    """flips > tau * count, evaluated in float32 as the decision is specified."""
    return (flips.astype(np.float32) > np.float32(tau) * counts.astype(np.float32)).astype(np.int32)
