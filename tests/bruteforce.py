"""Pure-Python nested-loop forward pass, used only to pin the C reference on tiny
inputs. Same definitions (valid cross-correlation, ReLU, 2x2 stride-1 max filter,
sigmoid) and the same summation order (bias first, then ci, i, j ascending), so
results are bitwise equal to the C reference.
"""
import math


def sigmoid(t):
    if t >= 0.0:
        return 1.0 / (1.0 + math.exp(-t))
    e = math.exp(t)
    return e / (1.0 + e)


def forward_slice(img, net, params):
    H, W = len(img), len(img[0])
    a = [[[img[y][x] / 255.0 for x in range(W)] for y in range(H)]]
    off = 0
    for L in net:
        C, h, w = len(a), len(a[0]), len(a[0][0])
        if L["kind"] == "pool":
            a = [[[max(a[c][y][x], a[c][y][x + 1], a[c][y + 1][x], a[c][y + 1][x + 1])
                   for x in range(w - 1)] for y in range(h - 1)] for c in range(C)]
            continue
        k, ci_n, co_n = L["k"], L["cin"], L["cout"]
        assert ci_n == C
        nw = co_n * ci_n * k * k
        wt = params[off:off + nw]
        bs = params[off + nw:off + nw + co_n]
        off += nw + co_n
        out = []
        for co in range(co_n):
            plane = []
            for y in range(h - k + 1):
                row = []
                for x in range(w - k + 1):
                    s = bs[co]
                    for ci in range(ci_n):
                        for i in range(k):
                            for j in range(k):
                                s += wt[((co * ci_n + ci) * k + i) * k + j] * a[ci][y + i][x + j]
                    if L["act"] == "relu":
                        s = s if s > 0.0 else 0.0
                    elif L["act"] == "sigmoid":
                        s = sigmoid(s)
                    row.append(s)
                plane.append(row)
            out.append(plane)
        a = out
    assert len(a) == 1
    return a[0]
