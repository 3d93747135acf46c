"""Exact-rational brute force of the one-sided box filter for tiny inputs.

TEST INFRASTRUCTURE ONLY.  Pure Python with ``fractions.Fraction``: every
window mean and every distance is exact, so exact ties are resolved by the
stated window order (R, L, D, U, SE, SW, NE, NW) without rounding.  It pins the
FP64 oracle in ``osbf_oracle.c``; it is far too slow for anything but images of
a few dozen pixels.

Windows follow Sec. II-A (Eq. 6-13) with y pointing down, boundary is the
per-sweep replicate extension, iteration is T Jacobi sweeps of Alg. 2.
"""
from __future__ import annotations

from fractions import Fraction

ORDER = ("R", "L", "D", "U", "SE", "SW", "NE", "NW")


def _span(name: str, x: int, y: int, r: int):
    xs = {"R": (x, x + r), "L": (x - r, x), "D": (x - r, x + r), "U": (x - r, x + r),
          "SE": (x, x + r), "SW": (x - r, x), "NE": (x, x + r), "NW": (x - r, x)}[name]
    ys = {"R": (y - r, y + r), "L": (y - r, y + r), "D": (y, y + r), "U": (y - r, y),
          "SE": (y, y + r), "SW": (y, y + r), "NE": (y - r, y), "NW": (y - r, y)}[name]
    return xs, ys


def window_mean(u, name: str, x: int, y: int, r: int) -> Fraction:
    H, W = len(u), len(u[0])
    (x0, x1), (y0, y1) = _span(name, x, y, r)
    total = Fraction(0)
    count = 0
    for yy in range(y0, y1 + 1):
        for xx in range(x0, x1 + 1):
            total += u[min(max(yy, 0), H - 1)][min(max(xx, 0), W - 1)]
            count += 1
    return total / count


def sweep(u, r: int):
    """One Jacobi sweep; returns (next iterate, selection indices)."""
    H, W = len(u), len(u[0])
    nxt = [[Fraction(0)] * W for _ in range(H)]
    sel = [[0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            c = u[y][x]
            best = None
            for i, name in enumerate(ORDER):
                mean = window_mean(u, name, x, y, r)
                dist = abs(mean - c)
                if best is None or dist < best[0]:
                    best = (dist, i, mean)
            nxt[y][x] = best[2]
            sel[y][x] = best[1]
    return nxt, sel


def forward(img, r: int, T: int):
    """T sweeps on a list-of-lists (or 2D array) image; returns (U^T, [sel_t])."""
    u = [[Fraction(v) for v in row] for row in img]
    sels = []
    for _ in range(T):
        u, s = sweep(u, r)
        sels.append(s)
    return u, sels


# ----------------------------------------------------------------- volumes
# Sec. "Higher Dimension Case": along each axis a window is one-sided towards
# + ([c, c+r]), towards - ([c-r, c]) or full ([c-r, c+r]).  Six halves take one
# axis one-sided and two full; eight octants are one-sided along all three.
# Order (= tie order): +x, -x, +y, -y, +z, -z, then octants with x varying
# fastest and + before - on every axis.

def _sides3():
    halves = []
    for axis in range(3):
        for s in (1, -1):
            side = [0, 0, 0]
            side[axis] = s
            halves.append(tuple(side))
    octants = [(sx, sy, sz) for sz in (1, -1) for sy in (1, -1) for sx in (1, -1)]
    return halves + octants


SIDES3 = _sides3()


def _range(c: int, s: int, r: int):
    return range(c, c + r + 1) if s > 0 else range(c - r, c + 1) if s < 0 else range(c - r, c + r + 1)


def window_mean3(u, side, x: int, y: int, z: int, r: int) -> Fraction:
    D, H, W = len(u), len(u[0]), len(u[0][0])
    total = Fraction(0)
    count = 0
    for zz in _range(z, side[2], r):
        for yy in _range(y, side[1], r):
            for xx in _range(x, side[0], r):
                total += u[min(max(zz, 0), D - 1)][min(max(yy, 0), H - 1)][min(max(xx, 0), W - 1)]
                count += 1
    return total / count


def sweep3(u, r: int):
    """One Jacobi sweep on a volume u[z][y][x]; returns (next, selection)."""
    D, H, W = len(u), len(u[0]), len(u[0][0])
    nxt = [[[Fraction(0)] * W for _ in range(H)] for _ in range(D)]
    sel = [[[0] * W for _ in range(H)] for _ in range(D)]
    for z in range(D):
        for y in range(H):
            for x in range(W):
                c = u[z][y][x]
                best = None
                for i, side in enumerate(SIDES3):
                    mean = window_mean3(u, side, x, y, z, r)
                    dist = abs(mean - c)
                    if best is None or dist < best[0]:
                        best = (dist, i, mean)
                nxt[z][y][x] = best[2]
                sel[z][y][x] = best[1]
    return nxt, sel


def forward3(vol, r: int, T: int):
    """T sweeps on a volume; returns (U^T, [sel_t])."""
    u = [[[Fraction(v) for v in row] for row in sl] for sl in vol]
    sels = []
    for _ in range(T):
        u, s = sweep3(u, r)
        sels.append(s)
    return u, sels
