"""Parity protocol between the HIP path and the FP64 oracle.

One sweep is compared teacher-forced: the oracle runs one sweep on exactly the
GPU's input iterate.  Every GPU value must lie within ``tol`` of the oracle's
mean for the window the GPU selected, and that window must be a true minimum
or a near-tie flip: the oracle's scaled distance for the GPU's window may
exceed the minimum by at most tau = 2^-19 * N * (1 + max|U|), a bound on the
FP32 rounding of the window sums (N = (r+1)^2 (2r+1)).
"""
from __future__ import annotations

import numpy as np

import oracle


def tau(r: int, u: np.ndarray) -> float:
    N = (r + 1) ** 2 * (2 * r + 1)
    return 2.0 ** -19 * N * (1.0 + float(np.abs(u).max()))


def check_sweep(u_in, u_out, r: int, sel=None, tol: float = 1e-5):
    """Teacher-forced check of one sweep on one plane.

    u_in, u_out: (H, W) arrays (GPU input and output iterate, any float type).
    sel: optional GPU selection map (H, W).  Returns a stats dict; raises
    AssertionError on a violation.
    """
    u_in = np.asarray(u_in, np.float64)
    u_out = np.asarray(u_out, np.float64)
    _, sel_o, err, means = oracle.sweep(u_in, r, return_means=True)
    t = tau(r, u_in)
    emin = err.min(axis=2)
    H, W = u_in.shape
    if sel is not None:
        sel = np.asarray(sel).astype(np.int64)
        assert sel.min() >= 0 and sel.max() <= 7, "selection index out of range"
        e_gpu = np.take_along_axis(err, sel[..., None], 2)[..., 0]
        bad = e_gpu - emin > t
        assert not bad.any(), (f"{int(bad.sum())} selections are not near-minimal "
                               f"(worst gap {float((e_gpu - emin).max()):.3e} > tau {t:.3e})")
        want = np.take_along_axis(means, sel[..., None], 2)[..., 0]
        dev = np.abs(u_out - want)
        assert dev.max() <= tol, f"value off the selected mean by {dev.max():.3e} > {tol}"
        # a flip that matters picks a window whose mean differs from the oracle's choice
        m_o = np.take_along_axis(means, sel_o[..., None].astype(np.int64), 2)[..., 0]
        flips = int(((sel != sel_o) & (np.abs(want - m_o) > tol)).sum())
    else:
        # value must equal the mean of some near-minimal window
        near = err - emin[..., None] <= t
        dev_all = np.abs(u_out[..., None] - means)
        dev = np.where(near, dev_all, np.inf).min(axis=2)
        assert dev.max() <= tol, f"value matches no near-minimal window mean (off by {dev.max():.3e})"
        flips = int((np.abs(u_out - np.take_along_axis(means, sel_o[..., None].astype(np.int64), 2)[..., 0]) > tol).sum())
    return {"flips": flips, "max_err": float(dev.max()), "pixels": H * W}


def check_sweep_planes(u_in, u_out, r, sel=None, tol=1e-5):
    """check_sweep over the leading plane axes of (..., H, W) arrays."""
    u_in = np.asarray(u_in)
    H, W = u_in.shape[-2:]
    a = u_in.reshape(-1, H, W)
    b = np.asarray(u_out).reshape(-1, H, W)
    s = None if sel is None else np.asarray(sel).reshape(-1, H, W)
    tot = {"flips": 0, "max_err": 0.0, "pixels": 0}
    for p in range(a.shape[0]):
        st = check_sweep(a[p], b[p], r, None if s is None else s[p], tol)
        tot["flips"] += st["flips"]
        tot["pixels"] += st["pixels"]
        tot["max_err"] = max(tot["max_err"], st["max_err"])
    return tot


def crop_check(u_in, u_out, r, sel, y0, x0, size, tol=1e-5):
    """Teacher-forced check of one sweep on a crop of a large plane: the oracle
    runs on the crop grown by r (clipped to the image); pixels of the crop whose
    windows stay inside that region are exact."""
    H, W = u_in.shape
    ya, yb = max(0, y0 - r), min(H, y0 + size + r)
    xa, xb = max(0, x0 - r), min(W, x0 + size + r)
    sub_in = np.asarray(u_in[ya:yb, xa:xb], np.float64)
    _, sel_o, err, means = oracle.sweep(sub_in, r, return_means=True)
    # interior of the grown crop: pixels at distance >= r from a cut that is not an image edge
    iy0 = 0 if ya == 0 else r
    ix0 = 0 if xa == 0 else r
    iy1 = (yb - ya) if yb == H else (yb - ya - r)
    ix1 = (xb - xa) if xb == W else (xb - xa - r)
    err = err[iy0:iy1, ix0:ix1]
    means = means[iy0:iy1, ix0:ix1]
    out = np.asarray(u_out[ya + iy0:ya + iy1, xa + ix0:xa + ix1], np.float64)
    s = np.asarray(sel[ya + iy0:ya + iy1, xa + ix0:xa + ix1]).astype(np.int64)
    t = tau(r, sub_in)
    emin = err.min(axis=2)
    e_gpu = np.take_along_axis(err, s[..., None], 2)[..., 0]
    assert (e_gpu - emin <= t).all(), "crop: selection not near-minimal"
    want = np.take_along_axis(means, s[..., None], 2)[..., 0]
    dev = np.abs(out - want)
    assert dev.max() <= tol, f"crop: value off by {dev.max():.3e}"
    so = sel_o[iy0:iy1, ix0:ix1].astype(np.int64)
    m_o = np.take_along_axis(means, so[..., None], 2)[..., 0]
    return int(((s != so) & (np.abs(want - m_o) > tol)).sum()), out.size


def replay_check(u0, u_gpu, sels, r: int, tol: float = 1e-5, max_outliers: int = 0):
    """End-to-end check of T sweeps: the oracle replays the GPU's selection
    maps (its linear map with each selection held fixed, in FP64); every GPU
    selection must be near-minimal for the replayed iterate, and the GPU's
    final iterate must equal the replay within ``tol``.  ``max_outliers``
    allows a few pixels to miss both tests (fused launches recompute halo
    pixels in neighbouring tiles, where a near-tie may resolve differently
    from the owner tile's map).  Returns (outliers, max deviation, flips vs
    the oracle's own choice)."""
    u = np.asarray(u0, np.float64)
    sels = np.asarray(sels)
    bad = np.zeros(u.shape, bool)
    flips = 0
    for t in range(sels.shape[0]):
        s = sels[t].astype(np.int64)
        _, sel_o, err, means = oracle.sweep(u, r, return_means=True)
        emin = err.min(axis=2)
        e_gpu = np.take_along_axis(err, s[..., None], 2)[..., 0]
        bad |= e_gpu - emin > tau(r, u)
        nxt = np.take_along_axis(means, s[..., None], 2)[..., 0]
        m_o = np.take_along_axis(means, sel_o[..., None].astype(np.int64), 2)[..., 0]
        flips += int(((s != sel_o) & (np.abs(nxt - m_o) > tol)).sum())
        u = nxt
    dev = np.abs(np.asarray(u_gpu, np.float64) - u)
    bad |= dev > tol
    n_bad = int(bad.sum())
    assert n_bad <= max_outliers, f"{n_bad} pixels fail the replay (max dev {dev.max():.3e})"
    return n_bad, float(dev.max()), flips


def replay_check_planes(u0, u_gpu, sels, r, tol=1e-5, max_outliers=0):
    """replay_check over the plane axes: u0, u_gpu (..., H, W); sels (T, ..., H, W)."""
    u0 = np.asarray(u0)
    H, W = u0.shape[-2:]
    a = u0.reshape(-1, H, W)
    b = np.asarray(u_gpu).reshape(-1, H, W)
    s = np.asarray(sels).reshape(np.shape(sels)[0], -1, H, W)
    tot_bad, worst, flips = 0, 0.0, 0
    for p in range(a.shape[0]):
        n, d, f = replay_check(a[p], b[p], s[:, p], r, tol, max_outliers)
        tot_bad += n
        worst = max(worst, d)
        flips += f
    assert tot_bad <= max_outliers
    return tot_bad, worst, flips


def untethered_errors(u0, u_gpu, sels, r: int):
    """One plane (H, W) against the oracle's own, untethered T sweeps: the
    absolute errors and the flip cones.  A seed is a pixel where the GPU
    selected, at sweep t, a window whose mean on the oracle's iterate differs
    (by more than 1e-7) from the oracle's choice (equal-mean windows, as in
    flat regions, give the same value); its difference may spread by r
    pixels (Chebyshev) per later sweep, so the cone of a seed at sweep t
    reaches r (T - 1 - t) pixels.  Every pixel outside all cones read, at
    every sweep, only values both runs computed with windows of the same
    mean."""
    from scipy.ndimage import maximum_filter
    u = np.asarray(u0, np.float64)
    s = np.asarray(sels)
    T = s.shape[0]
    cone = np.zeros(u.shape, bool)
    for t in range(T):
        nxt, so, _, means = oracle.sweep(u, r, return_means=True)
        m_gpu = np.take_along_axis(means, s[t][..., None].astype(np.int64), 2)[..., 0]
        seed = (s[t] != so) & (np.abs(m_gpu - nxt) > 1e-7)
        if seed.any():
            d = r * (T - 1 - t)
            cone |= maximum_filter(seed, size=2 * d + 1, mode="constant", cval=False) if d else seed
        u = nxt
    return np.abs(np.asarray(u_gpu, np.float64) - u), cone


def untethered_check(u0, u_gpu, sels, r: int, tol: float = 1e-5):
    """untethered_errors over the plane axes (u0, u_gpu (..., H, W), sels
    (T, ..., H, W)); every pixel outside the flip cones must agree within
    ``tol``.  Returns (max error outside the cones, fraction of pixels inside
    them, max error overall)."""
    u0 = np.asarray(u0, np.float64)
    H, W = u0.shape[-2:]
    a = u0.reshape(-1, H, W)
    b = np.asarray(u_gpu, np.float64).reshape(-1, H, W)
    s = np.asarray(sels).reshape(np.shape(sels)[0], -1, H, W)
    errs, cones = zip(*(untethered_errors(a[p], b[p], s[:, p], r) for p in range(a.shape[0])))
    err, cone = np.stack(errs), np.stack(cones)
    outside = float(err[~cone].max()) if (~cone).any() else 0.0
    assert outside <= tol, f"untethered error {outside:.3e} outside the flip cones"
    return outside, float(cone.mean()), float(err.max())


def check_fast_sweep(u_in, u_out, r: int, tol: float = 1e-5):
    """Teacher-forced check of one sweep of the fast approximation (Alg. 3):
    the GPU value must be the oracle's value of a near-minimal candidate
    (distances scaled by 2 (r+1)^2, tau as for the exact filter with that
    scale).  Returns the number of value-changing flips."""
    u_in = np.asarray(u_in, np.float64)
    u_out = np.asarray(u_out, np.float64)
    out_o, sel_o, cand = oracle.fast_sweep(u_in, r)
    scale = 2.0 * (r + 1) ** 2
    err = np.abs(cand - u_in[..., None]) * scale
    emin = err.min(axis=2)
    t = 2.0 ** -19 * scale * (1.0 + float(np.abs(u_in).max()))
    near = err - emin[..., None] <= t
    dev = np.where(near, np.abs(u_out[..., None] - cand), np.inf).min(axis=2)
    assert dev.max() <= tol, f"fast: value matches no near-minimal candidate (off by {dev.max():.3e})"
    return int((np.abs(u_out - out_o) > tol).sum())


def cut_distance(shape, cuts):
    """Distance of every pixel of a region to its nearest interior cut.
    ``cuts`` = (top, bottom, left, right): True where that side of the region
    was cut out of a larger plane (False where it is an image edge, which the
    clamp reproduces exactly)."""
    h, w = shape
    yy, xx = np.mgrid[0:h, 0:w]
    d = np.full(shape, np.iinfo(np.int64).max // 4, np.int64)
    top, bottom, left, right = cuts
    if top:
        d = np.minimum(d, yy)
    if bottom:
        d = np.minimum(d, h - 1 - yy)
    if left:
        d = np.minimum(d, xx)
    if right:
        d = np.minimum(d, w - 1 - xx)
    return d


def region_of(H, W, y0, x0, size, margin):
    """Region [ya, yb) x [xa, xb) of a size x size crop grown by ``margin``
    and clipped to the image, with its cut flags."""
    ya, yb = max(0, y0 - margin), min(H, y0 + size + margin)
    xa, xb = max(0, x0 - margin), min(W, x0 + size + margin)
    return (ya, yb, xa, xb), (ya > 0, yb < H, xa > 0, xb < W)


def sweep_region(u_in, u_out, sel, r, cuts, tol=1e-5):
    """Teacher-forced check of one sweep on a region: pixels at distance >= r
    from every cut see exactly their windows.  Returns (flips, pixels,
    max |value - mean of the selected window|); raises on a violation."""
    u_in = np.asarray(u_in, np.float64)
    _, sel_o, err, means = oracle.sweep(u_in, r, return_means=True)
    ok = cut_distance(u_in.shape, cuts) >= r
    s = np.asarray(sel).astype(np.int64)
    emin = err.min(axis=2)
    e_gpu = np.take_along_axis(err, s[..., None], 2)[..., 0]
    t = tau(r, u_in)
    gap = np.where(ok, e_gpu - emin, 0.0)
    assert (gap <= t).all(), f"selection not near-minimal (gap {gap.max():.3e} > tau {t:.3e})"
    want = np.take_along_axis(means, s[..., None], 2)[..., 0]
    dev = np.where(ok, np.abs(np.asarray(u_out, np.float64) - want), 0.0)
    assert dev.max() <= tol, f"value off the selected mean by {dev.max():.3e}"
    m_o = np.take_along_axis(means, sel_o[..., None].astype(np.int64), 2)[..., 0]
    flips = int((ok & (s != sel_o) & (np.abs(want - m_o) > tol)).sum())
    return flips, int(ok.sum()), float(dev.max())


def replay_region(u0, u_gpu, sels, r, cuts, tol=1e-5):
    """The oracle replays the GPU's T selection maps on a region cut out of a
    larger plane.  At sweep t a pixel's selection is checked (near-minimal
    for the replayed iterate) where its dependency cone, r * (t + 1) wide,
    stays inside the region; the final GPU values are compared with the
    replay where the cone r * T does.  Returns (outliers, max deviation of the
    final values, value-changing flips against the oracle's own choice,
    pixels compared at the end)."""
    u = np.asarray(u0, np.float64)
    sels = np.asarray(sels)
    T = sels.shape[0]
    d = cut_distance(u.shape, cuts)
    bad = np.zeros(u.shape, bool)
    flips = 0
    for t in range(T):
        s = sels[t].astype(np.int64)
        _, sel_o, err, means = oracle.sweep(u, r, return_means=True)
        ok = d >= r * (t + 1)
        emin = err.min(axis=2)
        e_gpu = np.take_along_axis(err, s[..., None], 2)[..., 0]
        bad |= ok & (e_gpu - emin > tau(r, u))
        nxt = np.take_along_axis(means, s[..., None], 2)[..., 0]
        m_o = np.take_along_axis(means, sel_o[..., None].astype(np.int64), 2)[..., 0]
        flips += int((ok & (s != sel_o) & (np.abs(nxt - m_o) > tol)).sum())
        u = nxt
    fin = d >= r * T
    dev = np.where(fin, np.abs(np.asarray(u_gpu, np.float64) - u), 0.0)
    bad |= dev > tol
    return int(bad.sum()), float(dev.max()), flips, int(fin.sum())
