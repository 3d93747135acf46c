"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test ties the oracle to something other than itself: hand-worked values,
closed forms (constant images), the edge/corner preservation guarantee
(Sec. II-A end, Sec. III-E), the maximum principle of averaging, an
exact-rational brute force, a 1D reduction checked against numpy's moving
averages, and the appendix's definition evaluated with scipy's 2D convolution.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.signal import convolve2d

import oracle
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


# ------------------------------------------------------------ golden, by hand

def _golden():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", [c for c in _golden() if c.get("method", "exact") == "exact"],
                         ids=lambda c: c["name"])
def test_hand_worked(case):
    img = np.array(case["image"], np.float64)
    r, T = case["r"], case["T"]
    out, sel = oracle.forward(img, r, T, return_sel=True)
    if "out" in case:
        np.testing.assert_array_equal(out, np.array(case["out"], np.float64))
    if "sel" in case:
        np.testing.assert_array_equal(sel[-1, 0], np.array(case["sel"]))
    if "sel_per_sweep" in case:
        np.testing.assert_array_equal(sel[:, 0], np.array(case["sel_per_sweep"]))
    if "pixel" in case:
        x, y = case["pixel"]
        want = float(Fraction(case["pixel_out"]))
        assert out[y, x] == pytest.approx(want, abs=1e-15)
        assert sel[0, 0, y, x] == case["pixel_sel"]
        # the eight means, via the scaled distances the oracle reports
        _, _, err = oracle.sweep(img, r)
        means = [Fraction(m) for m in case["means"]]
        c = Fraction(img[y, x])
        N = (r + 1) ** 2 * (2 * r + 1)
        for i, m in enumerate(means):
            assert err[y, x, i] == pytest.approx(float(abs(m - c) * N), abs=1e-12)


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("r,T", [(0, 3), (1, 1), (2, 5), (5, 2)])
def test_constant_image_unchanged(r, T):
    img = np.full((2, 7, 9), 0.375)
    np.testing.assert_array_equal(oracle.forward(img, r, T), img)


def test_identity_cases():
    rng = np.random.default_rng(0)
    img = rng.random((2, 6, 5))
    np.testing.assert_array_equal(oracle.forward(img, 0, 4), img)
    np.testing.assert_array_equal(oracle.forward(img, 3, 0), img)


def test_maximum_principle():
    rng = np.random.default_rng(1)
    img = rng.random((3, 17, 13))
    for r, T in [(1, 4), (2, 3), (4, 2)]:
        out = oracle.forward(img, r, T)
        for p in range(3):
            assert out[p].min() >= img[p].min() - 1e-12
            assert out[p].max() <= img[p].max() + 1e-12


# --------------------------------------------- edge / corner preservation

@pytest.mark.parametrize("a,b,c", [(1, 0, 5), (0, 1, 7), (1, 1, 9), (2, -1, 3), (1, -3, -4), (3, 2, 20)])
@pytest.mark.parametrize("r", [1, 2, 3])
def test_straight_step_edge_is_fixed_point(a, b, c, r):
    """A straight edge a*x + b*y >= c between two dyadic levels: every pixel has
    a quadrant wholly on its own side (the clamp keeps it there), so its own
    level is at distance 0 and the image is a fixed point for any T."""
    H, W = 15, 16
    yy, xx = np.mgrid[0:H, 0:W]
    img = np.where(a * xx + b * yy >= c, 0.75, 0.125)
    out = oracle.forward(img, r, 6)
    np.testing.assert_array_equal(out, img)


def _uniform_window_exists(img, r):
    """Brute force: does any of the eight (clamped) windows hold only the
    centre's value?"""
    H, W = img.shape
    ok = np.zeros((H, W), bool)
    for y in range(H):
        for x in range(W):
            for w in range(8):
                x0, x1, y0, y1 = oracle.window_extent(w, x, y, r)
                xs = np.clip(np.arange(x0, x1 + 1), 0, W - 1)
                ys = np.clip(np.arange(y0, y1 + 1), 0, H - 1)
                if np.all(img[np.ix_(ys, xs)] == img[y, x]):
                    ok[y, x] = True
                    break
    return ok


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_corner_preservation_predicate(seed):
    """Overlapping dyadic rectangles: every pixel that has a window made only
    of its own level keeps its value exactly after one sweep."""
    from paper_2108_05021_amd.synth import dyadic_rectangles
    rng = np.random.default_rng(seed)
    img = dyadic_rectangles(18, 21, 6, rng).astype(np.float64)
    for r in (1, 2, 3):
        ok = _uniform_window_exists(img, r)
        out = oracle.forward(img, r, 1)
        assert ok.sum() > 0
        np.testing.assert_array_equal(out[ok], img[ok])


def test_axis_aligned_rectangles_fixed_point():
    """Rectangles whose sides and gaps are at least 2r: every pixel keeps a
    uniform window, so the image never changes."""
    r = 2
    img = np.full((24, 30), 0.5)
    img[4:12, 5:13] = 0.25      # 8x8 block
    img[16:24, 0:10] = 1.0      # touches the bottom and left borders
    img[0:8, 20:30] = 0.0       # touches the top and right borders
    assert _uniform_window_exists(img, r).all()
    np.testing.assert_array_equal(oracle.forward(img, r, 7), img)


# ------------------------------------------------ exact rational brute force

@pytest.mark.parametrize("seed,H,W,r,T", [(0, 5, 6, 1, 3), (1, 7, 5, 2, 2), (2, 6, 6, 3, 2),
                                          (3, 9, 4, 1, 3), (4, 4, 9, 2, 3)])
def test_exact_rational_random(seed, H, W, r, T):
    rng = np.random.default_rng(seed)
    img = rng.random((H, W))
    ex_u, ex_sel = exact.forward(img, r, T)
    out, sel = oracle.forward(img, r, T, return_sel=True)
    np.testing.assert_allclose(out, np.array([[float(v) for v in row] for row in ex_u]),
                               rtol=0, atol=1e-13)
    np.testing.assert_array_equal(sel[:, 0], np.array(ex_sel))


@pytest.mark.parametrize("seed,r", [(10, 1), (11, 2), (12, 3)])
def test_exact_ties_integer_data(seed, r):
    """Values in {0..3}: exact ties are common; the FP64 oracle, its int64
    path and the rational brute force must all resolve them identically."""
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 4, size=(8, 9))
    ex_u, ex_sel = exact.forward(img, r, 1)
    out, sel = oracle.forward(img.astype(np.float64), r, 1, return_sel=True)
    isel, _ = oracle.select_int64(img, r)
    np.testing.assert_array_equal(sel[0, 0], np.array(ex_sel[0]))
    np.testing.assert_array_equal(isel, np.array(ex_sel[0]))
    np.testing.assert_allclose(out, np.array([[float(v) for v in row] for row in ex_u]), atol=1e-15)


def test_exact_two_sweeps_integer_data():
    rng = np.random.default_rng(13)
    img = rng.integers(0, 5, size=(6, 7))
    ex_u, ex_sel = exact.forward(img, 2, 2)
    out, sel = oracle.forward(img.astype(np.float64), 2, 2, return_sel=True)
    np.testing.assert_allclose(out, np.array([[float(v) for v in row] for row in ex_u]), atol=1e-14)
    np.testing.assert_array_equal(sel[:, 0], np.array(ex_sel))


# --------------------------------------------------- 1D textbook reductions

def _filter_1d(v, r, T, order):
    """Textbook 1D filter in exact rationals: at each sample take, among the
    right mean v[x..x+r], the left mean v[x-r..x] and the centred mean
    v[x-r..x+r] (edge-replicated), the first in ``order`` closest to v[x]."""
    v = [Fraction(t) for t in v]
    n = len(v)
    for _ in range(T):
        at = lambda i: v[min(max(i, 0), n - 1)]
        nxt = []
        for x in range(n):
            cands = {"right": sum(at(x + j) for j in range(r + 1)) / (r + 1),
                     "left": sum(at(x - j) for j in range(r + 1)) / (r + 1),
                     "cent": sum(at(x + j) for j in range(-r, r + 1)) / (2 * r + 1)}
            best = None
            for k in order:
                d = abs(cands[k] - v[x])
                if best is None or d < best[0]:
                    best = (d, cands[k])
            nxt.append(best[1])
        v = nxt
    return np.array([float(t) for t in v])


def _row(seed, n, T):
    rng = np.random.default_rng(seed)
    # T = 1: eighths, so exact ties occur; T > 1: generic floats (no exact ties)
    return rng.integers(0, 64, size=n) / 8.0 if T == 1 else rng.random(n)


@pytest.mark.parametrize("r,T", [(1, 1), (2, 1), (4, 1), (1, 3), (2, 3), (3, 2)])
def test_rows_constant_reduce_to_1d(r, T):
    """Identical rows: R=SE=NE is the right mean, L=SW=NW the left mean and
    D=U the centred mean; the first-minimum order R, L, D becomes right,
    left, centred."""
    row = _row(20 + r, 23, T)
    img = np.tile(row, (7, 1))
    out = oracle.forward(img, r, T)
    want = _filter_1d(row, r, T, ("right", "left", "cent"))
    np.testing.assert_allclose(out, np.tile(want, (7, 1)), atol=1e-13)


@pytest.mark.parametrize("r,T", [(1, 1), (2, 1), (4, 1), (1, 3), (2, 3), (3, 2)])
def test_columns_constant_reduce_to_1d(r, T):
    """Identical columns: R=L is the centred vertical mean, D=SE=SW the
    downward mean, U=NE=NW the upward mean; order centred, down, up."""
    col = _row(30 + r, 19, T)
    img = np.tile(col[:, None], (1, 6))
    out = oracle.forward(img, r, T)
    want = _filter_1d(col, r, T, ("cent", "right", "left"))  # 'right' = rows y..y+r
    np.testing.assert_allclose(out, np.tile(want[:, None], (1, 6)), atol=1e-13)


# --------------------------------------- appendix definition via scipy conv2

def _appendix_planes(frame, r):
    """Window sums of the appendix's eight kernel pairs on a frame (zero beyond
    it), using scipy's 2D convolution in 'same' mode. The 1D kernels are the
    centred box k (2r+1 taps), k_L (weight on the first r+1 taps) and its flip
    k_R; the pairs (column kernel, row kernel) come in the listing's order."""
    k = np.ones(2 * r + 1)
    kL = np.zeros(2 * r + 1)
    kL[:r + 1] = 1.0
    kR = kL[::-1].copy()
    pairs = [(k, kL), (k, kR), (kL, k), (kR, k), (kL, kL), (kL, kR), (kR, kL), (kR, kR)]
    sums = np.stack([convolve2d(frame, np.outer(u, v), mode="same") for u, v in pairs])
    counts = np.array([u.sum() * v.sum() for u, v in pairs])
    return sums, counts


def _appendix_forward(img, r, T):
    """Pad once by replicate, T sweeps on the frame, crop (integer-exact sums)."""
    frame = np.pad(img.astype(np.float64), r, mode="edge")
    sels = []
    for _ in range(T):
        sums, counts = _appendix_planes(frame, r)
        N = (r + 1) ** 2 * (2 * r + 1)
        w = N / counts                                   # 2r+1 for quadrants, r+1 for halves
        e = np.abs(w[:, None, None] * sums - N * frame)
        idx = np.argmin(e, axis=0)
        frame = np.take_along_axis(sums, idx[None], 0)[0] / counts[idx]
        sels.append(idx[r:frame.shape[0] - r, r:frame.shape[1] - r])
    return frame[r:frame.shape[0] - r, r:frame.shape[1] - r], sels


@pytest.mark.parametrize("seed,H,W,r", [(40, 12, 15, 1), (41, 16, 11, 2), (42, 9, 20, 3), (43, 21, 21, 4)])
def test_appendix_definition_one_sweep_matches_clamp_mode(seed, H, W, r):
    """For one sweep, replicate-pad-once and the per-sweep clamp read the same
    values, so the library-convolution evaluation of the appendix must equal the
    oracle everywhere: values, and the selection map bit for bit (integer data,
    exact distances). This pins window orientation, divisors and tie order."""
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=(H, W)).astype(np.float64)
    want, sels = _appendix_forward(img, r, 1)
    out, sel = oracle.forward(img, r, 1, return_sel=True)
    np.testing.assert_array_equal(sel[0, 0], sels[0])
    np.testing.assert_array_equal(out, want)


@pytest.mark.parametrize("seed,r,T", [(50, 1, 4), (51, 2, 3), (52, 3, 2)])
def test_padonce_mode_and_interior_agreement(seed, r, T):
    """The oracle's pad-once mode equals the scipy evaluation everywhere; the
    clamp mode agrees with both on pixels at least r*(T-1) from every edge."""
    rng = np.random.default_rng(seed)
    H, W = 20, 23
    img = rng.integers(0, 256, size=(H, W)).astype(np.float64)
    want, _ = _appendix_forward(img, r, T)
    pad = oracle.forward_padonce(img, r, T)
    np.testing.assert_allclose(pad, want, rtol=0, atol=1e-9)
    clamp = oracle.forward(img, r, T)
    m = r * (T - 1)
    np.testing.assert_allclose(clamp[m:H - m, m:W - m], want[m:H - m, m:W - m], rtol=0, atol=1e-9)
    # near the edge the two boundary readings do differ for T > 1
    assert np.abs(clamp - want).max() > 1e-6


# ------------------------------------------------------------- symmetries

def test_flip_and_transpose_equivariance():
    rng = np.random.default_rng(60)
    img = rng.random((13, 17))
    r, T = 2, 3
    out = oracle.forward(img, r, T)
    np.testing.assert_allclose(oracle.forward(img[:, ::-1], r, T), out[:, ::-1], atol=1e-13)
    np.testing.assert_allclose(oracle.forward(img[::-1, :], r, T), out[::-1, :], atol=1e-13)
    np.testing.assert_allclose(oracle.forward(img.T.copy(), r, T), out.T, atol=1e-13)


# ------------------------------------------------------------ adjoint pins

@pytest.mark.parametrize("seed,H,W,r", [(70, 9, 11, 1), (71, 13, 7, 2), (72, 6, 6, 3), (73, 1, 9, 2), (74, 8, 1, 1)])
def test_adjoint_dot_product(seed, H, W, r):
    """<A x, y> = <x, A^T y> for the sweep with its selection held fixed."""
    rng = np.random.default_rng(seed)
    u = rng.random((H, W))
    _, sel, _ = oracle.sweep(u, r)
    x, y = rng.normal(size=(H, W)), rng.normal(size=(H, W))
    lhs = float(np.sum(oracle.apply_fixed(x, sel, r) * y))
    rhs = float(np.sum(x * oracle.adjoint(y, sel, r)))
    assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12)


def test_adjoint_dense_matrix():
    """The adjoint equals the transpose of the forward map's dense matrix,
    built column by column from unit images."""
    rng = np.random.default_rng(75)
    H, W, r = 5, 6, 2
    u = rng.random((H, W))
    _, sel, _ = oracle.sweep(u, r)
    n = H * W
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = oracle.apply_fixed(e.reshape(H, W), sel, r).ravel()
    # every row of A averages one window: non-negative, sums to one
    assert (A >= 0).all()
    np.testing.assert_allclose(A.sum(axis=1), 1.0, atol=1e-14)
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        np.testing.assert_allclose(oracle.adjoint(e.reshape(H, W), sel, r).ravel(), A[j], atol=1e-14)


def test_adjoint_conserves_mass():
    rng = np.random.default_rng(76)
    u = rng.random((12, 10))
    _, sel, _ = oracle.sweep(u, 3)
    g = rng.normal(size=u.shape)
    assert oracle.adjoint(g, sel, 3).sum() == pytest.approx(g.sum(), rel=1e-12)


@pytest.mark.parametrize("seed,r,T", [(80, 1, 3), (81, 2, 2), (82, 3, 2)])
def test_backward_matches_finite_differences(seed, r, T):
    """The filter is piecewise linear in its input: where a +-h perturbation
    of a pixel changes no selection map, the central difference of
    sum(w * filter(x)) equals the gradient up to FP64 rounding."""
    rng = np.random.default_rng(seed)
    H, W = 10, 9
    x = rng.random((H, W))
    w = rng.normal(size=(H, W))
    grad, sel = oracle.backward(x, w, r, T, return_sel=True)
    h = 1e-6
    checked = 0
    for (yy, xx) in [(0, 0), (4, 5), (9, 8), (2, 7), (7, 1), (5, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[yy, xx] += h
        xm[yy, xx] -= h
        yp, sp = oracle.forward(xp, r, T, return_sel=True)
        ym, sm = oracle.forward(xm, r, T, return_sel=True)
        if not (np.array_equal(sp, sel) and np.array_equal(sm, sel)):
            continue
        fd = (np.sum(w * yp) - np.sum(w * ym)) / (2 * h)
        assert fd == pytest.approx(grad[yy, xx], rel=1e-6, abs=1e-8)
        checked += 1
    assert checked >= 3


# ------------------------------------------- fast approximation (Alg. 3)

@pytest.mark.parametrize("case", [c for c in _golden() if c.get("method") == "fast"], ids=lambda c: c["name"])
def test_fast_hand_worked(case):
    u = np.array(case["image"], np.float64)
    for t in range(case["T"]):
        u, sel, _ = oracle.fast_sweep(u, case["r"])
        np.testing.assert_array_equal(u, np.array(case["out_per_sweep"][t], np.float64))
        np.testing.assert_array_equal(sel, np.array(case["sel_per_sweep"][t]))
    np.testing.assert_array_equal(oracle.fast_forward(np.array(case["image"], float), case["r"], case["T"]), u)


@pytest.mark.parametrize("seed,r", [(90, 1), (91, 2), (92, 4)])
def test_fast_candidates_are_exact_quadrants_and_pair_averages(seed, r):
    """The fast filter's quadrant candidates are the exact filter's quadrant
    means, and each half candidate is the mean of its two quadrants (eq:app);
    the exact oracle computes these from its own direct window sums."""
    rng = np.random.default_rng(seed)
    u = rng.random((11, 13))
    _, _, cand = oracle.fast_sweep(u, r)
    _, _, _, means = oracle.sweep(u, r, return_means=True)
    np.testing.assert_allclose(cand[..., 4:], means[..., 4:], rtol=0, atol=1e-14)
    SE, SW, NE, NW = (means[..., i] for i in (4, 5, 6, 7))
    want_halves = np.stack([(NE + SE) / 2, (NW + SW) / 2, (SW + SE) / 2, (NW + NE) / 2], axis=-1)
    np.testing.assert_allclose(cand[..., :4], want_halves, rtol=0, atol=1e-14)


def test_fast_invariants():
    img = np.full((9, 10), 0.625)
    np.testing.assert_array_equal(oracle.fast_forward(img, 2, 4), img)
    yy, xx = np.mgrid[0:15, 0:16]
    for a, b, c in [(1, 0, 5), (1, 1, 9), (2, -1, 3)]:
        step = np.where(a * xx + b * yy >= c, 0.75, 0.125)
        np.testing.assert_array_equal(oracle.fast_forward(step, 2, 5), step)
    rng = np.random.default_rng(93)
    x = rng.random((2, 14, 12))
    out = oracle.fast_forward(x, 3, 3)
    for p in range(2):
        assert out[p].min() >= x[p].min() - 1e-12 and out[p].max() <= x[p].max() + 1e-12


def _fast_1d(v, r, T):
    """Exact-rational 1D fast filter: candidates right mean, left mean and
    their average, first minimum in that order (R, L, D)."""
    v = [Fraction(t) for t in v]
    n = len(v)
    for _ in range(T):
        at = lambda i: v[min(max(i, 0), n - 1)]
        nxt = []
        for x in range(n):
            right = sum(at(x + j) for j in range(r + 1)) / (r + 1)
            left = sum(at(x - j) for j in range(r + 1)) / (r + 1)
            best = None
            for cval in (right, left, (left + right) / 2):
                dd = abs(cval - v[x])
                if best is None or dd < best[0]:
                    best = (dd, cval)
            nxt.append(best[1])
        v = nxt
    return np.array([float(t) for t in v])


@pytest.mark.parametrize("r,T", [(1, 1), (2, 1), (1, 3), (3, 2)])
def test_fast_rows_constant_reduce_to_1d(r, T):
    row = _row(60 + r, 21, T)
    out = oracle.fast_forward(np.tile(row, (5, 1)), r, T)
    np.testing.assert_allclose(out, np.tile(_fast_1d(row, r, T), (5, 1)), atol=1e-13)


# ------------------------------------------------------- box filter baseline

@pytest.mark.parametrize("r,T", [(1, 1), (2, 3), (4, 2)])
def test_box_matches_scipy_uniform_filter(r, T):
    """The classical box filter with replicate boundary is scipy's
    uniform_filter with mode='nearest', applied T times."""
    from scipy.ndimage import uniform_filter
    rng = np.random.default_rng(100 + r)
    img = rng.random((17, 23))
    want = img.copy()
    for _ in range(T):
        want = uniform_filter(want, size=2 * r + 1, mode="nearest")
    np.testing.assert_allclose(oracle.box_forward(img, r, T), want, rtol=0, atol=1e-13)
