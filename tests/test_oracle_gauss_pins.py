"""Pins of the FP64 one-sided Gaussian oracle (Sec. II-B separable kernels) to
facts outside it: the sigma -> infinity limit is the one-sided box filter,
every window mean equals scipy's weighted correlation with clamp ('nearest')
boundary, the sigma -> 0 limit is the identity, step edges are fixed points,
the maximum principle, mirror symmetry and the identity cases."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2108_05021_amd import synth

SIDES = {"R": (1, 0), "L": (-1, 0), "D": (0, 1), "U": (0, -1),
         "SE": (1, 1), "SW": (-1, 1), "NE": (1, -1), "NW": (-1, -1)}
ORDER = ("R", "L", "D", "U", "SE", "SW", "NE", "NW")


def _kernel(name, r, sigma):
    """(2r+1)^2 correlation kernel of window `name`: weight g(a) g(b) at
    offset (a, b) inside the window, normalised to sum 1."""
    g = np.exp(-np.arange(-r, r + 1) ** 2 / (2.0 * sigma ** 2))
    sx, sy = SIDES[name]
    a = np.arange(-r, r + 1)
    mx = (a * sx >= 0) if sx else np.ones_like(a, bool)
    my = (a * sy >= 0) if sy else np.ones_like(a, bool)
    k = np.outer(g * my, g * mx)  # rows = b (y offset), columns = a (x offset)
    return k / k.sum()


@pytest.mark.parametrize("r", [1, 2, 5])
def test_infinite_sigma_is_the_box_filter(r):
    img = synth.voronoi(40, 37, 6, 0.05, np.random.default_rng(r))[0].astype(np.float64)
    for sigma in (np.inf, 1e9):
        g, gs = oracle.gauss_forward(img, r, sigma, 3, return_sel=True)
        b, bs = oracle.forward(img, r, 3, return_sel=True)
        assert np.array_equal(g, b) and np.array_equal(gs, bs)


@pytest.mark.parametrize("r,sigma", [(1, 0.7), (3, 2.0), (5, 2.5), (4, 0.9)])
def test_window_means_match_scipy_correlation(r, sigma):
    rng = np.random.default_rng(10 * r)
    img = rng.random((23, 31))
    out, sel, err, means = oracle.gauss_sweep(img, r, sigma)
    want = np.stack([ndimage.correlate(img, _kernel(n, r, sigma), mode="nearest") for n in ORDER], axis=-1)
    np.testing.assert_allclose(means, want, rtol=0, atol=1e-12)
    want_sel = np.argmin(np.abs(want - img[..., None]), axis=-1)
    assert np.array_equal(sel, want_sel)
    np.testing.assert_allclose(out, np.take_along_axis(want, want_sel[..., None], -1)[..., 0], rtol=0, atol=1e-12)


@pytest.mark.parametrize("r,sigma", [(1, 0.6), (3, 1.7), (5, 4.0)])
def test_exact_quadrant_tie_goes_to_se(r, sigma):
    """A single spike: at the spike the four quadrant means are equal (each
    holds the spike once with weight g(0)^2 over Zh^2) and closer to it than
    the halves, so the first quadrant in the order, SE, is taken."""
    img = np.zeros((2 * r + 5, 2 * r + 7))
    cy, cx = r + 2, r + 3
    img[cy, cx] = 1.0
    out, sel, _, means = oracle.gauss_sweep(img, r, sigma)
    assert len(set(means[cy, cx, 4:].tolist())) == 1
    assert sel[cy, cx] == ORDER.index("SE")
    zh = np.exp(-np.arange(r + 1) ** 2 / (2.0 * sigma ** 2)).sum()
    assert out[cy, cx] == pytest.approx(1.0 / zh ** 2, rel=1e-14)


def test_small_sigma_is_the_identity():
    img = np.random.default_rng(3).random((17, 19))
    np.testing.assert_allclose(oracle.gauss_forward(img, 3, 0.04, 2), img, rtol=0, atol=1e-12)


@pytest.mark.parametrize("angle", [0.0, 0.6, 1.3, 2.2])
def test_step_edges_are_fixed_points(angle):
    """A straight edge between two levels: the quadrant facing away from the
    edge normal lies on the pixel's side, so its mean is the pixel's level."""
    H, W = 24, 27
    y, x = np.mgrid[0:H, 0:W]
    img = np.where(np.cos(angle) * (x - 13.3) + np.sin(angle) * (y - 11.7) < 0, 0.25, 0.75)
    for r, s in ((1, 0.8), (3, 1.5), (6, 3.0)):
        np.testing.assert_allclose(oracle.gauss_forward(img, r, s, 3), img, rtol=0, atol=1e-12)


@pytest.mark.parametrize("r,sigma,T", [(2, 1.0, 4), (5, 2.5, 2)])
def test_maximum_principle_and_identity(r, sigma, T):
    img = synth.voronoi(30, 33, 5, 0.05, np.random.default_rng(r))[0].astype(np.float64)
    out = oracle.gauss_forward(img, r, sigma, T)
    assert out.min() >= img.min() - 1e-15 and out.max() <= img.max() + 1e-15
    assert np.array_equal(oracle.gauss_forward(img, 0, sigma, T), img)
    assert np.array_equal(oracle.gauss_forward(img, r, sigma, 0), img)


def test_mirror_symmetry():
    """Flipping columns flips the output and swaps R<->L, SE<->SW, NE<->NW."""
    img = np.random.default_rng(8).random((19, 22))
    out, sel, _, _ = oracle.gauss_sweep(img, 3, 1.4)
    out_f, sel_f, _, _ = oracle.gauss_sweep(img[:, ::-1].copy(), 3, 1.4)
    np.testing.assert_allclose(out_f[:, ::-1], out, rtol=0, atol=1e-12)
    swap = np.array([1, 0, 2, 3, 5, 4, 7, 6])
    assert np.array_equal(swap[sel], sel_f[:, ::-1])
