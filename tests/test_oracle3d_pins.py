"""Pins of the FP64 volume oracle (Sec. "Higher Dimension Case") to facts that
do not come from the oracle itself: exact-rational brute force, exact integer
selection, reduction to the planar filter (plus the full box) on volumes that
are constant along one axis, planar-edge fixed points, the maximum principle,
axis-permutation symmetry and the identity cases."""
import zlib

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2108_05021_amd import synth

PLANAR = ("R", "L", "D", "U", "SE", "SW", "NE", "NW")


def _sides(w):
    """(sx, sy, sz) of volume window w: +1 / -1 one-sided, 0 full."""
    return exact.SIDES3[w]


@pytest.mark.parametrize("shape,r,T,kind", [((3, 4, 5), 1, 2, "int"), ((4, 3, 4), 2, 1, "int"),
                                            ((2, 5, 3), 1, 1, "float"), ((5, 2, 2), 2, 2, "float"),
                                            ((1, 3, 4), 1, 2, "int"), ((3, 3, 3), 3, 1, "int")])
def test_exact_rational_brute_force(shape, r, T, kind):
    rng = np.random.default_rng(zlib.crc32(repr((shape, r, T, kind)).encode()))
    if kind == "int":
        vol = rng.integers(0, 4, size=shape).astype(np.float64)  # many exact ties
    else:
        vol = rng.random(shape)
    want, sels = exact.forward3(vol.tolist(), r, T)
    got, gsel = oracle.forward3d(vol, r, T, return_sel=True)
    np.testing.assert_allclose(got, np.array(want, dtype=np.float64), rtol=0, atol=1e-12)
    assert np.array_equal(gsel[:, 0], np.array(sels, dtype=np.uint8))


@pytest.mark.parametrize("r", [1, 2, 3])
def test_integer_selection_is_exact(r):
    rng = np.random.default_rng(40 + r)
    vol = rng.integers(0, 256, size=(6, 9, 11))
    sel_i, _ = oracle.select_int64_3d(vol, r)
    _, sel_f, _ = oracle.sweep3d(vol.astype(np.float64), r)
    assert np.array_equal(sel_i, sel_f)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("r", [1, 2])
def test_reduces_to_planar_filter_plus_box(axis, r):
    """A volume constant along one axis: each window's mean is the planar mean
    of its extent in the two other axes (halves along the constant axis give
    the full (2r+1)^2 box), so the volume filter picks, in its own order, among
    the planar oracle's eight means and the planar box mean."""
    rng = np.random.default_rng(70 + axis + 10 * r)
    n = (5, 7, 6)  # extents along z, y, x
    other = [a for a in (0, 1, 2) if a != axis]  # (slow, fast) axes of the plane, in z,y,x order
    img = rng.random((n[other[0]], n[other[1]]))
    vol = np.expand_dims(img, axis).repeat(n[axis], axis=axis)
    _, _, _, m2 = oracle.sweep(img, r, return_means=True)
    box = oracle.box_forward(img, r, 1)
    # volume axes in window side order (x, y, z) are array axes (2, 1, 0);
    # the plane's x is its fast axis, its y the slow one
    side_axis = {2: 0, 1: 1, 0: 2}
    cand = []
    for w in range(14):
        s = _sides(w)
        sx, sy = s[side_axis[other[1]]], s[side_axis[other[0]]]
        if sx == 0 and sy == 0:
            cand.append(box)
        elif sy == 0:
            cand.append(m2[..., PLANAR.index("R" if sx > 0 else "L")])
        elif sx == 0:
            cand.append(m2[..., PLANAR.index("D" if sy > 0 else "U")])
        else:
            name = ("S" if sy > 0 else "N") + ("E" if sx > 0 else "W")
            cand.append(m2[..., PLANAR.index(name)])
    cand = np.stack(cand, axis=-1)
    want_sel = np.argmin(np.abs(cand - img[..., None]), axis=-1)  # first minimum
    want = np.take_along_axis(cand, want_sel[..., None], axis=-1)[..., 0]
    got, sel, _ = oracle.sweep3d(vol, r)
    np.testing.assert_allclose(got, np.expand_dims(want, axis).repeat(n[axis], axis=axis), rtol=0, atol=1e-12)
    assert np.array_equal(sel, np.expand_dims(want_sel, axis).repeat(n[axis], axis=axis))


@pytest.mark.parametrize("seed", range(4))
def test_planar_edges_are_fixed_points(seed):
    """Two dyadic levels split by any plane: the octant facing away from the
    plane's normal (clamped into the volume) stays on the voxel's side, so
    every voxel has a window at distance 0 and keeps its value, bit-exact."""
    rng = np.random.default_rng(seed)
    D, H, W = 7, 9, 8
    nrm = rng.normal(size=3)
    z, y, x = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    p0 = rng.uniform([0, 0, 0], [W, H, D])  # a point of the plane, inside the volume
    side = nrm[0] * x + nrm[1] * y + nrm[2] * z < nrm @ p0
    a, b = rng.integers(0, 64, size=2) / 64.0
    vol = np.where(side, a, b)
    for r in (1, 2, 3):
        out = oracle.forward3d(vol, r, 3)
        assert np.array_equal(out, vol)


@pytest.mark.parametrize("r,T", [(1, 3), (2, 2), (4, 1)])
def test_constant_and_maximum_principle(r, T):
    vol = np.full((4, 6, 5), 0.375)
    assert np.array_equal(oracle.forward3d(vol, r, T), vol)
    rng = np.random.default_rng(r)
    v = synth.voronoi3d(6, 8, 7, 5, 0.05, rng).astype(np.float64)
    out = oracle.forward3d(v, r, T)
    assert out.min() >= v.min() and out.max() <= v.max()


def test_identity_cases():
    v = np.random.default_rng(1).random((3, 4, 5))
    assert np.array_equal(oracle.forward3d(v, 0, 3), v)
    assert np.array_equal(oracle.forward3d(v, 2, 0), v)


def test_axis_swap_symmetry():
    """Swapping the x and y axes of the input swaps them in the output, and
    each selected window maps to its mirror (+x <-> +y, octant (sx,sy,sz) ->
    (sy,sx,sz)) on tie-free data."""
    rng = np.random.default_rng(5)
    v = rng.random((5, 6, 7))
    out, sel, _ = oracle.sweep3d(v, 2)
    out_t, sel_t, _ = oracle.sweep3d(v.transpose(0, 2, 1).copy(), 2)
    np.testing.assert_allclose(out_t.transpose(0, 2, 1), out, rtol=0, atol=1e-12)
    mirror = []
    for w in range(14):
        sx, sy, sz = _sides(w)
        mirror.append(exact.SIDES3.index((sy, sx, sz)))
    assert np.array_equal(np.array(mirror)[sel], sel_t.transpose(0, 2, 1))


def test_window_sizes_and_centre():
    """Every window contains its centre voxel; halves hold (r+1)(2r+1)^2
    voxels, octants (r+1)^3, and the 14 windows are distinct."""
    for r in (1, 2, 3):
        seen = set()
        for w in range(14):
            e = oracle.window_extent3(w, 10, 20, 30, r)
            assert e[0] <= 10 <= e[1] and e[2] <= 20 <= e[3] and e[4] <= 30 <= e[5]
            size = (e[1] - e[0] + 1) * (e[3] - e[2] + 1) * (e[5] - e[4] + 1)
            assert size == ((r + 1) * (2 * r + 1) ** 2 if w < 6 else (r + 1) ** 3)
            seen.add(e)
        assert len(seen) == 14
