"""CPU checks of the region checkers in parity.py: the oracle's own
trajectory replays with no outlier, on the whole plane and on a region cut
out of it (only the dependency cones inside the region are compared), and a
planted error in the checked values or maps is caught."""
import numpy as np
import pytest

import oracle
from paper_2108_05021_amd import synth

import parity


@pytest.mark.parametrize("r,T", [(1, 4), (2, 3), (3, 2)])
def test_replay_of_oracle_maps_has_no_outlier(r, T):
    rng = np.random.default_rng(60 + r)
    u0 = synth.voronoi(70, 66, 8, 0.05, rng)[0].astype(np.float64)
    out, sel = oracle.forward(u0, r, T, return_sel=True)
    n_bad, dev, flips, px = parity.replay_region(u0, out, sel[:, 0], r, (False,) * 4)
    assert n_bad == 0 and dev < 1e-12 and flips == 0 and px == u0.size
    # a region cut out of the plane: interior cones only
    reg = (slice(11, 59), slice(7, 52))
    n_bad, dev, flips, px = parity.replay_region(u0[reg], out[reg], sel[:, 0][(slice(None),) + reg], r,
                                                 (True,) * 4)
    assert n_bad == 0 and dev < 1e-12 and flips == 0
    assert px == (48 - 2 * r * T) * (45 - 2 * r * T)


def test_replay_catches_planted_errors():
    rng = np.random.default_rng(70)
    r, T = 2, 3
    u0 = synth.voronoi(50, 50, 6, 0.05, rng)[0].astype(np.float64)
    out, sel = oracle.forward(u0, r, T, return_sel=True)
    bad_out = out.copy()
    bad_out[25, 25] += 1e-3
    assert parity.replay_region(u0, bad_out, sel[:, 0], r, (False,) * 4)[0] == 1
    # a map whose window is far from minimal at one pixel
    s = sel[:, 0].copy()
    _, _, err = oracle.sweep(u0, r)
    y, x = np.unravel_index(np.argmax(err.max(axis=2) - err.min(axis=2)), err.shape[:2])
    s[0, y, x] = int(np.argmax(err[y, x]))
    assert parity.replay_region(u0, out, s, r, (False,) * 4)[0] >= 1


def test_sweep_region_matches_and_catches():
    rng = np.random.default_rng(71)
    r = 3
    u = synth.voronoi(60, 61, 7, 0.05, rng)[0].astype(np.float64)
    nxt, sel, _ = oracle.sweep(u, r)
    reg = (slice(5, 40), slice(9, 50))
    flips, px, dev = parity.sweep_region(u[reg], nxt[reg], sel[reg], r, (True, True, True, True))
    assert flips == 0 and px == (35 - 2 * r) * (41 - 2 * r) and dev < 1e-12
    wrong = nxt.copy()
    wrong[20, 20] += 1e-3
    with pytest.raises(AssertionError):
        parity.sweep_region(u[reg], wrong[reg], sel[reg], r, (True,) * 4)


def test_untethered_check_cones():
    """untethered_check: the oracle's own run passes with no cone; a run that
    took another window at one pixel and sweep (a planted flip, carried on
    through the fixed-selection map) passes with the difference confined to
    that pixel's cone; an error planted outside every cone is caught."""
    rng = np.random.default_rng(80)
    r, T = 2, 4
    u0 = synth.voronoi(40, 46, 6, 0.05, rng)[0].astype(np.float64)
    out, sel = oracle.forward(u0, r, T, return_sel=True)
    outside, frac, _ = parity.untethered_check(u0, out, sel, r)
    assert outside == 0.0 and frac == 0.0
    # plant a flip at sweep 1, pixel (20, 23): a different window there, the
    # oracle's own choices elsewhere and later (recomputed on the new iterate)
    u = oracle.forward(u0, r, 1)
    s1 = oracle.sweep(u, r)[1].copy()
    s1[20, 23] = (s1[20, 23] + 3) % 8
    u = oracle.apply_fixed(u, s1, r)
    u, rest = oracle.forward(u, r, T - 2, return_sel=True)
    sels = np.concatenate([sel[:1, 0], s1[None], rest[:, 0]])
    outside, frac, worst = parity.untethered_check(u0, u, sels, r)
    assert worst > 1e-5                     # the flip changed values ...
    side = 2 * r * (T - 2) + 1              # ... only inside its cone
    assert frac <= side * side / u0.size + 1e-12
    bad = u.copy()
    bad[2, 2] += 1e-3                       # far from (20, 23)
    with pytest.raises(AssertionError, match="outside the flip cones"):
        parity.untethered_check(u0, bad, sels, r)
