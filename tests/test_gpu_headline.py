"""The benchmark's own run (3x2048x2048 FP32, r in {2, 5, 10}, T = 30, the
launch plans bench.py times) checked end to end on crops: the oracle replays
the GPU's 30 selection maps on a 32x32 crop grown by r*T (every selection
near-minimal, the final values equal to the replay), and the maps-writing
call gives the same output as the call bench.py times."""
import numpy as np
import pytest
import torch

import bench
import parity
from paper_2108_05021_amd import osbf, synth


@pytest.fixture(scope="module")
def image(dev):
    return torch.from_numpy(synth.workload_rgb()).to(dev)


@pytest.mark.gpu
@pytest.mark.parametrize("r", bench.RADII)
def test_headline_run_replays_on_crops(image, r):
    x = image
    C, H, W = x.shape
    T = bench.T_SWEEPS
    y, sels = osbf.forward(x, r, T, return_sel=True)
    assert torch.equal(y, osbf.forward(x, r, T))
    for (p, y0, x0) in [(1, 1008, 1008), (2, 2048 - 32, 0)]:
        (ya, yb, xa, xb), cuts = parity.region_of(H, W, y0, x0, 32, r * T)
        n_bad, dev, flips, px = parity.replay_region(
            x[p, ya:yb, xa:xb].cpu().numpy(), y[p, ya:yb, xa:xb].cpu().numpy(),
            sels[:, p, ya:yb, xa:xb].cpu().numpy(), r, cuts)
        assert n_bad == 0 and px >= 32 * 32, (r, p, y0, x0, n_bad, dev)
