"""The classical box filter kernel (the paper's timing baseline, Table I)
against the FP64 oracle's box filter: every compiled radius, ragged and
one-pixel shapes, images taller than one chunk, several sweeps, in place,
and 16-bit storage (each sweep within half a storage ulp of the oracle run
on the GPU's own input)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_05021_amd import osbf, synth

RADII = [1, 2, 3, 4, 5, 8, 10, 16]


@pytest.mark.gpu
@pytest.mark.parametrize("r", RADII)
@pytest.mark.parametrize("shape", [(2, 97, 301), (1, 1, 1), (1, 1, 77), (1, 77, 1), (1, 2500, 131)])
def test_box_kernel_matches_oracle(dev, r, shape):
    rng = np.random.default_rng(1300 + r + shape[1])
    img = synth.voronoi(shape[1], shape[2], 9, 0.05, rng, C=shape[0])
    x = torch.from_numpy(img).to(dev)
    for T in (1, 3):
        y = osbf.box_forward(x, r, T).cpu().numpy()
        want = oracle.box_forward(img.astype(np.float64), r, T)
        np.testing.assert_allclose(y, want, rtol=0, atol=2e-6, err_msg=f"r={r} T={T} {shape}")
    z = x.clone()
    osbf.box_forward(z, r, 3, out=z)
    assert torch.equal(z, osbf.box_forward(x, r, 3))
    assert torch.equal(osbf.box_forward(x, r, 0), x)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("r", [2, 5, 16])
def test_box_kernel_reduced_precision(dev, dtype, r):
    rng = np.random.default_rng(1400 + r)
    x = torch.from_numpy(synth.voronoi(260, 333, 9, 0.05, rng, C=2)).to(dev).to(dtype)
    cur = x
    for _ in range(3):
        nxt = osbf.box_forward(cur, r, 1)
        want = oracle.box_forward(cur.float().cpu().numpy().astype(np.float64), r, 1)
        got = nxt.float().cpu().numpy()
        # half an ulp of the storage type at the value's binade (mantissa
        # 7 bits for BF16, 10 for FP16), plus the FP32 sum's rounding
        step = 2.0 ** -7 if dtype == torch.bfloat16 else 2.0 ** -10
        binade = 2.0 ** np.floor(np.log2(np.maximum(np.abs(want), 2.0 ** -14)))
        assert (np.abs(got - want) <= 0.5 * step * binade + 2e-6).all(), (r, float(np.abs(got - want).max()))
        cur = nxt
