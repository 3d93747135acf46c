"""The autotuner (osbf_autotune): it measures launch plans on the device and
caches the fastest per (device, radius, dtype, size class).  Every plan
computes the same bits, so tuning may change the plan but never the result."""
import numpy as np
import pytest
import torch

from paper_2108_05021_amd import osbf, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("r,T", [(3, 6), (2, 1), (7, 4), (10, 2)])
def test_autotune_changes_plan_not_bits(dev, r, T):
    x = torch.from_numpy(synth.voronoi(300, 500, 12, 0.05, np.random.default_rng(r), C=3)).to(dev)
    osbf.autotune_clear()
    base_plan = osbf.forward_plan(3, 300, 500, torch.float32, r, T)
    y0, s0 = osbf.forward(x, r, T, return_sel=True)
    tuned = osbf.autotune(x, r, T)
    assert tuned["fused"] >= 1 and tuned["fused"] <= T
    p = osbf.forward_plan(3, 300, 500, torch.float32, r, T)
    assert p["tile"] == tuned["tile"] and p["fused"] == tuned["fused"]
    y1, s1 = osbf.forward(x, r, T, return_sel=True)
    assert torch.equal(y0, y1) and torch.equal(s0, s1)
    # checkpoint recompute under the tuned plan reproduces the stored maps
    w = torch.randn_like(x)
    _, ck = osbf.forward(x, r, T, ckpt_every=2)
    assert torch.equal(osbf.backward(w, r, T, ckpt=ck, ck=2), osbf.backward(w, r, T, sel=s0))
    osbf.autotune_clear()
    assert osbf.forward_plan(3, 300, 500, torch.float32, r, T) == base_plan


def test_autotune_is_per_dtype_and_size_class(dev):
    osbf.autotune_clear()
    big = torch.rand(1, 1024, 1100, device=dev)
    small = torch.rand(1, 100, 90, device=dev)
    t_big = osbf.autotune(big, 5, 30)
    assert osbf.forward_plan(1, 1024, 1100, torch.float32, 5, 30)["tile"] == t_big["tile"]
    # another size class and another dtype keep the untuned plans
    osbf.autotune_clear()
    ref_small = osbf.forward_plan(1, 100, 90, torch.float32, 5, 30)
    ref_bf16 = osbf.forward_plan(1, 1024, 1100, torch.bfloat16, 5, 30)
    osbf.autotune(big, 5, 30)
    assert osbf.forward_plan(1, 100, 90, torch.float32, 5, 30) == ref_small
    assert osbf.forward_plan(1, 1024, 1100, torch.bfloat16, 5, 30) == ref_bf16
    osbf.autotune(small, 5, 30)
    osbf.autotune_clear()


def test_autotune_identity_cases(dev):
    x = torch.rand(1, 20, 30, device=dev)
    assert osbf.autotune(x, 0, 5) == {"tile": (0, 0), "fused": 0}
    assert osbf.autotune(x, 2, 0) == {"tile": (0, 0), "fused": 0}


def test_batched_after_autotune_equals_single(dev):
    """Batched images take the fusion depth of a tuned plan on their class
    when it uses the batch's region; the results stay the per-image ones."""
    rng = np.random.default_rng(9)
    xs = [torch.from_numpy(synth.voronoi(h, w, 8, 0.05, rng, C=c)).to(dev)
          for h, w, c in ((300, 420, 1), (1100, 1000, 1), (64, 900, 3))]
    rs, ts = [2, 3, 1], [7, 5, 9]
    osbf.autotune_clear()
    for x, r, t in zip(xs, rs, ts):
        osbf.autotune(x, r, t)
    ys = osbf.batched(xs, rs, ts)
    for x, y, r, t in zip(xs, ys, rs, ts):
        assert torch.equal(y, osbf.forward(x, r, t))
    osbf.autotune_clear()
