"""Host-side checks of the launch-plan tables (osbf_forward_plan needs no
device): images below 2^17 and below 2^20 plane-pixels take the two
small-image tables (the tiled kernel with several fused sweeps per launch),
images up to 2^21 keep tiles at r = 1 and 2, larger ones take the
row-streaming plans (two fused sweeps per launch at r = 1, one above), and above 2^25 plane-pixels the two huge-image tables; fused sweeps never exceed T and the launch count covers T.  Every
plan gives the same bits (the GPU tests check that); this pins which one the
tables pick."""
import pytest
import torch

from paper_2108_05021_amd import osbf

TINY_K = {1: 8, 2: 6, 3: 6, 4: 4, 5: 4, 8: 2, 10: 2}   # below 2^17 plane-pixels
SMALL_K = {1: 6, 2: 5, 3: 3, 4: 2, 5: 2, 8: 1, 10: 1}  # 2^17 up to 2^20
SMALL_SHAPES = {(1, 256, 256): TINY_K, (1, 64, 64): TINY_K, (1, 128, 160): TINY_K, (1, 362, 362): TINY_K,
                (3, 512, 512): SMALL_K, (1, 1024, 1023): SMALL_K, (3, 300, 400): SMALL_K,
                (2, 256, 256): SMALL_K}


@pytest.mark.parametrize("shape", sorted(SMALL_SHAPES))
@pytest.mark.parametrize("r", sorted(SMALL_K))
def test_small_images_use_tiled_plans(shape, r):
    table = SMALL_SHAPES[shape]
    for T in (1, 3, 10, 30):
        p = osbf.forward_plan(*shape, torch.float32, r, T)
        assert p["tile"][1] > 0, (shape, r, T, p)   # tiled: explicit tile height
        assert p["fused"] == min(table[r], T), (shape, r, T, p)
        assert p["launches"] == -(-T // p["fused"])
        assert p["tile"][0] % r == 0 and p["tile"][1] % r == 0


# strip lanes of the large-image table (2^21 up to 2^25 plane-pixels)
LARGE_LANES = {1: 128, 2: 192, 3: 128, 4: 128, 5: 128, 8: 128, 10: 192, 16: 128}


@pytest.mark.parametrize("shape", [(1, 2048, 1024), (3, 2048, 2048), (1, 4096, 600), (2, 4096, 4096)])
@pytest.mark.parametrize("r", sorted(LARGE_LANES))
def test_large_images_use_streaming_plans(shape, r):
    for T in (1, 2, 30):
        p = osbf.forward_plan(*shape, torch.float32, r, T)
        assert p["tile"][1] == 0, (shape, r, T, p)  # streaming: rows chosen at launch
        # two fused sweeps per launch at r = 1 (never more than T), else one
        assert p["fused"] == (min(2, T) if r == 1 else 1), (shape, r, T, p)
        assert p["tile"][0] == (LARGE_LANES[r] - 2 * p["fused"] * r) // r * r, (shape, r, T, p)
        assert p["launches"] == -(-T // p["fused"])


@pytest.mark.parametrize("shape", [(1, 1024, 1024), (1, 1400, 1400), (1, 4096, 300)])
@pytest.mark.parametrize("r", sorted(LARGE_LANES))
def test_mid_images_keep_tiles_at_small_radii(shape, r):
    # 2^20 up to 2^21 plane-pixels: the tiled kernel (64x60 with 5 fused
    # sweeps at r = 1, 64x48 with 2 at r = 2), streaming plans from r = 3
    for T in (1, 3, 10):
        p = osbf.forward_plan(*shape, torch.float32, r, T)
        if r == 1:
            assert p["fused"] == min(5, T) and p["tile"][1] > 0, (shape, T, p)
            assert p["tile"] == (64 - 2 * p["fused"], 60 - 2 * p["fused"]), (shape, T, p)
        elif r == 2:
            assert p["fused"] == min(2, T) and p["tile"][1] > 0, (shape, T, p)
            assert p["tile"] == ((64 - 4 * p["fused"]) // 2 * 2, (48 - 4 * p["fused"]) // 2 * 2), (shape, T, p)
        else:
            assert p["tile"][1] == 0 and p["fused"] == 1, (shape, r, T, p)


# Above 2^25 plane-pixels: (strip width, fused sweeps, rows per workgroup)
# of the table for a ping-pong larger than the 256 MiB Infinity Cache (FP32;
# 16-bit above 2^26 pixels) and of the one for 16-bit storage within it.
DRAM = {1: (128, 2, 64), 2: (192, 2, 64), 3: (192, 2, 0), 4: (192, 2, 0), 5: (256, 1, 64),
        8: (192, 1, 0), 10: (192, 1, 0), 16: (128, 1, 0)}
HUGE16 = {1: (128, 1, 0), 2: (128, 1, 64), 3: (128, 1, 64), 4: (128, 1, 64), 5: (256, 1, 64),
          8: (192, 1, 0), 10: (192, 1, 0), 16: (128, 1, 0)}
CASES = [((1, 8192, 8192), torch.float32, DRAM), ((3, 4096, 4096), torch.float32, DRAM),
         ((3, 8192, 8192), torch.bfloat16, DRAM), ((1, 8192, 8192), torch.bfloat16, HUGE16),
         ((1, 8192, 8192), torch.float16, HUGE16), ((3, 4096, 4096), torch.float16, HUGE16)]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("r", sorted(DRAM))
def test_huge_images_use_their_tables(case, r):
    shape, dtype, table = CASES[case]
    lanes, k, rows = table[r]
    step = {1: 2, 2: 4, 16: 8}.get(r, r)
    for T in (1, 2, 10):
        p = osbf.forward_plan(*shape, dtype, r, T)
        assert p["fused"] == min(k, T), (shape, dtype, r, T, p)
        assert p["tile"][0] == (lanes - 2 * p["fused"] * r) // r * r, (shape, dtype, r, T, p)
        assert p["tile"][1] == -(-rows // step) * step, (shape, dtype, r, T, p)
        assert p["launches"] == -(-T // p["fused"])


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("r", sorted(DRAM))
def test_up_to_2_pow_25_pixels_is_a_large_image(dtype, r):
    # exactly 2^25 plane-pixels (an FP32 ping-pong of 256 MiB): the large-image table
    p = osbf.forward_plan(2, 4096, 4096, dtype, r, 10)
    assert p["fused"] == (2 if r == 1 else 1) and p["tile"][1] == 0, (dtype, r, p)


def test_plan_override_from_environment(monkeypatch):
    monkeypatch.setenv("OSBF_PLAN", "5,1,32")
    p = osbf.forward_plan(1, 256, 256, torch.float32, 2, 10)
    assert p == {"tile": (124, 32), "fused": 1, "launches": 10}   # 128 lanes - 2r, 32 rows
    monkeypatch.setenv("OSBF_PLAN", "1,4")
    p = osbf.forward_plan(3, 2048, 2048, torch.float32, 3, 10)
    # 64 x 48 region less 2kr of halo each way, rounded down to whole blocks of r
    assert p == {"tile": (39, 24), "fused": 4, "launches": 3}
