"""Host-side argument checks of the Python binding (no device needed: every
case is rejected before the C ABI is called)."""
import pytest
import torch

from paper_2108_05021_amd import osbf


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16, torch.float64])
@pytest.mark.parametrize("ck", [0, 2])
def test_autograd_rejects_non_fp32(dtype, ck):
    x = torch.zeros(1, 8, 8, dtype=dtype, requires_grad=dtype.is_floating_point)
    with pytest.raises(TypeError, match="float32"):
        osbf.osbf(x, 1, 3, ckpt_every=ck)


def test_backward_rejects_wrong_dtypes():
    g = torch.zeros(1, 8, 8)
    with pytest.raises(TypeError, match="ckpt"):
        osbf.osbf_backward(g, torch.empty_like(g), 1, 2, ckpt=torch.zeros(1, 1, 8, 8, dtype=torch.bfloat16), ck=2)
    with pytest.raises(TypeError, match="sel"):
        osbf.osbf_backward(g, torch.empty_like(g), 1, 2, sel=torch.zeros(2, 1, 8, 8, dtype=torch.int32))
    with pytest.raises(TypeError, match="grad_out"):
        osbf.osbf_backward(g.half(), torch.empty_like(g), 1, 2, sel=torch.zeros(2, 1, 8, 8, dtype=torch.uint8))


def test_batch_rejects_mixed_dtypes_shapes_and_lengths():
    a = torch.zeros(1, 16, 16)
    b = torch.zeros(1, 16, 16, dtype=torch.float16)
    with pytest.raises(ValueError, match="dtype"):
        osbf.batched([a, b], [1, 1], [2, 2])
    with pytest.raises(ValueError, match="dtype"):
        osbf.BatchPlan([a, a], [1, 1], [2, 2], outs=[torch.empty_like(a), torch.empty_like(b)])
    with pytest.raises(ValueError, match="shape"):
        osbf.batched([a, a], [1, 1], [2, 2], outs=[torch.empty_like(a), torch.zeros(1, 16, 17)])
    with pytest.raises(ValueError, match="length"):
        osbf.batched([a, a], [1], [2, 2])
    with pytest.raises(ValueError, match="length"):
        osbf.BatchPlan([a, a], [1, 1], [2])


def test_strided_geometry_of_views():
    """Batch images may be views: rows must have unit stride and the leading
    dimensions must collapse into one plane index with a uniform stride."""
    big = torch.zeros(2, 4, 40, 50)
    assert osbf._strided_geometry(big) == (8, 40, 50, 2000, 50)
    assert osbf._strided_geometry(big[:, :, 3:30, 7:44]) == (8, 27, 37, 2000, 50)
    assert osbf._strided_geometry(big[1, 2, 5:9, :]) == (1, 4, 50, 0, 50)
    assert osbf._strided_geometry(big[0, 0, 5:6, 3:9]) == (1, 1, 6, 0, 0)
    with pytest.raises(ValueError, match="collapse"):
        osbf._strided_geometry(big[:, 1:3])              # channel slice: planes not uniformly spaced
    with pytest.raises(ValueError, match="unit stride"):
        osbf._strided_geometry(big.transpose(-1, -2))    # columns strided
    with pytest.raises(ValueError, match="rows overlap"):
        osbf._strided_geometry(torch.zeros(1, 50).expand(40, 50))          # one row seen 40 times
    with pytest.raises(ValueError, match="planes overlap"):
        osbf._strided_geometry(torch.zeros(1, 40, 50).expand(3, 40, 50))  # one plane seen 3 times
    # a batch of such views is marshalled with each side's strides
    x = big[:, :, 3:30, 7:44]
    y = torch.zeros(2, 4, 27, 37)
    img = osbf._images([x], [y], [2], [3])[0]
    assert (img.planes, img.height, img.width) == (8, 27, 37)
    assert (img.src_plane_stride, img.src_row_stride, img.dst_plane_stride, img.dst_row_stride) == (2000, 50, 999, 37)
