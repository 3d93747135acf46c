"""CPU-side checks of the C ABI: the library loads, exports every function that
include/*.h declares, and rejects bad arguments before touching the device."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2108_05021_amd", "libosbf.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(osbf_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libosbf.so is not built (run python -m paper_2108_05021_amd.build)")
    from paper_2108_05021_amd import osbf
    return osbf.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "osbf_forward" in names
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for n in names:
        getattr(lib, n)  # resolvable through ctypes too


def test_version_and_status_strings(lib):
    assert lib.osbf_abi_version() == 2
    for s in range(6):
        assert lib.osbf_status_string(s)
    assert lib.osbf_status_string(99) == b"unknown status"


def test_workspace_size(lib):
    from paper_2108_05021_amd import osbf
    import torch
    assert osbf.forward_workspace_size(3, 64, 80, torch.float32, 2, 5) == 3 * 64 * 80 * 4
    assert osbf.forward_workspace_size(3, 64, 80, torch.bfloat16, 2, 5) == 3 * 64 * 80 * 2
    assert osbf.forward_workspace_size(3, 64, 80, torch.float32, 0, 5) == 0
    assert osbf.forward_workspace_size(3, 64, 80, torch.float32, 2, 0) == 0
    bad = ctypes.c_size_t(-1).value
    assert lib.osbf_forward_workspace_size(0, 64, 80, 0, 2, 5) == bad
    assert lib.osbf_forward_workspace_size(1, 64, 80, 7, 2, 5) == bad
    assert lib.osbf_forward_workspace_size(1, 64, 80, 0, 33, 5) == bad
    assert lib.osbf_forward_workspace_size(1, 64, 80, 0, 2, -1) == bad


@pytest.mark.parametrize("args,status", [
    ((1, 0, 8, 0, 1, 1, 0), 1),     # H = 0
    ((0, 8, 8, 0, 1, 1, 0), 1),     # planes = 0
    ((1, 8, 8, 3, 1, 1, 0), 1),     # bad dtype
    ((1, 8, 8, 0, -1, 1, 0), 1),    # r < 0
    ((1, 8, 8, 0, 33, 1, 0), 1),    # r > max
    ((1, 8, 8, 0, 1, -2, 0), 1),    # T < 0
    ((1, 8, 8, 0, 1, 1, 4), 1),     # bad boundary
])
def test_forward_rejects_bad_arguments(lib, args, status):
    planes, H, W, dt, r, T, b = args
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    rc = lib.osbf_forward(fake, fake, planes, H, W, dt, r, T, b, None, None, 0, None, 0, None)
    assert rc == status
    assert lib.osbf_last_error()


def test_forward_rejects_null_pointers_and_bad_checkpoint(lib):
    fake = ctypes.c_void_p(0x1000)
    assert lib.osbf_forward(None, fake, 1, 8, 8, 0, 1, 1, 0, None, None, 0, None, 0, None) == 1
    assert lib.osbf_forward(fake, None, 1, 8, 8, 0, 1, 1, 0, None, None, 0, None, 0, None) == 1
    assert lib.osbf_forward(fake, fake, 1, 8, 8, 0, 1, 1, 0, None, fake, 0, None, 0, None) == 1


def test_gpu_code_object_targets_gfx950():
    out = subprocess.run(["strings", LIB], capture_output=True, text=True).stdout
    assert "gfx950" in out


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of osbf_image / osbf_batch match the C header."""
    from paper_2108_05021_amd import osbf
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "osbf.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(osbf_image), sizeof(osbf_batch),'
        ' offsetof(osbf_batch, max_items), offsetof(osbf_batch, ws), offsetof(osbf_batch, identity),'
        ' offsetof(osbf_image, radius), offsetof(osbf_image, dst_row_stride));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(osbf.Image), ctypes.sizeof(osbf.Batch), osbf.Batch.max_items.offset,
            osbf.Batch.ws.offset, osbf.Batch.identity.offset, osbf.Image.radius.offset,
            osbf.Image.dst_row_stride.offset]
    assert got == want


def test_batched_rejects_bad_lists(lib):
    from paper_2108_05021_amd import osbf
    fake = ctypes.c_void_p(0x1000)
    imgs = (osbf.Image * 1)(osbf.Image(fake, ctypes.c_void_p(0x2000), 1, 8, 8, 33, 2))
    assert lib.osbf_batched(imgs, 1, 0, 0, None, 0, None) == 1          # radius above the limit
    imgs[0].radius = 6                                                  # no batched kernel: single-image path
    assert lib.osbf_batched(imgs, 1, 0, 0, None, 0, None) == 3          # workspace missing
    imgs[0].src_row_stride = 9
    assert lib.osbf_batched(imgs, 1, 0, 0, None, 0, None) == 2          # that path needs contiguous planes
    imgs[0].src_row_stride = 0
    imgs[0].radius = 2
    imgs[0].dst = fake
    assert lib.osbf_batched(imgs, 1, 0, 0, None, 0, None) == 1          # in place
    imgs[0].dst = ctypes.c_void_p(0x2000)
    imgs[0].height = 0
    assert lib.osbf_batched(imgs, 1, 0, 0, None, 0, None) == 1          # empty plane
    imgs[0].height = 8
    assert lib.osbf_batched(imgs, 1, 0, 0, None, 0, None) == 3          # workspace missing
    # strides: rows at least a row long, planes at least height rows apart
    imgs[0].planes = 2
    for field, value in (("src_row_stride", 7), ("dst_row_stride", -8), ("src_plane_stride", 63),
                         ("dst_plane_stride", -1)):
        setattr(imgs[0], field, value)
        assert lib.osbf_batched(imgs, 1, 0, 0, None, 0, None) == 1, field
        setattr(imgs[0], field, 0)
    imgs[0].src_row_stride, imgs[0].src_plane_stride = 10, 80
    imgs[0].dst_row_stride, imgs[0].dst_plane_stride = 8, 64
    assert lib.osbf_batched(imgs, 1, 0, 0, None, 0, None) == 3          # valid strides: workspace missing
    imgs[0].src_row_stride = 1 << 28                                    # rows beyond 32-bit offsets
    imgs[0].src_plane_stride = 0
    assert lib.osbf_batched(imgs, 1, 0, 0, None, 0, None) == 2


def test_volume_entry_validation(lib):
    """osbf3d_forward checks its arguments before touching the device."""
    bad = ctypes.c_size_t(-1).value
    assert lib.osbf3d_forward_workspace_size(2, 8, 9, 10, 3, 4) == 2 * 8 * 9 * 10 * 4
    assert lib.osbf3d_forward_workspace_size(2, 8, 9, 10, 0, 4) == 0
    assert lib.osbf3d_forward_workspace_size(2, 8, 9, 10, 3, 0) == 0
    assert lib.osbf3d_forward_workspace_size(0, 8, 9, 10, 3, 4) == bad
    assert lib.osbf3d_forward_workspace_size(1, 8, 9, 10, 5, 4) == bad
    fake = ctypes.c_void_p(0x1000)
    f = lib.osbf3d_forward
    assert f(fake, fake, 0, 8, 8, 8, 2, 1, None, None, 0, None) == 1      # no volume
    assert f(fake, fake, 1, 8, 0, 8, 2, 1, None, None, 0, None) == 1      # empty slice
    assert f(fake, fake, 1, 8, 8, 8, -1, 1, None, None, 0, None) == 1     # negative radius
    assert f(fake, fake, 1, 8, 8, 8, 5, 1, None, None, 0, None) == 2      # radius without kernel
    assert f(fake, fake, 1, 8, 8, 8, 2, -1, None, None, 0, None) == 1     # negative T
    assert f(None, fake, 1, 8, 8, 8, 2, 1, None, None, 0, None) == 1      # null source
    assert f(fake, ctypes.c_void_p(0x2000), 1, 8, 8, 8, 2, 2, None, None, 0, None) == 3  # ping-pong needs ws
    assert f(fake, fake, 1, 8, 8, 8, 2, 1, None, None, 0, None) == 3      # in place needs ws
    assert lib.osbf_last_error()


def test_gaussian_entry_validation(lib):
    """osbf_gaussian_forward checks its arguments before touching the device."""
    bad = ctypes.c_size_t(-1).value
    assert lib.osbf_gaussian_workspace_size(2, 9, 10, 3, 4) == 2 * 9 * 10 * 4
    assert lib.osbf_gaussian_workspace_size(2, 9, 10, 0, 4) == 0
    assert lib.osbf_gaussian_workspace_size(2, 9, 10, 9, 4) == bad
    fake = ctypes.c_void_p(0x1000)
    f = lib.osbf_gaussian_forward
    assert f(fake, fake, 1, 8, 8, 9, 1.0, 1, None, None, 0, None) == 2        # radius without kernel
    assert f(fake, fake, 1, 8, 8, 2, 0.0, 1, None, None, 0, None) == 1        # sigma <= 0
    assert f(fake, fake, 1, 8, 8, 2, float("nan"), 1, None, None, 0, None) == 1
    assert f(fake, fake, 0, 8, 8, 2, 1.0, 1, None, None, 0, None) == 1        # no plane
    assert f(fake, ctypes.c_void_p(0x2000), 1, 8, 8, 2, 1.0, 2, None, None, 0, None) == 3  # needs ws
    assert lib.osbf_last_error()


def test_autotune_entry_validation(lib):
    """osbf_autotune checks its arguments before touching the device."""
    fake, other = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    out = [ctypes.c_int32(7) for _ in range(3)]
    refs = [ctypes.byref(v) for v in out]
    assert lib.osbf_autotune(fake, fake, 1, 8, 8, 0, 2, 3, None, *refs) == 1        # in place
    assert lib.osbf_autotune(None, other, 1, 8, 8, 0, 2, 3, None, *refs) == 1       # null source
    assert lib.osbf_autotune(fake, other, 0, 8, 8, 0, 2, 3, None, *refs) == 1       # no plane
    assert lib.osbf_autotune(fake, other, 1, 8, 8, 9, 2, 3, None, *refs) == 1       # bad dtype
    assert lib.osbf_autotune(fake, other, 1, 8, 8, 0, 2, 3, None, None, None, None) == 1
    assert lib.osbf_autotune(fake, other, 1, 8, 8, 0, 0, 3, None, *refs) == 0       # r = 0: nothing to tune
    assert [v.value for v in out] == [0, 0, 0]
    lib.osbf_autotune_clear()
