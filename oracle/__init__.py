"""CPU FP64 oracle of the one-sided box filter.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the GPU product path never imports it.  It shares
no code with the GPU path.

The arithmetic lives in ``osbf_oracle.c`` (plain direct window sums in double
precision, see its header for every reading of the paper); this module only
builds that file with gcc and marshals numpy arrays into it.  ``exact.py``
holds an exact-rational brute force for tiny inputs.

Window index order (= tie order): R, L, D, U, SE, SW, NE, NW.  The volume
filter (``osbf3d_oracle.c``) has 14 windows: +x, -x, +y, -y, +z, -z, then the
octants with x varying fastest and + before -.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "osbf_oracle.c")
_SRC3 = os.path.join(_HERE, "osbf3d_oracle.c")
_SRCG = os.path.join(_HERE, "osbf_gauss_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libosbf_oracle.so")

WINDOWS = ("R", "L", "D", "U", "SE", "SW", "NE", "NW")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP). Returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-o", tmp, _SRC, _SRC3, _SRCG, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
            os.path.getmtime(f) for f in (_SRC, _SRC3, _SRCG)):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    d = ctypes.POINTER(ctypes.c_double)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    i64 = ctypes.POINTER(ctypes.c_int64)
    ci = ctypes.c_int
    lib.oracle_sweep.argtypes = [d, d, u8, d, d, ci, ci, ci, ci]
    lib.oracle_sweep.restype = None
    lib.oracle_forward.argtypes = [d, d, u8, ci, ci, ci, ci, ci, ci]
    lib.oracle_forward.restype = ci
    lib.oracle_forward_padonce.argtypes = [d, d, ci, ci, ci, ci, ci]
    lib.oracle_forward_padonce.restype = ci
    lib.oracle_select_int64.argtypes = [i64, u8, i64, ci, ci, ci]
    lib.oracle_select_int64.restype = None
    lib.oracle_apply_fixed.argtypes = [d, u8, d, ci, ci, ci]
    lib.oracle_apply_fixed.restype = None
    lib.oracle_adjoint_scatter.argtypes = [d, u8, d, ci, ci, ci]
    lib.oracle_adjoint_scatter.restype = None
    lib.oracle_backward.argtypes = [d, d, d, u8, ci, ci, ci, ci, ci, ci]
    lib.oracle_backward.restype = ci
    lib.oracle_fast_sweep.argtypes = [d, d, u8, d, ci, ci, ci, ci]
    lib.oracle_fast_sweep.restype = None
    lib.oracle_fast_forward.argtypes = [d, d, ci, ci, ci, ci, ci, ci]
    lib.oracle_fast_forward.restype = ci
    lib.oracle_box_forward.argtypes = [d, d, ci, ci, ci, ci, ci]
    lib.oracle_box_forward.restype = ci
    lib.oracle_window_extent.argtypes = [ci, ci, ci, ci] + [ctypes.POINTER(ci)] * 4
    lib.oracle_window_extent.restype = None
    lib.oracle3d_window_extent.argtypes = [ci, ci, ci, ci, ci, ctypes.POINTER(ci)]
    lib.oracle3d_window_extent.restype = None
    lib.oracle3d_sweep.argtypes = [d, d, u8, d, d, ci, ci, ci, ci, ci]
    lib.oracle3d_sweep.restype = None
    lib.oracle3d_forward.argtypes = [d, d, u8, ci, ci, ci, ci, ci, ci, ci]
    lib.oracle3d_forward.restype = ci
    lib.oracle3d_select_int64.argtypes = [i64, u8, i64, ci, ci, ci, ci]
    lib.oracle3d_select_int64.restype = None
    cd = ctypes.c_double
    lib.oracle_gauss_sweep.argtypes = [d, d, u8, d, d, ci, ci, ci, cd, ci]
    lib.oracle_gauss_sweep.restype = None
    lib.oracle_gauss_forward.argtypes = [d, d, u8, ci, ci, ci, ci, cd, ci, ci]
    lib.oracle_gauss_forward.restype = ci
    _lib = lib
    return lib


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pu8(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _planes(x):
    """View an array of shape (H,W), (P,H,W) or (N,C,H,W) as (P,H,W) FP64."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    if a.ndim == 2:
        return a.reshape(1, *a.shape)
    return a.reshape(-1, a.shape[-2], a.shape[-1])


def window_extent(w: int, x: int, y: int, r: int):
    """Pixel set [x0,x1] x [y0,y1] of window ``w`` at (x, y)."""
    lib = _load()
    v = [ctypes.c_int() for _ in range(4)]
    lib.oracle_window_extent(w, x, y, r, *[ctypes.byref(t) for t in v])
    return tuple(t.value for t in v)


def forward(x, r: int, T: int, *, return_sel: bool = False, nthreads: int = 0):
    """T sweeps of Alg. 2 with the per-sweep replicate boundary.

    ``x`` is (H,W), (P,H,W) or (N,C,H,W); the result has the same shape, FP64.
    With ``return_sel`` also returns the selection maps, uint8 [T][P][H][W].
    """
    shape = np.shape(x)
    a = _planes(x)
    P, H, W = a.shape
    out = np.empty_like(a)
    sel = np.empty((T, P, H, W), np.uint8) if return_sel else None
    rc = _load().oracle_forward(_pd(a), _pd(out), _pu8(sel), P, H, W, r, T, nthreads)
    if rc != 0:
        raise ValueError("oracle_forward failed")
    out = out.reshape(shape)
    return (out, sel) if return_sel else out


def sweep(u, r: int, *, nthreads: int = 0, return_means: bool = False):
    """One sweep on one plane: returns (next, sel [H,W] uint8, err [H,W,8])
    where err holds the scaled distances |w_i S_i - N c|; with ``return_means``
    also the eight window means [H,W,8]."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    H, W = u.shape
    out = np.empty_like(u)
    sel = np.empty((H, W), np.uint8)
    err = np.empty((H, W, 8), np.float64)
    means = np.empty((H, W, 8), np.float64) if return_means else None
    _load().oracle_sweep(_pd(u), _pd(out), _pu8(sel), _pd(err),
                         None if means is None else _pd(means), H, W, r, nthreads)
    return (out, sel, err, means) if return_means else (out, sel, err)


def forward_padonce(x, r: int, T: int):
    """Pad-once reading of the appendix listing (zero beyond the padded frame)."""
    shape = np.shape(x)
    a = _planes(x)
    P, H, W = a.shape
    out = np.empty_like(a)
    if _load().oracle_forward_padonce(_pd(a), _pd(out), P, H, W, r, T) != 0:
        raise ValueError("oracle_forward_padonce failed")
    return out.reshape(shape)


def select_int64(x, r: int):
    """Exact integer selection for one sweep: (sel [H,W] uint8, sums [H,W,8] int64)."""
    a = np.ascontiguousarray(x, dtype=np.int64)
    H, W = a.shape
    sel = np.empty((H, W), np.uint8)
    sums = np.empty((H, W, 8), np.int64)
    _load().oracle_select_int64(a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _pu8(sel),
                                sums.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), H, W, r)
    return sel, sums


def apply_fixed(x, sel, r: int):
    """One sweep as a linear map with the selection map ``sel`` held fixed."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    sel = np.ascontiguousarray(sel, dtype=np.uint8)
    H, W = x.shape
    y = np.empty_like(x)
    _load().oracle_apply_fixed(_pd(x), _pu8(sel), _pd(y), H, W, r)
    return y


def adjoint(g_next, sel, r: int):
    """Transpose of :func:`apply_fixed` (scatter form)."""
    g_next = np.ascontiguousarray(g_next, dtype=np.float64)
    sel = np.ascontiguousarray(sel, dtype=np.uint8)
    H, W = g_next.shape
    g = np.empty_like(g_next)
    _load().oracle_adjoint_scatter(_pd(g_next), _pu8(sel), _pd(g), H, W, r)
    return g


def backward(x, grad_out, r: int, T: int, *, return_sel: bool = False, nthreads: int = 0):
    """Gradient of sum(grad_out * forward(x)) w.r.t. x, selections held fixed."""
    shape = np.shape(x)
    a = _planes(x)
    g = _planes(grad_out)
    P, H, W = a.shape
    gin = np.empty_like(a)
    sel = np.empty((T, P, H, W), np.uint8) if return_sel else None
    rc = _load().oracle_backward(_pd(a), _pd(g), _pd(gin), _pu8(sel), P, H, W, r, T, nthreads)
    if rc != 0:
        raise ValueError("oracle_backward failed")
    gin = gin.reshape(shape)
    return (gin, sel) if return_sel else gin


def fast_sweep(u, r: int, *, nthreads: int = 0):
    """One sweep of the fast approximation (Alg. 3) on one plane: returns
    (next, sel [H,W] uint8, candidates [H,W,8])."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    H, W = u.shape
    out = np.empty_like(u)
    sel = np.empty((H, W), np.uint8)
    cand = np.empty((H, W, 8), np.float64)
    _load().oracle_fast_sweep(_pd(u), _pd(out), _pu8(sel), _pd(cand), H, W, r, nthreads)
    return out, sel, cand


def fast_forward(x, r: int, T: int, *, nthreads: int = 0):
    """T sweeps of the fast approximation (Alg. 3), clamp boundary."""
    shape = np.shape(x)
    a = _planes(x)
    P, H, W = a.shape
    out = np.empty_like(a)
    if _load().oracle_fast_forward(_pd(a), _pd(out), P, H, W, r, T, nthreads) != 0:
        raise ValueError("oracle_fast_forward failed")
    return out.reshape(shape)


def box_forward(x, r: int, T: int):
    """T sweeps of the classical (2r+1)^2 box filter, clamp boundary."""
    shape = np.shape(x)
    a = _planes(x)
    P, H, W = a.shape
    out = np.empty_like(a)
    if _load().oracle_box_forward(_pd(a), _pd(out), P, H, W, r, T) != 0:
        raise ValueError("oracle_box_forward failed")
    return out.reshape(shape)


# ----------------------------------------------------------------- volumes

WINDOWS3 = ("+x", "-x", "+y", "-y", "+z", "-z",
            "+x+y+z", "-x+y+z", "+x-y+z", "-x-y+z", "+x+y-z", "-x+y-z", "+x-y-z", "-x-y-z")


def _volumes(x):
    """View an array of shape (D,H,W) or (V,D,H,W) as (V,D,H,W) FP64."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    if a.ndim == 3:
        return a.reshape(1, *a.shape)
    return a.reshape(-1, *a.shape[-3:])


def window_extent3(w: int, x: int, y: int, z: int, r: int):
    """Voxel set [x0,x1] x [y0,y1] x [z0,z1] of volume window ``w``."""
    e = (ctypes.c_int * 6)()
    _load().oracle3d_window_extent(w, x, y, z, r, e)
    return tuple(e)


def forward3d(x, r: int, T: int, *, return_sel: bool = False, nthreads: int = 0):
    """T sweeps of the volume filter (clamp boundary in x, y, z).  ``x`` is
    (D,H,W) or (V,D,H,W); with ``return_sel`` also the maps [T][V][D][H][W]."""
    shape = np.shape(x)
    a = _volumes(x)
    V, D, H, W = a.shape
    out = np.empty_like(a)
    sel = np.empty((T, V, D, H, W), np.uint8) if return_sel else None
    if _load().oracle3d_forward(_pd(a), _pd(out), _pu8(sel), V, D, H, W, r, T, nthreads) != 0:
        raise ValueError("oracle3d_forward failed")
    out = out.reshape(shape)
    return (out, sel) if return_sel else out


def sweep3d(u, r: int, *, nthreads: int = 0, return_means: bool = False):
    """One sweep on one volume: (next, sel [D,H,W], err [D,H,W,14]) and with
    ``return_means`` the 14 window means [D,H,W,14]."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    D, H, W = u.shape
    out = np.empty_like(u)
    sel = np.empty((D, H, W), np.uint8)
    err = np.empty((D, H, W, 14), np.float64)
    means = np.empty((D, H, W, 14), np.float64) if return_means else None
    _load().oracle3d_sweep(_pd(u), _pd(out), _pu8(sel), _pd(err),
                           None if means is None else _pd(means), D, H, W, r, nthreads)
    return (out, sel, err, means) if return_means else (out, sel, err)


def select_int64_3d(x, r: int):
    """Exact integer selection for one volume sweep: (sel, sums [D,H,W,14])."""
    a = np.ascontiguousarray(x, dtype=np.int64)
    D, H, W = a.shape
    sel = np.empty((D, H, W), np.uint8)
    sums = np.empty((D, H, W, 14), np.int64)
    _load().oracle3d_select_int64(a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _pu8(sel),
                                  sums.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), D, H, W, r)
    return sel, sums


# --------------------------------------------------- one-sided Gaussian

def gauss_forward(x, r: int, sigma: float, T: int, *, return_sel: bool = False, nthreads: int = 0):
    """T sweeps of the one-sided Gaussian filter (same windows and order as
    the box filter, weights exp(-u^2/(2 sigma^2)) per axis), clamp boundary."""
    shape = np.shape(x)
    a = _planes(x)
    P, H, W = a.shape
    out = np.empty_like(a)
    sel = np.empty((T, P, H, W), np.uint8) if return_sel else None
    if _load().oracle_gauss_forward(_pd(a), _pd(out), _pu8(sel), P, H, W, r, float(sigma), T, nthreads) != 0:
        raise ValueError("oracle_gauss_forward failed")
    out = out.reshape(shape)
    return (out, sel) if return_sel else out


def gauss_sweep(u, r: int, sigma: float, *, nthreads: int = 0):
    """One Gaussian sweep on one plane: (next, sel [H,W], err [H,W,8] =
    N |mean_i - c| with N = Zh^2 Zf, means [H,W,8])."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    H, W = u.shape
    out = np.empty_like(u)
    sel = np.empty((H, W), np.uint8)
    err = np.empty((H, W, 8), np.float64)
    means = np.empty((H, W, 8), np.float64)
    _load().oracle_gauss_sweep(_pd(u), _pd(out), _pu8(sel), _pd(err), _pd(means), H, W, r, float(sigma),
                               nthreads)
    return out, sel, err, means
