"""FP64 CPU oracle for gridding / degridding (ctypes wrapper of oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports it and it
imports nothing from the GPU library.

The arithmetic lives in oracle.c; this module only marshals numpy arrays.
See oracle.c for the definition followed and its citations.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    lp = C.POINTER(C.c_int64)
    geom = [C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
            C.c_int32, ip, C.c_double, C.c_int32]
    lib.orc_index.argtypes = geom + [C.c_int64, dp, ip, ip, ip, ip, ip,
                                     C.POINTER(C.c_uint8)]
    lib.orc_index.restype = C.c_int64
    lib.orc_grid_window.argtypes = geom + [dp, lp, C.c_int64, dp, C.c_int32, dp,
                                           C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp]
    lib.orc_grid_window.restype = C.c_int64
    lib.orc_degrid.argtypes = geom + [dp, lp, C.c_int64, dp, C.c_int32, dp, dp]
    lib.orc_degrid.restype = C.c_int64
    lib.orc_dft.argtypes = [C.c_int64, dp, dp, C.c_int32, C.c_int32, dp]
    lib.orc_dft.restype = None
    lib.orc_grid_window_par.argtypes = lib.orc_grid_window.argtypes + [C.c_int32, C.c_int32]
    lib.orc_grid_window_par.restype = C.c_int64
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = C.c_int32
    lib.orc_hybrid_grid_window.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                           C.c_double, C.c_int32, dp, C.c_int64, dp, C.c_int32,
                                           dp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp]
    lib.orc_hybrid_grid_window.restype = C.c_int64
    lib.orc_prune_columns.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                      dp, dp, dp]
    lib.orc_prune_columns.restype = C.c_int64
    _lib = lib
    return lib


def _ptr(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


@dataclasses.dataclass
class Geometry:
    """Grid + kernel description handed to the oracle.

    kind "separable": taps is a real table of length beta*support + 1.
    kind "wproj": taps is the concatenation of complex planes, plane p of
    shape (beta*S_p + 1)^2 starting at plane_offset[p] (complex elements).
    """
    nu: int
    nv: int
    beta: int
    scale_u: float
    scale_v: float
    kind: str = "separable"
    support: int = 0
    plane_support: Optional[Sequence[int]] = None
    plane_offset: Optional[Sequence[int]] = None
    inv_dw: float = 0.0

    @property
    def nplanes(self) -> int:
        return 0 if self.kind == "separable" else len(self.plane_support)


def _geom_args(g: Geometry):
    if g.kind == "separable":
        ps = np.zeros(1, np.int32)
        nplanes = 0
    else:
        ps = np.ascontiguousarray(g.plane_support, np.int32)
        nplanes = len(ps)
    return ps, (g.nu, g.nv, g.beta, float(g.scale_u), float(g.scale_v), nplanes,
                _ptr(ps, C.c_int32), float(g.inv_dw), int(g.support))


def _taps_args(g: Geometry, taps):
    if g.kind == "separable":
        t = np.ascontiguousarray(np.asarray(taps, np.float64))
        off = np.zeros(1, np.int64)
    else:
        t = np.ascontiguousarray(np.asarray(taps, np.complex128)).view(np.float64)
        off = np.ascontiguousarray(g.plane_offset, np.int64)
    return t, off


def _uvw64(uvw):
    return np.ascontiguousarray(np.asarray(uvw).astype(np.float64, copy=False))


def index(g: Geometry, uvw):
    """Per-record integer indices: dict of k_lo_u, k_lo_v, o_u, o_v, plane
    (int32), valid (uint8), and the skipped count."""
    lib = _load()
    uvw = _uvw64(uvw)
    n = uvw.shape[0]
    out = {k: np.zeros(n, np.int32) for k in ("k_lo_u", "k_lo_v", "o_u", "o_v", "plane")}
    out["valid"] = np.zeros(n, np.uint8)
    ps, ga = _geom_args(g)
    sk = lib.orc_index(*ga, n, _ptr(uvw), *(_ptr(out[k], C.c_int32) for k in
                                           ("k_lo_u", "k_lo_v", "o_u", "o_v", "plane")),
                       _ptr(out["valid"], C.c_uint8))
    if sk < 0:
        raise ValueError("oracle: invalid geometry")
    out["nskipped"] = int(sk)
    return out


def grid(g: Geometry, taps, uvw, vis, window=None, out=None):
    """Gridding (accumulating into `out` if given).  vis: complex [nrec, npol].
    window = (u0, v0, wu, wv) restricts the output to that sub-rectangle of
    the grid.  Returns (grid complex128 [npol, wv, wu], nskipped)."""
    lib = _load()
    uvw = _uvw64(uvw)
    vis = np.ascontiguousarray(np.asarray(vis, np.complex128))
    if vis.ndim == 1:
        vis = vis[:, None]
    npol = vis.shape[1]
    u0, v0, wu, wv = window if window is not None else (0, 0, g.nu, g.nv)
    if out is None:
        out = np.zeros((npol, wv, wu), np.complex128)
    assert out.dtype == np.complex128 and out.flags.c_contiguous and out.shape == (npol, wv, wu)
    t, off = _taps_args(g, taps)
    ps, ga = _geom_args(g)
    sk = lib.orc_grid_window(*ga, _ptr(t), _ptr(off, C.c_int64), uvw.shape[0], _ptr(uvw), npol,
                             _ptr(vis.view(np.float64)), u0, v0, wu, wv,
                             _ptr(out.view(np.float64)))
    if sk < 0:
        raise ValueError("oracle: invalid geometry")
    return out, int(sk)


def grid_par(g: Geometry, taps, uvw, vis, window=None, out=None, nthreads: int = 0,
             nbands: int = 0):
    """The same gridding as grid(), on several host threads (row bands owned
    by one thread each, records in input order inside a band: the result
    equals grid() bit for bit).  Used for the CPU rate.  nthreads <= 0: the
    OpenMP default; nbands <= 0: 8 bands per thread."""
    lib = _load()
    uvw = _uvw64(uvw)
    vis = np.ascontiguousarray(np.asarray(vis, np.complex128))
    if vis.ndim == 1:
        vis = vis[:, None]
    npol = vis.shape[1]
    u0, v0, wu, wv = window if window is not None else (0, 0, g.nu, g.nv)
    if out is None:
        out = np.zeros((npol, wv, wu), np.complex128)
    assert out.dtype == np.complex128 and out.flags.c_contiguous and out.shape == (npol, wv, wu)
    nt = nthreads if nthreads > 0 else max_threads()
    nb = nbands if nbands > 0 else 8 * nt
    t, off = _taps_args(g, taps)
    ps, ga = _geom_args(g)
    sk = lib.orc_grid_window_par(*ga, _ptr(t), _ptr(off, C.c_int64), uvw.shape[0], _ptr(uvw),
                                 npol, _ptr(vis.view(np.float64)), u0, v0, wu, wv,
                                 _ptr(out.view(np.float64)), int(nthreads), int(nb))
    if sk == -2:
        raise MemoryError("oracle: record lists")
    if sk < 0:
        raise ValueError("oracle: invalid geometry")
    return out, int(sk)


def hybrid_grid(g: Geometry, taps, uvw, vis, window=None, out=None):
    """Hybrid Gridding Step (separable geometry only): the kernel along u,
    nearest neighbour onto the beta-oversampled v axis.  Grid complex128
    [npol, beta nv, nu] (or the window (u0, v0, wu, wv) of it, v0 and wv in
    rows of the oversampled axis).  Returns (grid, nskipped)."""
    assert g.kind == "separable"
    lib = _load()
    uvw = _uvw64(uvw)
    vis = np.ascontiguousarray(np.asarray(vis, np.complex128))
    if vis.ndim == 1:
        vis = vis[:, None]
    npol = vis.shape[1]
    rows = g.beta * g.nv
    u0, v0, wu, wv = window if window is not None else (0, 0, g.nu, rows)
    if out is None:
        out = np.zeros((npol, wv, wu), np.complex128)
    assert out.dtype == np.complex128 and out.flags.c_contiguous and out.shape == (npol, wv, wu)
    t = np.ascontiguousarray(np.asarray(taps, np.float64))
    sk = lib.orc_hybrid_grid_window(g.nu, g.nv, g.beta, float(g.scale_u), float(g.scale_v),
                                    int(g.support), _ptr(t), uvw.shape[0], _ptr(uvw), npol,
                                    _ptr(vis.view(np.float64)), u0, v0, wu, wv,
                                    _ptr(out.view(np.float64)))
    if sk < 0:
        raise ValueError("oracle: invalid geometry")
    return out, int(sk)


def prune_columns(grid_in, alpha: int, ztaps, support_z: int):
    """Column pruning: every column of grid_in [npol, M, ncols] circularly
    convolved with the pruning kernel (table of alpha Sz + 1 values) and
    downsampled by alpha.  Returns complex128 [npol, M / alpha, ncols]."""
    lib = _load()
    G = np.ascontiguousarray(np.asarray(grid_in, np.complex128))
    npol, M, ncols = G.shape
    out = np.zeros((npol, M // alpha, ncols), np.complex128)
    z = np.ascontiguousarray(np.asarray(ztaps, np.float64))
    assert z.shape[0] >= alpha * support_z + 1
    rc = lib.orc_prune_columns(npol, M, ncols, alpha, support_z, _ptr(z),
                               _ptr(G.view(np.float64)), _ptr(out.view(np.float64)))
    if rc < 0:
        raise ValueError("oracle: invalid pruning geometry")
    return out


def max_threads() -> int:
    """Host threads the parallel gridder uses by default."""
    return int(_load().orc_max_threads())


def degrid(g: Geometry, taps, uvw, grid_in):
    """Degridding.  grid_in: complex [npol, nv, nu].  Returns
    (vis complex128 [nrec, npol], nskipped)."""
    lib = _load()
    uvw = _uvw64(uvw)
    G = np.ascontiguousarray(np.asarray(grid_in, np.complex128))
    npol = G.shape[0]
    assert G.shape == (npol, g.nv, g.nu)
    out = np.zeros((uvw.shape[0], npol), np.complex128)
    t, off = _taps_args(g, taps)
    ps, ga = _geom_args(g)
    sk = lib.orc_degrid(*ga, _ptr(t), _ptr(off, C.c_int64), uvw.shape[0], _ptr(uvw), npol,
                        _ptr(G.view(np.float64)), _ptr(out.view(np.float64)))
    if sk < 0:
        raise ValueError("oracle: invalid geometry")
    return out, int(sk)


def dft(pos_cells, F, nx: int, ny: int):
    """Direct Fourier sum at positions in cells from the grid centre;
    returns complex128 [ny, nx]."""
    lib = _load()
    pos = np.ascontiguousarray(np.asarray(pos_cells, np.float64))
    Fv = np.ascontiguousarray(np.asarray(F, np.complex128))
    img = np.zeros((ny, nx), np.complex128)
    lib.orc_dft(pos.shape[0], _ptr(pos), _ptr(Fv.view(np.float64)), nx, ny,
                _ptr(img.view(np.float64)))
    return img
