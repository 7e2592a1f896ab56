"""FP64 oracle for W-stacking with the plain gridder.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): imported by tests/ and
by the benchmark's CPU-baseline leg; the GPU library never imports it.

W-stacking (Section 1.7.1, correction of the W-term in the (l, m)-plane;
the W-handling route the thesis leaves open for its gridders, Section 9.1):
records with similar w are gridded with the plain convolutional gridder
onto separate grids, each grid is inverse transformed, multiplied by the
inverse W-term of its layer,
    gbar_{w_j}(l, m) = exp(+j2pi w_j (sqrt(1 - l^2 - m^2) - 1))   (Section 1.3),
and the images are summed (then corrected for the gridding kernel).

Layer rule (a reading; the thesis gives none): L layers of spacing dw
centred on w_j = (j - (L-1)/2) dw; a record goes to
    j = floor(w / dw + L/2) clamped to [0, L-1]
(w times inv_dw, plus L/2, each rounded in FP64 as written).  Each layer is
an ordinary nu x nv grid with the usual index rule and bounds; the layers
are kept as [npol][L][nv][nu].  Image coordinates: l = (x - nx/2)/nx times
the field in radians (the grid's cells-per-wavelength scale), likewise m.
"""
from __future__ import annotations

import numpy as np

from . import grid as _grid
from .imaging import inverse_transform


def layer_of(w, layers: int, inv_dw: float) -> np.ndarray:
    """Layer index of each w (float64 arithmetic as written)."""
    a = np.asarray(w, np.float64) * np.float64(inv_dw)
    a = a + np.float64(0.5 * layers)
    j = np.floor(a)
    return np.clip(j, 0, layers - 1).astype(np.int64)


def layer_w(layers: int, dw: float) -> np.ndarray:
    return (np.arange(layers) - (layers - 1) / 2.0) * dw


def grid_layers(geom, taps, uvw, vis, layers: int, inv_dw: float):
    """Grid every layer's records onto its own grid with the oracle gridder.
    Returns (grids complex128 [npol, L, nv, nu], skipped)."""
    uvw = np.asarray(uvw, np.float64)
    vis = np.asarray(vis)
    if vis.ndim == 1:
        vis = vis[:, None]
    j = layer_of(uvw[:, 2], layers, inv_dw)
    out = np.zeros((vis.shape[1], layers, geom.nv, geom.nu), np.complex128)
    skipped = 0
    for lay in range(layers):
        sel = j == lay
        if not np.any(sel):
            continue
        g, sk = _grid(geom, taps, uvw[sel], vis[sel])
        out[:, lay] = g
        skipped += sk
    return out, skipped


def gbar(w: float, nx: int, ny: int, fov_x: float, fov_y: float) -> np.ndarray:
    """Inverse W-term on the image pixels, [ny, nx]."""
    l = (np.arange(nx) - nx // 2) / nx * fov_x
    m = (np.arange(ny) - ny // 2) / ny * fov_y
    r2 = m[:, None] ** 2 + l[None, :] ** 2
    return np.exp(2j * np.pi * w * (np.sqrt(np.maximum(1.0 - r2, 0.0)) - 1.0))


def image(grids, corr_x, corr_y, fov_x: float, fov_y: float, dw: float) -> np.ndarray:
    """Sum over layers of inverse_transform(layer) x gbar_{w_j}, corrected:
    [npol, ny, nx]."""
    G = np.asarray(grids)
    npol, L, ny, nx = G.shape
    ws = layer_w(L, dw)
    out = np.zeros((npol, ny, nx), np.complex128)
    for j in range(L):
        out += inverse_transform(G[:, j]) * gbar(ws[j], nx, ny, fov_x, fov_y)[None]
    return out * np.asarray(corr_y, np.float64)[None, :, None] * np.asarray(corr_x, np.float64)[None, None, :]
