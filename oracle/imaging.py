"""FP64 imaging chain of the oracle: origin shift, inverse FFT and the
Correction Step, for convolutional and hybrid grids.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): imported by tests/ and
by the benchmark's CPU-baseline leg; the GPU library never imports it.

Definitions (numpy in float64; numpy's FFT is the library step):
  * The grids have their origin at the centre (cell n/2 is u = 0).  The
    inverse transform is the unnormalised sum with e^{+j2pi}, the direct
    imaging sum of Section 1.7 evaluated on the grid:
        I[y, x] = sum_{kv, ku} G[kv, ku] exp(+j2pi ((ku - nx/2)(x - nx/2)/nx
                                                    + (kv - ny/2)(y - ny/2)/ny)),
    i.e. fftshift(ifft2(ifftshift(G))) * nx * ny.
  * Correction Step (Algorithm "The studied Convolutional Gridding
    Algorithm", Section 2.4.5, corrector h_co of Section 2.5.5 after
    Greisen and Jackson et al.): per axis, divide by the transform of the
    oversampled kernel averaged over the record's sub-cell phases, times the
    sinc of the nearest-pixel snap onto the beta-oversampled grid:
        h(l) = 1 / ( (1/P) sum_e T[e] cos(2pi ((e - E/2)/beta) l) sinc(l/beta) )
    with l = (i - n/2)/n the image coordinate in units of the field, T the
    table of E + 1 symmetric values whose entry e lies (e - E/2)/beta cells
    from the centre, and P the number of phases (beta for the gridding
    kernel; alpha for the pruning kernel, whose taps act on the rows of the
    beta-oversampled axis, downsampled by alpha).
  * Hybrid Gridding (Algorithm "The studied Hybrid Gridding Algorithm",
    Section 2.4.4): the pruned grid has 2 nv rows at half-cell spacing, so
    its inverse transform covers twice the field along v; the central nv
    rows are kept (the cut-out of the Correction Step) and corrected by h_co
    along u and by the pruning kernel's corrector (h_pr) along v.
"""
from __future__ import annotations

import numpy as np


def corrector(n: int, beta: int, table, phases: int, nn_sinc: bool = True) -> np.ndarray:
    """h(l) at l = (i - n/2)/n, i < n (see the module docstring).  With
    nn_sinc False the sinc of the nearest-pixel snap is left out: the image
    then approximates the direct sum at the snapped positions q / beta."""
    t = np.asarray(table, np.float64)
    E = t.shape[0] - 1
    l = (np.arange(n) - n // 2) / n
    off = (np.arange(E + 1) - E / 2.0) / beta            # cells from the centre
    ct = (np.cos(2.0 * np.pi * np.outer(l, off)) @ t) / phases
    return 1.0 / (ct * np.sinc(l / beta)) if nn_sinc else 1.0 / ct


def inverse_transform(G) -> np.ndarray:
    """Unnormalised inverse 2-D transform of centred grids [..., ny, nx]."""
    G = np.asarray(G, np.complex128)
    ny, nx = G.shape[-2:]
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(G, axes=(-2, -1))),
                           axes=(-2, -1)) * (nx * ny)


def image_conv(G, corr_x, corr_y) -> np.ndarray:
    """Image of a convolutional grid [npol, n, n]: inverse transform times
    corr_x (along x) and corr_y (along y)."""
    I = inverse_transform(G)
    return I * np.asarray(corr_y)[:, None] * np.asarray(corr_x)[None, :]


def image_hybrid(P, corr_x, corr_y) -> np.ndarray:
    """Image of a pruned hybrid grid [npol, 2 nv, nu]: inverse transform over
    the 2 nv x nu grid, the central nv rows kept, corrected by corr_x (nu
    values) and corr_y (nv values)."""
    I = inverse_transform(P)
    rows = I.shape[-2]
    nv = rows // 2
    y0 = nv // 2
    return I[..., y0:y0 + nv, :] * np.asarray(corr_y)[:, None] * np.asarray(corr_x)[None, :]
