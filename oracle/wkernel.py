"""FP64 oracle for kernel generation: W-projection kernel tables, the map
error (misfit) of a gridding kernel, and the column-pruning aliasing
experiment.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): imported by tests/ and
by the benchmark's CPU-baseline leg; the GPU library never imports it.

W-projection tables (Section 1.3, plane at w = c: the W-term
g_w(l, m) = exp(-j2pi w (sqrt(1 - l^2 - m^2) - 1)) and its inverse
gbar_w = 1 / g_w; Section 1.7.1: W-projection grids a record at w with the
GCF convolved with Gbar_w = F gbar_w, which projects it onto the w = 0
plane):
    K_w(u, v) = F[ c(l) c(m) gbar_w(l, m) ](u, v),   c = F^-1 C,
F with exp(-j2pi (ul + vm)) (Section 1.3), C the separable GCF given by its
table T of beta S0 + 1 samples at 1/beta cells (entry t at (t - beta S0/2)/beta
cells).  Discretisation (the reading used throughout): an M x M image grid,
M = 2 beta S, of spacing beta/M in units of the field, so that its discrete
transform has uv spacing 1/beta cells and spans 2S cells; the table of a
plane of support S is the central beta S + 1 samples per axis.  Physical
direction cosines are the field coordinate times `fov` (radians spanned by
the grid, the cells-per-wavelength scale of the uv grid).  With i, a
centred indices in [-M/2, M/2):
    c[i]    = (1/M) sum_tau T[tau] exp(+j2pi tau i / M)       (tau centred)
    K[a, b] = sum_{i, j} c[i] c[j] gbar_w(l_i, m_j) exp(-j2pi (a i + b j)/M)
(the second by numpy's FFT, the library step; `wplane_tap_direct` evaluates
it as the plain double sum).  Row index a runs along v, b along u.

Map error (Section 2.3.5, the corrector that minimises the misfit; Ye et al.
as cited there): a record at sub-cell offset nu gridded with kernel C and
imaged gives, at image coordinate x (units of the field),
    r(x, nu) = sum_k C(nu - k) exp(+j2pi (k - nu) x);
the corrected output h(x) r should be 1.  Averaged over nu uniform in [0, 1)
the squared error is h^2 <|r|^2> - 2 h Re<r> + 1, least for
h = Re<r> / <|r|^2>, leaving the map error
    l2(x) = 1 - Re<r>^2 / <|r|^2>.
`misfit` evaluates it by brute force: the average over nu is a sum over
`n_nu` equally spaced offsets.  By Poisson summation <|r|^2> =
sum_b c(x + b)^2 and <r> = c(x), which is the corrector form the thesis
prints; the tests pin the brute force to that closed form.

Column-pruning aliasing experiment (Section 7.6): the test image I(x, y, a),
constant along x, and the reference method (crop).  See `pruning_image`.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# W-projection tables
# ---------------------------------------------------------------------------

def taper(base_taps, beta: int, M: int) -> np.ndarray:
    """c[i], i = -M/2 .. M/2 - 1 (centred order): the inverse DFT of the
    separable table on the M-point grid (plain sum)."""
    T = np.asarray(base_taps, np.float64)
    L = T.shape[0]
    tau = np.arange(L) - (L - 1) // 2
    i = np.arange(M) - M // 2
    return (np.exp(2j * np.pi * np.outer(i, tau) / M) @ T) / M


def gbar(w: float, l, m) -> np.ndarray:
    """Inverse W-term exp(+j2pi w (sqrt(1 - l^2 - m^2) - 1)) on the outer
    grid of l (rows) and m (columns); directions beyond the unit circle
    take n = 0 (they lie outside any physical field)."""
    l = np.asarray(l, np.float64)
    m = np.asarray(m, np.float64)
    r2 = l[:, None] ** 2 + m[None, :] ** 2
    n = np.sqrt(np.maximum(1.0 - r2, 0.0))
    return np.exp(2j * np.pi * w * (n - 1.0))


def _image(base_taps, beta: int, S: int, w: float, fov: float):
    M = 2 * beta * S
    c = taper(base_taps, beta, M)
    l = (np.arange(M) - M // 2) * (beta / M) * fov
    return M, c[:, None] * c[None, :] * gbar(w, l, l)


def wplane(base_taps, beta: int, S: int, w: float, fov: float) -> np.ndarray:
    """The table of one plane, complex128 [beta S + 1, beta S + 1]."""
    M, img = _image(base_taps, beta, S, w, fov)
    K = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(img)))
    lo = M // 2 - beta * S // 2
    return K[lo: lo + beta * S + 1, lo: lo + beta * S + 1]


def wplane_tap_direct(base_taps, beta: int, S: int, w: float, fov: float, ta: int,
                      tb: int) -> complex:
    """Entry (ta, tb) of `wplane` as the plain double sum over the image."""
    M, img = _image(base_taps, beta, S, w, fov)
    a = ta - beta * S // 2
    b = tb - beta * S // 2
    i = np.arange(M) - M // 2
    ea = np.exp(-2j * np.pi * a * i / M)
    eb = np.exp(-2j * np.pi * b * i / M)
    return complex(ea @ img @ eb)


def wbank(base_taps, beta: int, supports, ws, fov: float):
    """Planes one after another (row-major), normalised so that the largest
    |tap| of the bank is 1.  Returns (taps complex128, offsets int64)."""
    planes = [wplane(base_taps, beta, int(S), float(w), fov) for S, w in zip(supports, ws)]
    sizes = np.array([p.size for p in planes], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    taps = np.concatenate([p.ravel() for p in planes])
    return taps / np.max(np.abs(taps)), offs


# ---------------------------------------------------------------------------
# map error of a gridding kernel
# ---------------------------------------------------------------------------

def table_kernel(table, beta: int):
    """C(nu) of a table under nearest-entry lookup (the gridder's GCF
    oversampling): entry t covers offsets within half a step of
    (t - E/2)/beta; zero beyond the table."""
    T = np.asarray(table, np.float64)
    E = T.shape[0] - 1

    def C(nu):
        t = np.floor(np.asarray(nu, np.float64) * beta + 0.5).astype(np.int64) + E // 2
        ok = (t >= 0) & (t <= E)
        return np.where(ok, T[np.clip(t, 0, E)], 0.0)
    return C


def misfit(C, support: int, x, n_nu: int = 512) -> np.ndarray:
    """Map error l2(x) of kernel C (callable on cell offsets, zero outside
    |nu| <= support/2) by brute force over n_nu sub-cell offsets."""
    x = np.asarray(x, np.float64)
    nu = (np.arange(n_nu) + 0.5) / n_nu
    ks = np.arange(-(support // 2) - 1, support // 2 + 2)
    r = np.zeros((x.size, n_nu), np.complex128)
    for k in ks:
        r += C(nu - k)[None, :] * np.exp(2j * np.pi * np.outer(x, k - nu))
    mr = r.mean(axis=1).real
    m2 = (np.abs(r) ** 2).mean(axis=1)
    return 1.0 - mr ** 2 / m2


# ---------------------------------------------------------------------------
# column-pruning aliasing experiment
# ---------------------------------------------------------------------------

def pruning_image(nx: int, ny: int, alpha: int, a: float) -> np.ndarray:
    """I(x, y, a) of the aliasing experiment, [ny * alpha, nx], constant
    along x, origin at the centre.  The pruned field covers y in
    [-ny/2, ny/2); a row y' of the full image folds onto y = y' mod ny
    (centred).  Reading of the description: on the kept field the aliasing
    region -ny/4 <= y < 0 holds a square wave of period 8 between 0.1 and
    1, the zero region 0 <= y <= ny/4 holds 0, and the rest 0; every row
    that folds onto the aliasing region holds a square wave of period 16
    between 0.1a and a, and every other row outside the field 0."""
    Y = ny * alpha
    y = np.arange(Y) - Y // 2
    yf = ((y + ny // 2) % ny) - ny // 2           # folded row
    inside = (y >= -ny // 2) & (y < ny // 2)
    alias_region = (yf >= -ny // 4) & (yf < 0)
    sq8 = np.where((y // 4) % 2 == 0, 1.0, 0.1)
    sq16 = np.where((y // 8) % 2 == 0, a, 0.1 * a)
    col = np.where(inside, np.where(alias_region, sq8, 0.0),
                   np.where(alias_region, sq16, 0.0))
    return np.repeat(col[:, None], nx, axis=1)
