"""Seeded synthetic workloads for gridding and degridding.

Everything produced here is an *input* to the gridding map: record
coordinates (u, v, w) in wavelengths, 4-polarisation visibility values, the
oversampled kernel tables (separable prolate-spheroidal taps and W-projection
planes) and the grid geometry.  No gridding or degridding arithmetic lives
here, so the CPU oracle and the GPU library can both take their inputs from
this module without sharing any of the method's arithmetic.

Array geometry follows the (u, v, w) frame of the measurement equation (the
W axis points at the phase centre; u, v are baseline components in
wavelengths, Chapter 1, "The measurement equation").  Records are produced in
measurement-set order: [time][baseline][channel], 4 polarisations each.

The W-projection planes are samples of the Fourier transform of the
image-domain taper times the inverse W-term (Section 1.3, the convolution
relation between the plane w = c and the plane w = 0), cropped to the plane's
support; they are generated with numpy FFTs and handed to the gridders as a
table, like the separable taps.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

C_LIGHT = 299_792_458.0

SEED_ANTENNAS = 2111
SEED_VIS = 2112
SEED_NOISE = 2113
SEED_TRACE = 2114
SEED_SUBSAMPLE = 2115


# --------------------------------------------------------------------------
# array layouts and uvw synthesis
# --------------------------------------------------------------------------

def antennas_uniform_disc(n: int, diameter_m: float, seed: int = SEED_ANTENNAS) -> np.ndarray:
    """n antenna (E, N, U) positions, uniform over a disc, flat ground (U = 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = 0.5 * diameter_m * np.sqrt(rng.random(n))
    th = 2.0 * np.pi * rng.random(n)
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n)], axis=1)


def antennas_log_radial(n: int, r_min_m: float, r_max_m: float,
                        seed: int = SEED_ANTENNAS) -> np.ndarray:
    """n antennas with log-uniform radius in [r_min, r_max] and uniform angle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = r_min_m * (r_max_m / r_min_m) ** rng.random(n)
    th = 2.0 * np.pi * rng.random(n)
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n)], axis=1)


def baselines_enu(ant: np.ndarray) -> np.ndarray:
    """All antenna pairs i < j, as ENU difference vectors [B, 3] (metres)."""
    i, j = np.triu_indices(ant.shape[0], k=1)
    return ant[j] - ant[i]


def baseline_uvw_m(bl_enu: np.ndarray, lat_rad: float, dec_rad: float,
                   hour_angles_rad: np.ndarray) -> np.ndarray:
    """Earth-rotation synthesis: [T, B, 3] (u, v, w) in metres.

    ENU -> equatorial XYZ, then the textbook rotation for hour angle H and
    declination dec (W axis towards the phase centre).
    """
    e, n, u = bl_enu[:, 0], bl_enu[:, 1], bl_enu[:, 2]
    sl, cl = math.sin(lat_rad), math.cos(lat_rad)
    X = -n * sl + u * cl
    Y = e
    Z = n * cl + u * sl
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    H = hour_angles_rad[:, None]
    sh, ch = np.sin(H), np.cos(H)
    uu = sh * X + ch * Y
    vv = -sd * ch * X + sd * sh * Y + cd * Z
    ww = cd * ch * X - cd * sh * Y + sd * Z
    return np.stack([uu, vv, ww], axis=-1)


def hour_angles(n_times: int, span_hours: float = 6.0) -> np.ndarray:
    return np.linspace(-0.5 * span_hours, 0.5 * span_hours, n_times) * (2.0 * np.pi / 24.0)


def uvw_wavelengths(uvw_m: np.ndarray, freqs_hz: np.ndarray, dtype=np.float64) -> np.ndarray:
    """[T, B, 3] metres x [C] Hz -> [T*B*C, 3] wavelengths in MS order."""
    T, B, _ = uvw_m.shape
    out = uvw_m[:, :, None, :] * (np.asarray(freqs_hz, np.float64) / C_LIGHT)[None, None, :, None]
    return np.ascontiguousarray(out.reshape(T * B * len(freqs_hz), 3).astype(dtype))


def uv_scale(uvw: np.ndarray, n: int, support: int, fill: float = 0.5) -> float:
    """Cells per wavelength so that all records lie in the central `fill` of
    the grid, with room for the kernel footprint (records must stay inside the
    grid, the bounded-records rule, Section 2.3)."""
    umax = float(np.max(np.abs(uvw[:, :2])))
    return fill * (n / 2 - support) / umax


# --------------------------------------------------------------------------
# visibilities
# --------------------------------------------------------------------------

def vis_normal(nrec: int, npol: int = 4, seed: int = SEED_VIS) -> np.ndarray:
    """complex64 [nrec, npol], real and imaginary parts i.i.d. N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((nrec, npol, 2), dtype=np.float32)
    return x.view(np.complex64).reshape(nrec, npol)


def vis_normal_torch(nrec: int, npol: int, seed: int, device):
    """complex64 [nrec, npol] N(0,1) parts drawn with torch's generator on
    `device` (used for the large workloads, where numpy on the host would be
    slow).  Reproducible for a fixed device type and seed."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.randn(nrec, npol, 2, generator=g, device=device, dtype=torch.float32)
    return torch.view_as_complex(x)


# --------------------------------------------------------------------------
# kernel tables
# --------------------------------------------------------------------------

def pswf_taps(support: int, beta: int) -> np.ndarray:
    """Separable prolate-spheroidal taps, table of length beta*support + 1.

    Entry t holds the kernel at offset (t - beta*support/2)/beta cells; the
    centre entry is 1.  Shape (1 - eta^2) psi_0(c, eta) with c = pi*S/2, using
    scipy's prolate spheroidal angular function (the thesis grids with a
    prolate spheroidal of support 6 generated as in CASA, whose exact recipe
    it does not print; Chapter 4, "The GCF").
    """
    import scipy.special as sp
    S, b = int(support), int(beta)
    t = np.arange(b * S + 1, dtype=np.float64)
    eta = 2.0 * (t - b * S / 2) / (b * S)
    c = np.pi * S / 2
    psi, _ = sp.pro_ang1(0, 0, c, np.clip(eta, -1 + 1e-15, 1 - 1e-15))
    taps = (1.0 - eta ** 2) * psi
    taps /= taps[b * S // 2]
    taps[0] = taps[-1] = 0.0
    return taps


def wproj_support_schedule(nplanes: int, s_min: int, s_max: int) -> np.ndarray:
    """Even supports growing linearly from s_min to s_max over the planes."""
    if nplanes == 1:
        return np.array([s_min], np.int32)
    p = np.arange(nplanes)
    half = (s_max - s_min) // 2
    return (s_min + 2 * np.round(half * p / (nplanes - 1))).astype(np.int32)


def wproj_plane(base_taps: np.ndarray, base_support: int, beta: int, support: int,
                w: float, fov_rad: float) -> np.ndarray:
    """One W-projection table, complex128 [(beta*S+1), (beta*S+1)].

    K = FFT2[ c(l) c(m) * gbar_w(l, m) ] sampled every 1/beta cells, where c
    is the inverse DFT of the separable taps (so that K at w = 0 is exactly
    the outer product of the taps) and gbar_w = exp(+j 2 pi w (sqrt(1-l^2-m^2)
    - 1)) is the inverse W-term with l, m the physical direction cosines
    (normalised image coordinate times the field of view in radians).
    """
    b, S, S0 = int(beta), int(support), int(base_support)
    if (b * (S - S0)) % 2 or S < S0:
        raise ValueError("support must be >= base support with beta*(S-S0) even")
    M = 2 * b * S
    L = b * S0 + 1
    pad = np.zeros(M)
    pad[M // 2 - b * S0 // 2: M // 2 - b * S0 // 2 + L] = base_taps
    # image-domain taper (periodic with period beta in normalised l)
    c1 = np.fft.ifft(np.fft.ifftshift(pad))
    lnorm = np.fft.ifftshift((np.arange(M) - M // 2) * (b / M))
    lphys = lnorm * fov_rad
    l2 = lphys[:, None] ** 2 + lphys[None, :] ** 2
    n = np.sqrt(np.maximum(1.0 - l2, 0.0))
    gbar = np.exp(2j * np.pi * w * (n - 1.0))
    img = c1[:, None] * c1[None, :] * gbar
    K = np.fft.fftshift(np.fft.fft2(img))
    lo = M // 2 - b * S // 2
    return np.ascontiguousarray(K[lo: lo + b * S + 1, lo: lo + b * S + 1])


@dataclasses.dataclass
class WBank:
    """A W-projection kernel bank: planes over |w|, concatenated row-major."""
    beta: int
    supports: np.ndarray        # int32 [P]
    offsets: np.ndarray         # int64 [P], element offset of each plane
    taps: np.ndarray            # complex128 [sum (beta*S_p+1)^2]
    inv_dw: float

    @property
    def nplanes(self) -> int:
        return int(self.supports.shape[0])

    @property
    def support_max(self) -> int:
        return int(self.supports.max())

    def plane(self, p: int) -> np.ndarray:
        S = int(self.supports[p])
        n = self.beta * S + 1
        o = int(self.offsets[p])
        return self.taps[o: o + n * n].reshape(n, n)


def wproj_bank(nplanes: int, s_min: int, s_max: int, beta: int, w_absmax: float,
               fov_rad: float, base_support: int = 7) -> WBank:
    """Planes at w_p = p * dw, dw = w_absmax / (P - 1); plane p of support S_p
    from the linear schedule.  Normalised so that the largest |tap| is 1."""
    sup = wproj_support_schedule(nplanes, s_min, s_max)
    base = pswf_taps(base_support, beta)
    dw = w_absmax / max(nplanes - 1, 1)
    planes = [wproj_plane(base, base_support, beta, int(s), p * dw, fov_rad)
              for p, s in enumerate(sup)]
    sizes = np.array([pl.size for pl in planes], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    taps = np.concatenate([pl.ravel() for pl in planes])
    taps /= np.max(np.abs(taps))
    return WBank(beta=beta, supports=sup, offsets=offs, taps=taps,
                 inv_dw=(1.0 / dw) if dw > 0 else 0.0)


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    n: int                      # grid side (cells)
    npol: int
    beta: int
    scale: float                # cells per wavelength (= field of view, rad)
    uvw: np.ndarray             # [nrec, 3] wavelengths (float64 or float32)
    kind: str                   # "separable" | "wproj"
    support: int                # separable support, or max plane support
    taps: Optional[np.ndarray] = None   # separable taps (float64)
    bank: Optional[WBank] = None

    @property
    def nrec(self) -> int:
        return int(self.uvw.shape[0])


def config_small(seed: int = SEED_ANTENNAS) -> Workload:
    """64 antennas in a 1 km disc, 2016 baselines x 50 times x 1 channel at
    0.21 m, dec -30 deg, 6 h; 1024^2 grid, 7x7 prolate spheroidal, beta 8."""
    ant = antennas_uniform_disc(64, 1000.0, seed)
    bl = baselines_enu(ant)
    uvw_m = baseline_uvw_m(bl, math.radians(-30.0), math.radians(-30.0), hour_angles(50))
    uvw = uvw_wavelengths(uvw_m, np.array([C_LIGHT / 0.21]))
    n, S, beta = 1024, 7, 8
    return Workload("small-sep7-1024", n, 4, beta, uv_scale(uvw, n, S), uvw,
                    "separable", S, taps=pswf_taps(S, beta))


def config_wproj(n_ant: int = 256, n_times: int = 32, n_chan: int = 128, n: int = 8192,
                 nplanes: int = 32, s_min: int = 8, s_max: int = 64, beta: int = 4,
                 r_max_m: float = 2500.0, seed: int = SEED_ANTENNAS,
                 uvw_dtype=np.float32, name: Optional[str] = None) -> Workload:
    """Log-radial array (radius 20 m .. r_max), 1.2-1.6 GHz, W-projection bank
    with `nplanes` planes over |w|, supports s_min -> s_max, oversampling beta."""
    ant = antennas_log_radial(n_ant, 20.0, r_max_m, seed)
    bl = baselines_enu(ant)
    uvw_m = baseline_uvw_m(bl, math.radians(-30.0), math.radians(-30.0), hour_angles(n_times))
    freqs = np.linspace(1.2e9, 1.6e9, n_chan, endpoint=False)
    uvw = uvw_wavelengths(uvw_m, freqs, dtype=np.float64)
    scale = uv_scale(uvw, n, s_max)
    w_absmax = float(np.max(np.abs(uvw[:, 2])))
    bank = wproj_bank(nplanes, s_min, s_max, beta, w_absmax, scale)
    return Workload(name or f"wproj-{n}-P{nplanes}-S{s_min}to{s_max}", n, 4, beta, scale,
                    uvw.astype(uvw_dtype), "wproj", s_max, bank=bank)


def config_autograd(seed: int = SEED_ANTENNAS) -> Workload:
    """The 64-antenna 1 km array, 2016 baselines x 100 times x 50 channels
    (+-10 % around 1.43 GHz) = 10,080,000 records; 2048^2 grid, 7x7, beta 8."""
    ant = antennas_uniform_disc(64, 1000.0, seed)
    bl = baselines_enu(ant)
    uvw_m = baseline_uvw_m(bl, math.radians(-30.0), math.radians(-30.0), hour_angles(100))
    freqs = np.linspace(1.43e9 * 0.9, 1.43e9 * 1.1, 50)
    uvw = uvw_wavelengths(uvw_m, freqs, dtype=np.float64)
    n, S, beta = 2048, 7, 8
    return Workload("autograd-sep7-2048-10M", n, 4, beta, uv_scale(uvw, n, S),
                    uvw.astype(np.float32), "separable", S, taps=pswf_taps(S, beta))


def subsample(nrec: int, k: int, seed: int = SEED_SUBSAMPLE) -> np.ndarray:
    """Sorted random subset of k record indices out of nrec."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(nrec, size=min(k, nrec), replace=False))


def config_precision_sample(k: int = 1_000_000, seed: int = SEED_SUBSAMPLE,
                            n: int = 16384, nplanes: int = 32, s_min: int = 8,
                            s_max: int = 64, beta: int = 4) -> Workload:
    """A k-record random subsample of the 1,004,666,880-record precision
    workload: 512 antennas log-radial 20 m .. 5 km (130816 baselines) x 16
    times x 480 channels in 1.2-1.6 GHz, 16384^2 grid, W-projection with
    32 planes, S 8 -> 64, oversampling 4.  Only the sampled records are
    synthesised: record i of the [time][baseline][channel] order takes the
    same float64 product as uvw_wavelengths, so the values equal those rows
    of the full array.  The uv scale and the plane spacing come from the
    full array's extremes (the largest |u|, |v|, |w| sit at the highest
    frequency).  uvw is float32."""
    ant = antennas_log_radial(512, 20.0, 5000.0, SEED_ANTENNAS)
    bl = baselines_enu(ant)
    uvw_m = baseline_uvw_m(bl, math.radians(-30.0), math.radians(-30.0), hour_angles(16))
    freqs = np.linspace(1.2e9, 1.6e9, 480, endpoint=False)
    f = freqs / C_LIGHT
    T, B, _ = uvw_m.shape
    C = f.shape[0]
    idx = subsample(T * B * C, k, seed)
    t, b, c = idx // (B * C), (idx // C) % B, idx % C
    uvw = uvw_m[t, b] * f[c][:, None]
    umax = float(np.max(np.abs(uvw_m[..., :2]))) * f[-1]
    wmax = float(np.max(np.abs(uvw_m[..., 2]))) * f[-1]
    scale = 0.5 * (n / 2 - s_max) / umax
    bank = wproj_bank(nplanes, s_min, s_max, beta, wmax, scale)
    return Workload(f"precision-{n}-P{nplanes}-S{s_min}to{s_max}-{k}-of-1.0G", n, 4, beta,
                    scale, np.ascontiguousarray(uvw.astype(np.float32)), "wproj", s_max,
                    bank=bank)


def config_wproj_device(device, n_ant: int = 256, n_times: int = 32, n_chan: int = 128,
                        n: int = 8192, nplanes: int = 32, s_min: int = 8, s_max: int = 64,
                        beta: int = 4, r_max_m: float = 2500.0, seed: int = SEED_ANTENNAS,
                        name: Optional[str] = None) -> Workload:
    """config_wproj with the [time][baseline][channel] uvw expansion done on
    `device` (torch), for the large workloads.  The per-channel scaling is
    the same float64 product as the numpy path, so the values are identical;
    uvw is returned as a float32 device tensor."""
    import torch
    ant = antennas_log_radial(n_ant, 20.0, r_max_m, seed)
    bl = baselines_enu(ant)
    uvw_m = baseline_uvw_m(bl, math.radians(-30.0), math.radians(-30.0), hour_angles(n_times))
    freqs = np.linspace(1.2e9, 1.6e9, n_chan, endpoint=False)
    um = torch.from_numpy(uvw_m).to(device)
    fr = torch.from_numpy(freqs / C_LIGHT).to(device)
    T, B, _ = uvw_m.shape
    out = torch.empty(T * B * n_chan, 3, dtype=torch.float32, device=device)
    umax = 0.0
    wmax = 0.0
    step = max(1, T // 8)
    for t0 in range(0, T, step):
        blk = um[t0:t0 + step, :, None, :] * fr[None, None, :, None]
        umax = max(umax, float(blk[..., :2].abs().max()))
        wmax = max(wmax, float(blk[..., 2].abs().max()))
        out[t0 * B * n_chan:(t0 + blk.shape[0]) * B * n_chan] = blk.reshape(-1, 3).to(torch.float32)
        del blk
    scale = 0.5 * (n / 2 - s_max) / umax
    bank = wproj_bank(nplanes, s_min, s_max, beta, wmax, scale)
    return Workload(name or f"wproj-{n}-P{nplanes}-S{s_min}to{s_max}", n, 4, beta, scale,
                    out, "wproj", s_max, bank=bank)


def config_autograd_problem(device, seed: int = SEED_NOISE, n_sources: int = 50,
                            sigma: float = 0.1):
    """The differentiable grid/degrid workload: the 10,080,000-record
    64-antenna array of config_autograd on a 2048^2 grid (7x7, beta 8), a
    model grid W_true = FFT of a tapered image of `n_sources` point sources,
    and V_obs = (degridded W_true) + sigma (n_r + j n_i) noise is produced by
    the caller with the library (this function returns W_true and the noise).
    Returns (workload, W_true [4, n, n] complex64, noise [nrec, 4] complex64)
    as torch tensors on `device`."""
    import torch
    wl = config_autograd()
    n = wl.n
    rng = np.random.Generator(np.random.PCG64(seed))
    img = np.zeros((n, n), np.complex128)
    xs = rng.integers(n // 4, 3 * n // 4, (n_sources, 2))
    flux = rng.uniform(0.5, 2.0, n_sources)
    for (x, y), f in zip(xs, flux):
        img[y, x] += f
    # taper the image so the model grid is smooth (Gaussian image-plane taper)
    yy, xx = np.mgrid[0:n, 0:n]
    img *= np.exp(-(((xx - n / 2) / (0.3 * n)) ** 2 + ((yy - n / 2) / (0.3 * n)) ** 2))
    W1 = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(img)))
    W = np.stack([W1, 0.5 * W1, 0.25 * W1, W1]).astype(np.complex64)
    noise = vis_normal_torch(wl.nrec, 4, seed + 1, device) * sigma
    return wl, torch.from_numpy(W).to(device), noise
