"""Shared test helpers: turn a seeded Workload into the oracle's and the GPU
library's inputs (the same values on both sides)."""
import numpy as np

import oracle
from paper_2111_04141_amd import workload as W


def quantise_taps(taps: np.ndarray, dtype: str) -> np.ndarray:
    """Taps as the GPU table stores them, widened back to float64/complex128."""
    import torch
    if dtype == "f32":
        return taps.astype(np.complex64 if np.iscomplexobj(taps) else np.float32).astype(
            np.complex128 if np.iscomplexobj(taps) else np.float64)
    tdt = {"f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    if np.iscomplexobj(taps):
        t = torch.from_numpy(np.stack([taps.real, taps.imag], -1)).to(tdt).to(torch.float64)
        t = t.numpy()
        return t[..., 0] + 1j * t[..., 1]
    return torch.from_numpy(taps).to(tdt).to(torch.float64).numpy()


def oracle_geom(wl: W.Workload) -> oracle.Geometry:
    if wl.kind == "separable":
        return oracle.Geometry(nu=wl.n, nv=wl.n, beta=wl.beta, scale_u=wl.scale,
                               scale_v=wl.scale, support=wl.support)
    b = wl.bank
    return oracle.Geometry(nu=wl.n, nv=wl.n, beta=wl.beta, scale_u=wl.scale, scale_v=wl.scale,
                           kind="wproj", plane_support=b.supports, plane_offset=b.offsets,
                           inv_dw=b.inv_dw)


def oracle_taps(wl: W.Workload, dtype: str = "f32") -> np.ndarray:
    return quantise_taps(wl.taps if wl.kind == "separable" else wl.bank.taps, dtype)


def device_bank(wl: W.Workload, dtype: str = "f32", device="cuda"):
    import torch
    from paper_2111_04141_amd.api import KernelBank
    if wl.kind == "separable":
        tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
        t = torch.from_numpy(wl.taps).to(tdt).to(device)
        return KernelBank("separable", t, support=wl.support)
    b = wl.bank
    if dtype == "f32":
        t = torch.from_numpy(b.taps.astype(np.complex64)).to(device)
    else:
        tdt = {"f16": torch.float16, "bf16": torch.bfloat16}[dtype]
        t = torch.from_numpy(np.stack([b.taps.real, b.taps.imag], -1)).to(tdt).to(device)
    return KernelBank("wproj", t, plane_support=b.supports.tolist(),
                      plane_offset=b.offsets.tolist(), inv_dw=b.inv_dw)


def grid_spec(wl: W.Workload, npol: int = 4):
    from paper_2111_04141_amd.api import GridSpec
    return GridSpec(nu=wl.n, nv=wl.n, npol=npol, beta=wl.beta, scale_u=wl.scale,
                    scale_v=wl.scale)


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return float(d / n) if n > 0 else float(d)


def plan_chunk_records(nrec: int) -> int:
    """Largest record count of one gridding unit for a call of nrec records
    (the library's chunk size R: between 64 and 2048, about nrec / 4096)."""
    return int(max(64, min(2048, nrec // 4096)))


def fixed_point_cell_bound(geom, taps, uvw, vis, support: int, tile: int = 32, window=None,
                           par: bool = False):
    """Per-cell bound of |G_gpu - G_oracle| for the fixed-point window
    gridders (supports up to 32), from the oracle alone.

    Each commit into a unit's fixed-point region is off by at most half a
    quantum; the quantum is the power of two 2^(e - 30) with B < 2^e, so half
    of it is below 2^-30 B, where B = 2 (1.0001) sum over the unit's records of
    max|weight component| max|visibility component| <= 2.0002 R wmax Vmax;
    a unit's records lie in one tile, so Vmax for cell c can be taken over
    the records whose first cell lies within tile + support of c.  A cell
    receives at most one commit per record whose footprint covers it (a slot
    commits only sums it holds).  The FP32 sums add at most (n_c + 4) 2^-24
    of the sum of the magnitudes of the cell's terms (register accumulation,
    conversion back to FP32, one float atomic per unit).
    window = (u0, v0, wu, wv) restricts the bound to that rectangle; par
    uses the band-parallel oracle (bit-identical).
    Returns (bound [npol, wv, wu], n_c [wv, wu])."""
    from scipy.ndimage import maximum_filter
    vis = np.asarray(vis)
    nrec, npol = vis.shape
    u0, v0, wu, wv = window if window is not None else (0, 0, geom.nu, geom.nv)
    grid_fn = oracle.grid_par if par else oracle.grid
    kind_sep = geom.kind == "separable"
    if kind_sep:
        ones = np.ones(np.asarray(taps).shape, np.float64)
        at = np.abs(np.asarray(taps, np.float64))
        wmax = float(at.max()) ** 2
    else:
        t = np.asarray(taps)
        ones = np.ones(t.shape, np.complex128)
        at = (np.abs(t.real) + np.abs(t.imag)).astype(np.complex128)
        wmax = float(max(np.abs(t.real).max(), np.abs(t.imag).max()))
    count, _ = grid_fn(geom, ones, uvw, np.ones((nrec, 1)), window=(u0, v0, wu, wv))
    n_c = count[0].real
    av = np.abs(vis.real) + np.abs(vis.imag)
    mag, _ = grid_fn(geom, at, uvw, av, window=(u0, v0, wu, wv))
    mag = mag.real
    vmax_rec = np.max(np.maximum(np.abs(vis.real), np.abs(vis.imag)), axis=1)
    ix = oracle.index(geom, uvw)
    reach = tile + support
    ku, kv = ix["k_lo_u"] - (u0 - reach), ix["k_lo_v"] - (v0 - reach)
    ok = (ix["valid"] == 1) & (ku >= 0) & (ku < wu + 2 * reach) & (kv >= 0) & (kv < wv + 2 * reach)
    vmap = np.zeros((wv + 2 * reach, wu + 2 * reach))
    np.maximum.at(vmap, (kv[ok], ku[ok]), vmax_rec[ok])
    # records with first cell in [c - reach, c + reach] on both axes
    vnear = maximum_filter(vmap, size=2 * reach + 1, mode="constant")[reach:reach + wv,
                                                                       reach:reach + wu]
    R = plan_chunk_records(nrec)
    quantum_half = 2.0 ** -30 * 2.0002 * R * wmax * vnear
    bound = n_c[None] * quantum_half[None] + (n_c[None] + 4) * 2.0 ** -24 * mag
    return bound, n_c


def assert_within_cell_bound(G, G_ref, bound, what=""):
    """|G - G_ref| within the bound for every cell, real and imaginary
    parts separately."""
    for part in ("real", "imag"):
        d = np.abs(getattr(G, part) - getattr(G_ref, part))
        bad = d > bound
        assert not bad.any(), (what, part, int(bad.sum()), float((d - bound).max()))
