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
