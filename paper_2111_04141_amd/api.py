"""Python binding of libmigrid (include/migrid.h): argument marshalling only.

Every step of gridding and degridding runs in the HIP library; this module
checks tensor dtypes/devices/shapes, builds the C descriptors and passes raw
device pointers plus torch's current HIP stream.  There is no CPU fallback:
if the library is missing the import of the library raises.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import re
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmigrid.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "migrid.h")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_EDEVICE, MG_EUNSUPPORTED, MG_EBUSY = 0, -1, -2, -3, -4, -5
MG_F32, MG_F64, MG_F16, MG_BF16 = 0, 1, 2, 3
MG_KERNEL_SEPARABLE, MG_KERNEL_WPROJ, MG_KERNEL_WSTACK = 0, 1, 2

_TORCH_TO_MG = {torch.float32: MG_F32, torch.float64: MG_F64, torch.float16: MG_F16,
                torch.bfloat16: MG_BF16}


class MigridError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("nu", C.c_int32), ("nv", C.c_int32), ("npol", C.c_int32), ("beta", C.c_int32),
                ("scale_u", C.c_double), ("scale_v", C.c_double)]


class KernelDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("tap_dtype", C.c_int32), ("support", C.c_int32),
                ("nplanes", C.c_int32), ("plane_support", C.POINTER(C.c_int32)),
                ("plane_offset", C.POINTER(C.c_int64)), ("inv_dw", C.c_double),
                ("taps", C.c_void_p), ("ntaps", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("failed", C.c_uint64), ("bytes_in_use", C.c_uint64), ("bytes_peak", C.c_uint64),
                ("budget", C.c_uint64), ("running", C.c_int32), ("queued", C.c_int32),
                ("max_running", C.c_int32)]


_lib = None


def header_symbols() -> list:
    """Names of the functions declared in include/migrid.h."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_0-9]+)\s*\(", txt)))


def lib():
    """The loaded libmigrid.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2111_04141_amd/build.py "
                          "(there is no fallback path)")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    gd, kd = C.POINTER(GridDesc), C.POINTER(KernelDesc)
    L.mg_status_str.argtypes = [i32]
    L.mg_status_str.restype = C.c_char_p
    L.mg_last_error.argtypes = []
    L.mg_last_error.restype = C.c_char_p
    L.mg_compute_indices.argtypes = [gd, kd, i64, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.mg_plan_workspace_size.argtypes = [gd, kd, i64, C.POINTER(C.c_size_t)]
    L.mg_plan_create.argtypes = [C.POINTER(vp), gd, kd, i64, vp, i32, vp, vp]
    L.mg_plan_grid.argtypes = [vp, vp, vp, vp]
    L.mg_plan_degrid.argtypes = [vp, vp, vp, vp]
    L.mg_plan_nskipped.argtypes = [vp, C.POINTER(i64)]
    L.mg_plan_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.mg_plan_destroy.argtypes = [vp]
    L.mg_grid.argtypes = [gd, kd, i64, vp, i32, vp, vp, vp, vp]
    L.mg_degrid.argtypes = [gd, kd, i64, vp, i32, vp, vp, vp, vp]
    L.mg_grid_static.argtypes = [gd, kd, i64, vp, i32, vp, vp, vp, vp]
    L.mg_hybrid_plan_workspace_size.argtypes = [gd, kd, i64, C.POINTER(C.c_size_t)]
    L.mg_hybrid_plan_create.argtypes = [C.POINTER(vp), gd, kd, i64, vp, i32, vp, vp]
    L.mg_hybrid_plan_grid.argtypes = [vp, vp, vp, vp]
    L.mg_hybrid_plan_nskipped.argtypes = [vp, C.POINTER(i64)]
    L.mg_hybrid_plan_destroy.argtypes = [vp]
    L.mg_hybrid_grid.argtypes = [gd, kd, i64, vp, i32, vp, vp, vp, vp]
    L.mg_prune_columns.argtypes = [i32, i64, i32, i32, i32, vp, vp, vp, vp]
    L.mg_corrector.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp]
    L.mg_imager_create.argtypes = [C.POINTER(vp), i32, i32, i32]
    L.mg_imager_exec.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, vp]
    L.mg_imager_destroy.argtypes = [vp]
    L.mg_wkernel_bank_size.argtypes = [i32, vp, i32, C.POINTER(i64), C.POINTER(C.c_size_t)]
    L.mg_wkernel_bank.argtypes = [i32, vp, vp, i32, i32, vp, C.c_double, i32, vp, vp, vp,
                                  C.c_size_t, vp]
    L.mg_wstack_imager_create.argtypes = [C.POINTER(vp), i32, i32, i32, i32]
    L.mg_wstack_imager_exec.argtypes = [vp, vp, vp, vp, vp, vp, C.c_double, C.c_double,
                                        C.c_double, vp]
    L.mg_wstack_imager_destroy.argtypes = [vp]
    L.mg_grid_static_capacity.argtypes = []
    L.mg_grid_static_capacity.restype = C.c_size_t
    L.mg_server_create.argtypes = [C.POINTER(vp), C.c_size_t, i32, i32, i32]
    L.mg_server_submit.argtypes = [vp, gd, kd, i64, vp, i32, vp, vp, vp, C.POINTER(C.c_uint64)]
    L.mg_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(i32), C.POINTER(C.c_double)]
    L.mg_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(C.c_double)]
    L.mg_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
    L.mg_server_destroy.argtypes = [vp]
    for f in ("mg_compute_indices", "mg_plan_workspace_size", "mg_plan_create",
              "mg_plan_grid", "mg_plan_degrid",
              "mg_plan_nskipped", "mg_plan_bytes", "mg_plan_destroy", "mg_grid", "mg_degrid",
              "mg_grid_static", "mg_hybrid_plan_workspace_size", "mg_hybrid_plan_create",
              "mg_hybrid_plan_grid", "mg_hybrid_plan_nskipped", "mg_hybrid_plan_destroy",
              "mg_hybrid_grid", "mg_prune_columns", "mg_corrector", "mg_imager_create",
              "mg_imager_exec", "mg_imager_destroy", "mg_wkernel_bank_size", "mg_wkernel_bank",
              "mg_wstack_imager_create", "mg_wstack_imager_exec", "mg_wstack_imager_destroy",
              "mg_server_create", "mg_server_submit", "mg_server_poll", "mg_server_wait",
              "mg_server_get_stats", "mg_server_destroy"):
        getattr(L, f).restype = i32
    _lib = L
    return L


def _check(status: int, where: str):
    if status != MG_OK:
        L = lib()
        raise MigridError(status, where, L.mg_last_error().decode() or
                          L.mg_status_str(status).decode())


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ---------------------------------------------------------------------------
# descriptors
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class GridSpec:
    """nu x nv grid, npol polarisations, oversampling beta, cells per
    wavelength scale_u / scale_v (origin at cell (nu/2, nv/2))."""
    nu: int
    nv: int
    npol: int = 4
    beta: int = 8
    scale_u: float = 1.0
    scale_v: float = 1.0

    def desc(self) -> GridDesc:
        return GridDesc(self.nu, self.nv, self.npol, self.beta, float(self.scale_u),
                        float(self.scale_v))


class KernelBank:
    """A kernel table resident on the device.

    separable: taps real [beta*S + 1] (float32 / float16 / bfloat16).
    wproj: taps complex, concatenated planes [sum (beta*S_p+1)^2]; given as a
    complex64 tensor or as a [..., 2] float16 / bfloat16 tensor.
    wstack: W-stacking, separable taps as above plus `layers` layers of
    spacing 1 / inv_dw; grids are [npol, layers, nv, nu].
    """

    def __init__(self, kind: str, taps: torch.Tensor, support: int = 0,
                 plane_support: Sequence[int] = (), plane_offset: Sequence[int] = (),
                 inv_dw: float = 0.0, layers: int = 0):
        if kind not in ("separable", "wproj", "wstack"):
            raise ValueError("kind must be 'separable', 'wproj' or 'wstack'")
        if not taps.is_cuda:
            raise ValueError("taps must be a device tensor")
        taps = taps.contiguous()
        if kind == "wproj":
            if taps.dtype == torch.complex64:
                tdt, nt = MG_F32, taps.numel()
            elif taps.dtype in (torch.float16, torch.bfloat16) and taps.shape[-1] == 2:
                tdt, nt = _TORCH_TO_MG[taps.dtype], taps.numel() // 2
            else:
                raise ValueError("wproj taps: complex64, or [..., 2] float16/bfloat16")
        else:
            if taps.dtype not in (torch.float32, torch.float16, torch.bfloat16):
                raise ValueError("separable taps: float32, float16 or bfloat16")
            tdt, nt = _TORCH_TO_MG[taps.dtype], taps.numel()
        self.kind = kind
        self.taps = taps
        self.tap_dtype = tdt
        self.ntaps = nt
        self.support = int(support)
        self._ps = (C.c_int32 * max(1, len(plane_support)))(*[int(s) for s in plane_support])
        self._po = (C.c_int64 * max(1, len(plane_offset)))(*[int(o) for o in plane_offset])
        self.plane_support = [int(s) for s in plane_support]
        self.plane_offset = [int(o) for o in plane_offset]
        self.inv_dw = float(inv_dw)
        self.layers = int(layers) if kind == "wstack" else 0
        if kind == "wstack" and self.layers < 1:
            raise ValueError("wstack needs layers >= 1")

    @property
    def support_max(self) -> int:
        return self.support if self.kind != "wproj" else max(self.plane_support)

    def desc(self) -> KernelDesc:
        d = KernelDesc()
        d.kind = {"separable": MG_KERNEL_SEPARABLE, "wproj": MG_KERNEL_WPROJ,
                  "wstack": MG_KERNEL_WSTACK}[self.kind]
        d.tap_dtype = self.tap_dtype
        d.support = self.support
        d.nplanes = self.layers if self.kind == "wstack" else len(self.plane_support)
        d.plane_support = C.cast(self._ps, C.POINTER(C.c_int32))
        d.plane_offset = C.cast(self._po, C.POINTER(C.c_int64))
        d.inv_dw = self.inv_dw
        d.taps = self.taps.data_ptr()
        d.ntaps = self.ntaps
        return d


def _check_uvw(uvw: torch.Tensor) -> int:
    if not uvw.is_cuda or uvw.dim() != 2 or uvw.shape[1] != 3 or not uvw.is_contiguous():
        raise ValueError("uvw must be a contiguous [nrec, 3] device tensor")
    if uvw.dtype not in (torch.float32, torch.float64):
        raise ValueError("uvw must be float32 or float64")
    return _TORCH_TO_MG[uvw.dtype]


def _check_vis(vis: torch.Tensor, nrec: int, npol: int):
    if (not vis.is_cuda or vis.dtype != torch.complex64 or not vis.is_contiguous()
            or tuple(vis.shape) != (nrec, npol)):
        raise ValueError(f"vis must be a contiguous complex64 [{nrec}, {npol}] device tensor")


def grid_shape(spec: GridSpec, bank: Optional["KernelBank"] = None) -> tuple:
    """Shape of the grid a call with this bank reads or writes: [npol, nv,
    nu], or [npol, layers, nv, nu] for W-stacking."""
    if bank is not None and bank.kind == "wstack":
        return (spec.npol, bank.layers, spec.nv, spec.nu)
    return (spec.npol, spec.nv, spec.nu)


def _check_grid(g: torch.Tensor, spec: GridSpec, bank: Optional["KernelBank"] = None):
    shape = grid_shape(spec, bank)
    if (not g.is_cuda or g.dtype != torch.complex64 or not g.is_contiguous()
            or tuple(g.shape) != shape):
        raise ValueError(f"grid must be a contiguous complex64 {list(shape)} device tensor")


# ---------------------------------------------------------------------------
# calls
# ---------------------------------------------------------------------------

def compute_indices(spec: GridSpec, bank: KernelBank, uvw: torch.Tensor) -> dict:
    """Per-record integer indices (k_lo_u, k_lo_v, o_u, o_v, plane, valid) and
    the skipped count, in input order."""
    dt = _check_uvw(uvw)
    n = uvw.shape[0]
    dev = uvw.device
    out = {k: torch.empty(n, dtype=torch.int32, device=dev)
           for k in ("k_lo_u", "k_lo_v", "o_u", "o_v", "plane")}
    out["valid"] = torch.empty(n, dtype=torch.uint8, device=dev)
    nsk = torch.zeros(1, dtype=torch.int64, device=dev)
    gd, kd = spec.desc(), bank.desc()
    _check(lib().mg_compute_indices(C.byref(gd), C.byref(kd), n, uvw.data_ptr(), dt,
                                    *[out[k].data_ptr() for k in ("k_lo_u", "k_lo_v", "o_u",
                                                                  "o_v", "plane", "valid")],
                                    nsk.data_ptr(), _stream_ptr(dev)), "mg_compute_indices")
    out["nskipped"] = nsk
    return out


def grid(spec: GridSpec, bank: KernelBank, uvw: torch.Tensor, vis: torch.Tensor,
         out: Optional[torch.Tensor] = None, nskipped: Optional[torch.Tensor] = None):
    """One-shot gridding (index + sort + grid): out += G vis."""
    dt = _check_uvw(uvw)
    n = uvw.shape[0]
    _check_vis(vis, n, spec.npol)
    if out is None:
        out = torch.zeros(grid_shape(spec, bank), dtype=torch.complex64, device=uvw.device)
    _check_grid(out, spec, bank)
    gd, kd = spec.desc(), bank.desc()
    _check(lib().mg_grid(C.byref(gd), C.byref(kd), n, uvw.data_ptr(), dt, vis.data_ptr(),
                         out.data_ptr(), _ptr(nskipped), _stream_ptr(uvw.device)), "mg_grid")
    return out


def grid_static(spec: GridSpec, bank: KernelBank, uvw: torch.Tensor, vis: torch.Tensor,
                out: Optional[torch.Tensor] = None, nskipped: Optional[torch.Tensor] = None):
    """One-shot gridding that allocates no device memory in the library
    (mg_grid_static: scratch from a static array of static_capacity() bytes;
    calls on one GPU must not overlap): out += G vis."""
    dt = _check_uvw(uvw)
    n = uvw.shape[0]
    _check_vis(vis, n, spec.npol)
    if out is None:
        out = torch.zeros(grid_shape(spec, bank), dtype=torch.complex64, device=uvw.device)
    _check_grid(out, spec, bank)
    gd, kd = spec.desc(), bank.desc()
    _check(lib().mg_grid_static(C.byref(gd), C.byref(kd), n, uvw.data_ptr(), dt, vis.data_ptr(),
                                out.data_ptr(), _ptr(nskipped), _stream_ptr(uvw.device)),
           "mg_grid_static")
    return out


def static_capacity() -> int:
    """Bytes of the static scratch behind grid_static."""
    return int(lib().mg_grid_static_capacity())


def degrid(spec: GridSpec, bank: KernelBank, uvw: torch.Tensor, grid_in: torch.Tensor,
           out: Optional[torch.Tensor] = None, nskipped: Optional[torch.Tensor] = None):
    """One-shot degridding: returns vis = G^H grid (skipped records get 0)."""
    dt = _check_uvw(uvw)
    n = uvw.shape[0]
    _check_grid(grid_in, spec, bank)
    if out is None:
        out = torch.empty(n, spec.npol, dtype=torch.complex64, device=uvw.device)
    _check_vis(out, n, spec.npol)
    gd, kd = spec.desc(), bank.desc()
    _check(lib().mg_degrid(C.byref(gd), C.byref(kd), n, uvw.data_ptr(), dt, grid_in.data_ptr(),
                           out.data_ptr(), _ptr(nskipped), _stream_ptr(uvw.device)), "mg_degrid")
    return out


class Server:
    """Continuous-batching gridding server (mg_server_*): jobs are admitted in
    arrival order as slots and HBM budget free up and run on a pool of
    streams, so jobs that arrive while others run overlap on the device.
    Every tensor of a job must stay alive until the job is done."""

    JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, nstreams: int = 8,
                 device: int = -1):
        self._h = C.c_void_p()
        _check(lib().mg_server_create(C.byref(self._h), int(hbm_budget_bytes), int(max_slots),
                                      int(nstreams), int(device)), "mg_server_create")
        self._keep = {}

    def submit(self, spec: GridSpec, bank: KernelBank, uvw: torch.Tensor, vis: torch.Tensor,
               grid_out: torch.Tensor) -> int:
        dt = _check_uvw(uvw)
        n = uvw.shape[0]
        _check_vis(vis, n, spec.npol)
        _check_grid(grid_out, spec, bank)
        # inputs are produced on torch's current stream: the job's stream waits
        # for an event recorded there (no host synchronisation)
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(uvw.device))
        gd, kd = spec.desc(), bank.desc()
        jid = C.c_uint64()
        _check(lib().mg_server_submit(self._h, C.byref(gd), C.byref(kd), n, uvw.data_ptr(), dt,
                                      vis.data_ptr(), grid_out.data_ptr(), ev.cuda_event,
                                      C.byref(jid)), "mg_server_submit")
        self._keep[jid.value] = (uvw, vis, grid_out, bank)
        return jid.value

    def poll(self, job: int):
        st, lat = C.c_int32(), C.c_double()
        _check(lib().mg_server_poll(self._h, job, C.byref(st), C.byref(lat)), "mg_server_poll")
        return st.value, lat.value

    def wait(self, job: int) -> float:
        lat = C.c_double()
        _check(lib().mg_server_wait(self._h, job, C.byref(lat)), "mg_server_wait")
        self._keep.pop(job, None)
        return lat.value

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().mg_server_get_stats(self._h, C.byref(s)), "mg_server_get_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib().mg_server_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def workspace_size(spec: GridSpec, bank: KernelBank, nrec: int) -> int:
    """Device bytes a plan of nrec records holds (mg_plan_workspace_size)."""
    gd, kd = spec.desc(), bank.desc()
    v = C.c_size_t()
    _check(lib().mg_plan_workspace_size(C.byref(gd), C.byref(kd), int(nrec), C.byref(v)),
           "mg_plan_workspace_size")
    return int(v.value)


class Plan:
    """Index + sort once; grid / degrid many times over the same records.
    The plan's device arrays live in a torch-allocated workspace."""

    def __init__(self, spec: GridSpec, bank: KernelBank, uvw: torch.Tensor):
        dt = _check_uvw(uvw)
        self.spec, self.bank = spec, bank
        self.nrec = uvw.shape[0]
        self.device = uvw.device
        self._h = C.c_void_p()
        gd, kd = spec.desc(), bank.desc()
        # the plan's device memory is a torch allocation (the caching
        # allocator accounts for it); it outlives the plan handle
        self.workspace = torch.empty(workspace_size(spec, bank, self.nrec), dtype=torch.uint8,
                                     device=uvw.device)
        _check(lib().mg_plan_create(C.byref(self._h), C.byref(gd), C.byref(kd), self.nrec,
                                    uvw.data_ptr(), dt, self.workspace.data_ptr(),
                                    _stream_ptr(uvw.device)), "mg_plan_create")

    def grid(self, vis: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _check_vis(vis, self.nrec, self.spec.npol)
        if out is None:
            out = torch.zeros(grid_shape(self.spec, self.bank), dtype=torch.complex64,
                              device=self.device)
        _check_grid(out, self.spec, self.bank)
        _check(lib().mg_plan_grid(self._h, vis.data_ptr(), out.data_ptr(),
                                  _stream_ptr(self.device)), "mg_plan_grid")
        return out

    def degrid(self, grid_in: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _check_grid(grid_in, self.spec, self.bank)
        if out is None:
            out = torch.empty(self.nrec, self.spec.npol, dtype=torch.complex64,
                              device=self.device)
        _check_vis(out, self.nrec, self.spec.npol)
        _check(lib().mg_plan_degrid(self._h, grid_in.data_ptr(), out.data_ptr(),
                                    _stream_ptr(self.device)), "mg_plan_degrid")
        return out

    @property
    def nskipped(self) -> int:
        v = C.c_int64()
        _check(lib().mg_plan_nskipped(self._h, C.byref(v)), "mg_plan_nskipped")
        return int(v.value)

    @property
    def nbytes(self) -> int:
        v = C.c_size_t()
        _check(lib().mg_plan_bytes(self._h, C.byref(v)), "mg_plan_bytes")
        return int(v.value)

    def close(self):
        if self._h:
            lib().mg_plan_destroy(self._h)
            self._h = C.c_void_p()
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------------------
# Hybrid Gridding and column pruning
# ---------------------------------------------------------------------------

def _check_hybrid_grid(g: torch.Tensor, spec: GridSpec):
    shape = (spec.npol, spec.beta * spec.nv, spec.nu)
    if (not g.is_cuda or g.dtype != torch.complex64 or not g.is_contiguous()
            or tuple(g.shape) != shape):
        raise ValueError(f"hybrid grid must be a contiguous complex64 {list(shape)} device tensor")


def hybrid_grid(spec: GridSpec, bank: KernelBank, uvw: torch.Tensor, vis: torch.Tensor,
                out: Optional[torch.Tensor] = None, nskipped: Optional[torch.Tensor] = None):
    """One-shot Hybrid Gridding Step: out [npol, beta nv, nu] += G_hy vis."""
    dt = _check_uvw(uvw)
    n = uvw.shape[0]
    _check_vis(vis, n, spec.npol)
    if out is None:
        out = torch.zeros(spec.npol, spec.beta * spec.nv, spec.nu, dtype=torch.complex64,
                          device=uvw.device)
    _check_hybrid_grid(out, spec)
    gd, kd = spec.desc(), bank.desc()
    _check(lib().mg_hybrid_grid(C.byref(gd), C.byref(kd), n, uvw.data_ptr(), dt, vis.data_ptr(),
                                out.data_ptr(), _ptr(nskipped), _stream_ptr(uvw.device)),
           "mg_hybrid_grid")
    return out


class HybridPlan:
    """Bin the records once by tile of the hybrid grid, then run the Hybrid
    Gridding Step many times; the plan's memory is a torch workspace."""

    def __init__(self, spec: GridSpec, bank: KernelBank, uvw: torch.Tensor):
        dt = _check_uvw(uvw)
        self.spec, self.bank = spec, bank
        self.nrec = uvw.shape[0]
        self.device = uvw.device
        gd, kd = spec.desc(), bank.desc()
        v = C.c_size_t()
        _check(lib().mg_hybrid_plan_workspace_size(C.byref(gd), C.byref(kd), self.nrec,
                                                   C.byref(v)), "mg_hybrid_plan_workspace_size")
        self.workspace = torch.empty(int(v.value), dtype=torch.uint8, device=uvw.device)
        self._h = C.c_void_p()
        _check(lib().mg_hybrid_plan_create(C.byref(self._h), C.byref(gd), C.byref(kd), self.nrec,
                                           uvw.data_ptr(), dt, self.workspace.data_ptr(),
                                           _stream_ptr(uvw.device)), "mg_hybrid_plan_create")

    def grid(self, vis: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _check_vis(vis, self.nrec, self.spec.npol)
        if out is None:
            out = torch.zeros(self.spec.npol, self.spec.beta * self.spec.nv, self.spec.nu,
                              dtype=torch.complex64, device=self.device)
        _check_hybrid_grid(out, self.spec)
        _check(lib().mg_hybrid_plan_grid(self._h, vis.data_ptr(), out.data_ptr(),
                                         _stream_ptr(self.device)), "mg_hybrid_plan_grid")
        return out

    @property
    def nskipped(self) -> int:
        v = C.c_int64()
        _check(lib().mg_hybrid_plan_nskipped(self._h, C.byref(v)), "mg_hybrid_plan_nskipped")
        return int(v.value)

    def close(self):
        if self._h:
            lib().mg_hybrid_plan_destroy(self._h)
            self._h = C.c_void_p()
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def prune_columns(grid_in: torch.Tensor, alpha: int, ztaps: torch.Tensor, support_z: int,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Column pruning: every column of grid_in [npol, M, ncols] circularly
    convolved with the pruning kernel (FP32 device table of alpha Sz + 1
    values) and downsampled by alpha; returns [npol, M / alpha, ncols]."""
    if (not grid_in.is_cuda or grid_in.dtype != torch.complex64 or not grid_in.is_contiguous()
            or grid_in.dim() != 3):
        raise ValueError("grid_in must be a contiguous complex64 [npol, M, ncols] device tensor")
    npol, M, ncols = grid_in.shape
    if (not ztaps.is_cuda or ztaps.dtype != torch.float32 or not ztaps.is_contiguous()
            or ztaps.numel() < alpha * support_z + 1):
        raise ValueError("ztaps must be a contiguous float32 device tensor of alpha*Sz+1 values")
    if out is None:
        out = torch.empty(npol, M // alpha, ncols, dtype=torch.complex64, device=grid_in.device)
    if (not out.is_contiguous() or out.dtype != torch.complex64
            or tuple(out.shape) != (npol, M // alpha, ncols)):
        raise ValueError("out must be a contiguous complex64 [npol, M/alpha, ncols] tensor")
    _check(lib().mg_prune_columns(npol, M, ncols, int(alpha), int(support_z), ztaps.data_ptr(),
                                  grid_in.data_ptr(), out.data_ptr(),
                                  _stream_ptr(grid_in.device)), "mg_prune_columns")
    return out


# ---------------------------------------------------------------------------
# imaging chain
# ---------------------------------------------------------------------------

def corrector(n: int, beta: int, table: torch.Tensor, phases: int,
              nn_sinc: bool = True) -> torch.Tensor:
    """Corrector vector h(l), l = (i - n/2)/n (mg_corrector); table: FP32
    device tensor of E + 1 symmetric values spaced 1/beta cells."""
    if not table.is_cuda or table.dtype != torch.float32 or not table.is_contiguous():
        raise ValueError("table must be a contiguous float32 device tensor")
    out = torch.empty(n, dtype=torch.float32, device=table.device)
    _check(lib().mg_corrector(int(n), int(beta), table.numel(), int(phases), int(nn_sinc),
                              table.data_ptr(), out.data_ptr(), _stream_ptr(table.device)),
           "mg_corrector")
    return out


class Imager:
    """Origin shift + batched inverse FFT + separable correction of centred
    [npol, ny, nx] grids (mg_imager_*)."""

    def __init__(self, npol: int, nx: int, ny: int, device="cuda"):
        self.npol, self.nx, self.ny = int(npol), int(nx), int(ny)
        self.device = torch.device(device)
        self._h = C.c_void_p()
        _check(lib().mg_imager_create(C.byref(self._h), self.npol, self.nx, self.ny),
               "mg_imager_create")
        self.work = torch.empty(self.npol, self.ny, self.nx, dtype=torch.complex64,
                                device=self.device)

    def image(self, grid: torch.Tensor, corr_x: torch.Tensor, corr_y: torch.Tensor,
              y0: int = 0, out_ny: Optional[int] = None,
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out_ny = self.ny if out_ny is None else int(out_ny)
        if (grid.dtype != torch.complex64 or not grid.is_contiguous()
                or tuple(grid.shape) != (self.npol, self.ny, self.nx)):
            raise ValueError(f"grid must be complex64 [{self.npol}, {self.ny}, {self.nx}]")
        if corr_x.numel() != self.nx or corr_y.numel() != out_ny:
            raise ValueError("corrector lengths must be nx and out_ny")
        if out is None:
            out = torch.empty(self.npol, out_ny, self.nx, dtype=torch.complex64,
                              device=self.device)
        _check(lib().mg_imager_exec(self._h, grid.data_ptr(), self.work.data_ptr(),
                                    out.data_ptr(), corr_x.data_ptr(), corr_y.data_ptr(),
                                    int(y0), out_ny, _stream_ptr(self.device)),
               "mg_imager_exec")
        return out

    def close(self):
        if self._h:
            lib().mg_imager_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# kernel generation
# ---------------------------------------------------------------------------

def wkernel_bank(plane_support: Sequence[int], plane_w: Sequence[float], beta: int,
                 base_taps: torch.Tensor, fov: float, dtype: str = "f32"):
    """W-projection kernel bank built on the device (mg_wkernel_bank).

    base_taps: float64 device tensor of the separable GCF's beta*S0 + 1
    taps; plane_support / plane_w: per-plane support and w (wavelengths);
    fov: radians spanned by the grid's field.  Returns (taps, offsets):
    taps a device tensor of the bank (complex64 for "f32", [n, 2] float16
    or bfloat16 pairs for "f16" / "bf16"), offsets the planes' element
    offsets (list), ready for KernelBank("wproj", ...)."""
    if (not base_taps.is_cuda or base_taps.dtype != torch.float64
            or not base_taps.is_contiguous() or base_taps.dim() != 1):
        raise ValueError("base_taps must be a contiguous float64 device vector")
    np_ = len(plane_support)
    if len(plane_w) != np_:
        raise ValueError("plane_support and plane_w must have the same length")
    sup = (C.c_int32 * np_)(*[int(x) for x in plane_support])
    ws = (C.c_double * np_)(*[float(x) for x in plane_w])
    n = C.c_int64()
    wb = C.c_size_t()
    L = lib()
    _check(L.mg_wkernel_bank_size(np_, sup, int(beta), C.byref(n), C.byref(wb)),
           "mg_wkernel_bank_size")
    dev = base_taps.device
    if dtype == "f32":
        bank = torch.empty(n.value, dtype=torch.complex64, device=dev)
        code = MG_F32
    elif dtype in ("f16", "bf16"):
        bank = torch.empty(n.value, 2, dtype=torch.float16 if dtype == "f16" else torch.bfloat16,
                           device=dev)
        code = MG_F16 if dtype == "f16" else MG_BF16
    else:
        raise ValueError("dtype must be f32, f16 or bf16")
    work = torch.empty(wb.value, dtype=torch.uint8, device=dev)
    offs = (C.c_int64 * np_)()
    _check(L.mg_wkernel_bank(np_, sup, ws, int(beta), base_taps.numel(), base_taps.data_ptr(),
                             float(fov), code, bank.data_ptr(), offs, work.data_ptr(), wb.value,
                             _stream_ptr(dev)), "mg_wkernel_bank")
    return bank, [int(x) for x in offs]


# ---------------------------------------------------------------------------
# W-stacking image
# ---------------------------------------------------------------------------

class WStackImager:
    """Image of W-stacking layer grids [npol, layers, ny, nx]: per-layer
    inverse FFT, inverse W-term screen of each layer, sum, separable
    correction (mg_wstack_imager_*)."""

    def __init__(self, npol: int, layers: int, nx: int, ny: int, device="cuda"):
        self.npol, self.layers, self.nx, self.ny = int(npol), int(layers), int(nx), int(ny)
        self.device = torch.device(device)
        self._h = C.c_void_p()
        _check(lib().mg_wstack_imager_create(C.byref(self._h), self.npol, self.layers, self.nx,
                                             self.ny), "mg_wstack_imager_create")
        self.work = torch.empty(self.npol, self.layers, self.ny, self.nx, dtype=torch.complex64,
                                device=self.device)

    def image(self, grids: torch.Tensor, corr_x: torch.Tensor, corr_y: torch.Tensor,
              fov_x: float, fov_y: float, dw: float,
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
        shape = (self.npol, self.layers, self.ny, self.nx)
        if grids.dtype != torch.complex64 or not grids.is_contiguous() or tuple(grids.shape) != shape:
            raise ValueError(f"grids must be complex64 {list(shape)}")
        if corr_x.numel() != self.nx or corr_y.numel() != self.ny:
            raise ValueError("corrector lengths must be nx and ny")
        if out is None:
            out = torch.empty(self.npol, self.ny, self.nx, dtype=torch.complex64,
                              device=self.device)
        _check(lib().mg_wstack_imager_exec(self._h, grids.data_ptr(), self.work.data_ptr(),
                                           out.data_ptr(), corr_x.data_ptr(), corr_y.data_ptr(),
                                           float(fov_x), float(fov_y), float(dw),
                                           _stream_ptr(self.device)), "mg_wstack_imager_exec")
        return out

    def close(self):
        if self._h:
            lib().mg_wstack_imager_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
