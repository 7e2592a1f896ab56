"""The C-ABI library loads, exports every function include/migrid.h
declares, and rejects bad arguments on the host before touching a device.
(No compute calls: these run without a GPU.)"""
import ctypes as C
import os

import pytest

from paper_2111_04141_amd import api


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(api.LIB_PATH):
        pytest.fail("libmigrid.so is not built (run __graft_entry__.build())")
    return api.lib()


def test_exports_every_header_symbol(L):
    names = api.header_symbols()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    assert L.mg_status_str(0) == b"ok"
    assert L.mg_status_str(-1) == b"invalid argument"
    assert L.mg_status_str(-4) == b"unsupported"


def _descs(**kw):
    g = api.GridDesc(kw.get("nu", 64), kw.get("nv", 64), kw.get("npol", 4), kw.get("beta", 8),
                     kw.get("scale", 1.0), kw.get("scale", 1.0))
    k = api.KernelDesc()
    k.kind = kw.get("kind", api.MG_KERNEL_SEPARABLE)
    k.tap_dtype = kw.get("tap_dtype", api.MG_F32)
    k.support = kw.get("support", 7)
    k.nplanes = kw.get("nplanes", 0)
    ps = (C.c_int32 * 4)(*kw.get("ps", [8, 8, 8, 8]))
    po = (C.c_int64 * 4)(*kw.get("po", [0, 0, 0, 0]))
    k.plane_support = C.cast(ps, C.POINTER(C.c_int32))
    k.plane_offset = C.cast(po, C.POINTER(C.c_int64))
    k.inv_dw = kw.get("inv_dw", 1.0)
    k.taps = kw.get("taps", 0x1000)
    k.ntaps = kw.get("ntaps", 57)
    return g, k, (ps, po)


BAD = [
    dict(nu=0), dict(nv=70000), dict(npol=0), dict(npol=5), dict(beta=0), dict(beta=300),
    dict(scale=float("nan")), dict(support=0), dict(support=65), dict(beta=3, support=7, ntaps=22),
    dict(ntaps=56), dict(tap_dtype=api.MG_F64), dict(taps=0),
    dict(kind=api.MG_KERNEL_WPROJ, nplanes=0),
    dict(kind=api.MG_KERNEL_WPROJ, nplanes=200),
    dict(kind=api.MG_KERNEL_WPROJ, nplanes=2, ps=[8, 66, 8, 8], ntaps=10 ** 6),
    dict(kind=api.MG_KERNEL_WPROJ, nplanes=2, ps=[8, 8, 8, 8], po=[0, 1000], ntaps=1100),
    dict(kind=api.MG_KERNEL_WPROJ, nplanes=1, inv_dw=-1.0, ntaps=10 ** 6),
    dict(kind=7),
]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_arguments_rejected_on_host(L, bad):
    g, k, keep = _descs(**bad)
    st = L.mg_grid(C.byref(g), C.byref(k), 10, 0x2000, api.MG_F32, 0x3000, 0x4000, None, None)
    assert st == api.MG_EINVAL, (bad, L.mg_last_error())
    assert L.mg_last_error() != b""
    st = L.mg_degrid(C.byref(g), C.byref(k), 10, 0x2000, api.MG_F32, 0x3000, 0x4000, None, None)
    assert st == api.MG_EINVAL
    h = C.c_void_p()
    st = L.mg_plan_create(C.byref(h), C.byref(g), C.byref(k), 10, 0x2000, api.MG_F32, None, None)
    assert st == api.MG_EINVAL and not h.value
    nb = C.c_size_t(123)
    assert L.mg_plan_workspace_size(C.byref(g), C.byref(k), 10, C.byref(nb)) == api.MG_EINVAL
    assert nb.value == 0


def test_null_pointers_and_counts(L):
    g, k, keep = _descs()
    assert L.mg_grid(None, C.byref(k), 1, 0x2000, 0, 0x3000, 0x4000, None, None) == api.MG_EINVAL
    assert L.mg_grid(C.byref(g), None, 1, 0x2000, 0, 0x3000, 0x4000, None, None) == api.MG_EINVAL
    assert L.mg_grid(C.byref(g), C.byref(k), 1, None, 0, 0x3000, 0x4000, None, None) == api.MG_EINVAL
    assert L.mg_grid(C.byref(g), C.byref(k), 1, 0x2000, 0, None, 0x4000, None, None) == api.MG_EINVAL
    assert L.mg_grid(C.byref(g), C.byref(k), 1, 0x2000, 0, 0x3000, None, None, None) == api.MG_EINVAL
    assert L.mg_grid(C.byref(g), C.byref(k), -1, 0x2000, 0, 0x3000, 0x4000, None, None) == api.MG_EINVAL
    assert L.mg_grid(C.byref(g), C.byref(k), 2 ** 31, 0x2000, 0, 0x3000, 0x4000, None, None) == api.MG_EINVAL
    assert L.mg_grid(C.byref(g), C.byref(k), 1, 0x2000, 2, 0x3000, 0x4000, None, None) == api.MG_EINVAL
    assert L.mg_plan_grid(None, 0x1, 0x2, None) == api.MG_EINVAL
    assert L.mg_plan_degrid(None, 0x1, 0x2, None) == api.MG_EINVAL
    assert L.mg_plan_destroy(None) == api.MG_OK
    assert L.mg_compute_indices(C.byref(g), C.byref(k), 5, 0x2000, 0, None, None, None, None,
                                None, None, None, None) == api.MG_EINVAL


def test_python_binding_rejects_host_tensors():
    import torch
    with pytest.raises(ValueError):
        api.KernelBank("separable", torch.zeros(57), support=7)
    with pytest.raises(ValueError):
        api._check_uvw(torch.zeros(4, 3))


def test_server_argument_checks_on_host(L):
    h = C.c_void_p()
    assert L.mg_server_create(None, 1 << 30, 4, 2, -1) == api.MG_EINVAL
    assert L.mg_server_create(C.byref(h), 0, 4, 2, -1) == api.MG_EINVAL
    assert L.mg_server_create(C.byref(h), 1 << 30, 0, 2, -1) == api.MG_EINVAL
    assert L.mg_server_create(C.byref(h), 1 << 30, 4, 0, -1) == api.MG_EINVAL
    assert L.mg_server_create(C.byref(h), 1 << 30, 4, 65, -1) == api.MG_EINVAL
    assert not h.value
    assert L.mg_server_submit(None, None, None, 0, None, 0, None, None, None, None) == api.MG_EINVAL
    assert L.mg_server_destroy(None) == api.MG_OK


def _workspace_bytes(L, **kw):
    g, k, keep = _descs(**kw)
    nb = C.c_size_t()
    st = L.mg_plan_workspace_size(C.byref(g), C.byref(k), kw.get("nrec", 1000), C.byref(nb))
    assert st == api.MG_OK, L.mg_last_error()
    return nb.value


def test_plan_workspace_size_on_host(L):
    """The workspace size is a host computation: it grows with the record
    count (at least 12 bytes of sorted metadata and permutation per record)
    and with the grid (bucket arrays), and is a multiple of the 256-byte
    alignment of its arrays."""
    a = _workspace_bytes(L, nrec=1000)
    b = _workspace_bytes(L, nrec=101000)
    c = _workspace_bytes(L, nrec=1000, nu=4096, nv=4096)
    assert a % 256 == 0 and b % 256 == 0
    assert b - a >= 12 * 100000
    assert c > a
    w = _workspace_bytes(L, kind=api.MG_KERNEL_WPROJ, nplanes=2, ps=[8, 16, 8, 8],
                         po=[0, 33 * 33], ntaps=33 * 33 + 65 * 65, beta=4, nrec=1000)
    assert w > 2 * 8 * (33 * 33 + 65 * 65)      # the tap table and its conjugate
