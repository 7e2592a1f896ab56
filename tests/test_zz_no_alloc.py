"""mg_grid_static, the one-shot gridding entry point that allocates nothing
(its plan and scratch live in a static device array inside the library),
against mg_grid, the entry point it is a variant of: two calls in a row,
the second with fewer records on a smaller grid, each within relative L2
1e-5 of mg_grid with the same skipped count; an input too large for the
static array is refused before anything is queued."""
import ctypes as C

import numpy as np
import pytest

from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _call(api, fn, spec, bank, uvw, vis, out, nsk, torch):
    gd, kd = spec.desc(), bank.desc()
    dt = api.MG_F64 if uvw.dtype == torch.float64 else api.MG_F32
    return getattr(api.lib(), fn)(C.byref(gd), C.byref(kd), uvw.shape[0], uvw.data_ptr(), dt,
                                  vis.data_ptr(), out.data_ptr(), nsk.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)


def test_static_entry_point_matches_mg_grid_twice_and_refuses_oversize():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api
    L = api.lib()
    assert L.mg_grid_static_capacity() == 64 << 20
    wl = W.config_small()
    rng = np.random.Generator(np.random.PCG64(41))
    uvw_all = np.concatenate([wl.uvw, [[np.nan, 0.0, 0.0], [1e9, 0.0, 0.0]]])
    vis_all = W.vis_normal(uvw_all.shape[0], 4, seed=42)
    cases = [(wl.n, uvw_all, vis_all)]
    # second call: fewer records, smaller grid (the array keeps the first
    # call's contents; everything that must start at zero is cleared)
    sel = np.sort(rng.choice(wl.nrec, 20000, replace=False))
    cases.append((512, wl.uvw[sel], vis_all[sel]))
    for n, uvw_h, vis_h in cases:
        scale = 0.5 * (n / 2 - wl.support) / float(np.abs(wl.uvw[:, :2]).max())
        spec = api.GridSpec(n, n, 4, wl.beta, scale, scale)
        bank = H.device_bank(wl)
        uvw = torch.from_numpy(np.ascontiguousarray(uvw_h)).cuda()
        vis = torch.from_numpy(np.ascontiguousarray(vis_h)).cuda()
        ref = torch.zeros(4, n, n, dtype=torch.complex64, device="cuda")
        got = torch.zeros_like(ref)
        nsk_ref = torch.zeros(1, dtype=torch.int64, device="cuda")
        nsk = torch.zeros(1, dtype=torch.int64, device="cuda")
        assert _call(api, "mg_grid", spec, bank, uvw, vis, ref, nsk_ref, torch) == api.MG_OK
        assert _call(api, "mg_grid_static", spec, bank, uvw, vis, got, nsk, torch) == api.MG_OK
        torch.cuda.synchronize()
        err = H.rel_l2(got.cpu().numpy(), ref.cpu().numpy())
        print(f"[no-alloc] {uvw.shape[0]} records on {n}^2: rel-L2 vs mg_grid {err:.2e}, "
              f"skipped {int(nsk.item())}", flush=True)
        assert err < TOL
        assert int(nsk.item()) == int(nsk_ref.item())
        assert float(got.abs().max()) > 0
    # too large for the static array: refused on the host, nothing queued
    big = torch.zeros(3_000_000, 3, dtype=torch.float32, device="cuda")
    bvis = torch.zeros(3_000_000, 4, dtype=torch.complex64, device="cuda")
    out = torch.zeros(4, 1024, 1024, dtype=torch.complex64, device="cuda")
    spec = api.GridSpec(1024, 1024, 4, wl.beta, 1.0, 1.0)
    nsk = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = _call(api, "mg_grid_static", spec, H.device_bank(wl), big, bvis, out, nsk, torch)
    assert st == api.MG_ENOMEM
    assert b"static scratch" in L.mg_last_error()
    torch.cuda.synchronize()
    assert int(nsk.item()) == 0 and float(out.abs().max()) == 0.0
