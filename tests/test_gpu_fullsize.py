"""Full-size parity: the 133,693,440-record W-projection workload (256
antennas, 32 planes, S 8 -> 64, oversampling 4) on an 8192^2 grid, through
the same calls the benchmark times (one-shot mg_grid, and a plan's grid and
degrid).  The oracle cannot grid the whole input in seconds, so it checks
sampled outputs: grid windows that it computes over ALL records, and the
degridded values of sampled records of a seeded random grid.  Coherent
inputs (every visibility 1, and one point source) check the fixed-point
commits at this size, on dense and sparse windows, cell by cell."""
import numpy as np
import pytest

import oracle
from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _windows(wl_uvw_host, scale, n, size=32):
    """Window origins: the grid centre and the cells of records at the 50th,
    90th and 99.9th percentile of |uv| (dense, medium, sparse coverage)."""
    r = np.hypot(wl_uvw_host[:, 0], wl_uvw_host[:, 1])
    order = np.argsort(r)
    wins = [(n // 2 - size // 2, n // 2 - size // 2, size, size)]
    for q in (0.5, 0.9, 0.999):
        i = order[int(q * (len(order) - 1))]
        cu = int(wl_uvw_host[i, 0] * scale + n // 2)
        cv = int(wl_uvw_host[i, 1] * scale + n // 2)
        u0 = min(max(cu - size // 2, 0), n - size)
        v0 = min(max(cv - size // 2, 0), n - size)
        wins.append((u0, v0, size, size))
    return wins


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api
    dev = torch.device("cuda:0")
    wl = W.config_wproj_device(dev, name="wproj-8192-P32-S8to64-134M")
    uvw_h = wl.uvw.cpu().numpy()
    return api, dev, wl, uvw_h


def test_full_size_wproj_grid_windows_and_sampled_degrid(full):
    import torch
    api, dev, wl, uvw_h = full
    nrec = wl.nrec
    assert nrec == 133_693_440
    print(f"[fullsize] {wl.name}: {nrec} records", flush=True)
    vis = W.vis_normal_torch(nrec, 4, W.SEED_VIS, dev)
    b = wl.bank
    bank = api.KernelBank("wproj", torch.from_numpy(b.taps.astype(np.complex64)).to(dev),
                          plane_support=b.supports.tolist(), plane_offset=b.offsets.tolist(),
                          inv_dw=b.inv_dw)
    spec = api.GridSpec(wl.n, wl.n, 4, wl.beta, wl.scale, wl.scale)

    skipped = torch.zeros(1, dtype=torch.int64, device=dev)
    g1 = api.grid(spec, bank, wl.uvw, vis, nskipped=skipped)
    plan = api.Plan(spec, bank, wl.uvw)
    g2 = plan.grid(vis)
    torch.cuda.synchronize()
    assert int(skipped.item()) == 0 and plan.nskipped == 0

    wins = _windows(uvw_h, wl.scale, wl.n)
    uvw64 = uvw_h.astype(np.float64)
    vis128 = vis.cpu().numpy().astype(np.complex128)
    geom = oracle.Geometry(nu=wl.n, nv=wl.n, beta=wl.beta, scale_u=wl.scale, scale_v=wl.scale,
                           kind="wproj", plane_support=b.supports, plane_offset=b.offsets,
                           inv_dw=b.inv_dw)
    taps = H.quantise_taps(b.taps, "f32")
    for (u0, v0, wu, wv) in wins:
        ref, sk = oracle.grid(geom, taps, uvw64, vis128, window=(u0, v0, wu, wv))
        assert sk == 0
        assert np.linalg.norm(ref) > 0
        for name, g in (("one-shot", g1), ("plan", g2)):
            got = g[:, v0:v0 + wv, u0:u0 + wu].cpu().numpy()
            err = H.rel_l2(got, ref)
            print(f"[fullsize] window {(u0, v0, wu, wv)} {name}: rel-L2 {err:.2e}", flush=True)
            assert err < TOL
    del vis128, g1, g2

    # degrid: a seeded N(0,1) grid, all records on the GPU, sampled records
    # on the oracle
    gin = W.vis_normal_torch(4 * wl.n * wl.n, 1, W.SEED_NOISE, dev).reshape(4, wl.n, wl.n)
    out = plan.degrid(gin)
    torch.cuda.synchronize()
    idx = W.subsample(nrec, 4096, W.SEED_SUBSAMPLE)
    got = out[torch.from_numpy(idx).to(dev)].cpu().numpy()
    ref, sk = oracle.degrid(geom, taps, uvw64[idx], gin.cpu().numpy())
    assert sk == 0
    err = H.rel_l2(got, ref)
    print(f"[fullsize] degrid, {len(idx)} sampled records: rel-L2 {err:.2e}", flush=True)
    assert err < TOL
    plan.close()


@pytest.mark.parametrize("kind", ["psf", "point"])
def test_full_size_coherent_inputs(full, kind):
    """Every visibility 1 (the thesis's PSF input, Section 8.1.2) and one
    point source, through a plan on the full workload: windows at the grid
    centre (densest) and at the 99.9th-percentile |uv| (sparse) against the
    oracle at relative L2 1e-5, and the dense window cell by cell within the
    fixed-point and FP32 bound.  All four polarisations carry the same values
    times 1, 0.5, -0.25 and 2j (exact), so the oracle grids one."""
    import torch
    api, dev, wl, uvw_h = full
    b = wl.bank
    bank = api.KernelBank("wproj", torch.from_numpy(b.taps.astype(np.complex64)).to(dev),
                          plane_support=b.supports.tolist(), plane_offset=b.offsets.tolist(),
                          inv_dw=b.inv_dw)
    spec = api.GridSpec(wl.n, wl.n, 4, wl.beta, wl.scale, wl.scale)
    pol_scale = np.array([1.0, 0.5, -0.25, 2j])
    if kind == "psf":
        v1 = torch.ones(wl.nrec, dtype=torch.complex64, device=dev)
    else:
        l0, m0 = 0.37 / wl.scale, -0.21 / wl.scale
        ph = -2.0 * np.pi * (wl.uvw[:, 0].double() * l0 + wl.uvw[:, 1].double() * m0)
        v1 = torch.polar(torch.ones_like(ph), ph).to(torch.complex64)
    vis = v1[:, None] * torch.from_numpy(pol_scale.astype(np.complex64)).to(dev)[None, :]
    with api.Plan(spec, bank, wl.uvw) as plan:
        g = plan.grid(vis.contiguous())
        torch.cuda.synchronize()
    del vis
    v1_h = v1.cpu().numpy().astype(np.complex128)[:, None]
    uvw64 = uvw_h.astype(np.float64)
    geom = oracle.Geometry(nu=wl.n, nv=wl.n, beta=wl.beta, scale_u=wl.scale, scale_v=wl.scale,
                           kind="wproj", plane_support=b.supports, plane_offset=b.offsets,
                           inv_dw=b.inv_dw)
    taps = H.quantise_taps(b.taps, "f32")
    wins = _windows(uvw_h, wl.scale, wl.n)
    for wi, (u0, v0, wu, wv) in enumerate([wins[0], wins[3]]):
        ref1, sk = oracle.grid_par(geom, taps, uvw64, v1_h, window=(u0, v0, wu, wv))
        assert sk == 0 and np.linalg.norm(ref1) > 0
        ref = pol_scale[:, None, None] * ref1[0][None]
        got = g[:, v0:v0 + wv, u0:u0 + wu].cpu().numpy()
        err = H.rel_l2(got, ref)
        print(f"[fullsize] {kind} window {(u0, v0, wu, wv)}: rel-L2 {err:.2e}", flush=True)
        assert err < TOL
        if wi == 0:
            # the unit's quantum follows the largest component over the
            # polarisations (|2j| = 2): bound every polarisation as the
            # largest one (conservative for the others)
            bound2, n_c = H.fixed_point_cell_bound(geom, taps, uvw64, 2.0 * v1_h, wl.support,
                                                   window=(u0, v0, wu, wv), par=True)
            for p in range(4):
                H.assert_within_cell_bound(got[p:p + 1], ref[p:p + 1], bound2, (kind, p))
            print(f"[fullsize] {kind} dense window within the per-cell bound "
                  f"(up to {int(n_c.max())} records per cell)", flush=True)
