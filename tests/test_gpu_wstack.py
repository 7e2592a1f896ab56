"""W-stacking on the GPU (MG_KERNEL_WSTACK through mg_compute_indices,
mg_grid, plans and mg_wstack_imager_*) against the oracle (oracle/wstack.py):

  * indices bit for bit: the FP64 layer rule, the per-layer index rule and
    the stacked row offset, with the records straddling layer boundaries,
    clamped beyond the outer layers and running off their layer's grid;
  * one-shot and plan gridding of the small separable workload (100,800
    records, 1024^2 per layer, 7x7, oversampling 8) over 8 layers against
    the oracle's per-layer grids (relative L2 1e-5), and plan degridding
    against the oracle's per-layer degridding;
  * the W-stacking image (per-layer inverse FFT, screens, sum, correction)
    against the FP64 oracle chain over the central half of the field;
  * a point source with w terms, gridded, stacked and imaged on the device,
    against the direct Fourier sum with the W-term;
  * W-stacking jobs served by mg_server_* beside a separable job."""
import numpy as np
import pytest

import oracle
from oracle import imaging as IM
from oracle import wstack as WS
from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def api(torch_cuda):
    from paper_2111_04141_amd import api as A
    A.lib()
    return A


def _small_wstack(layers=8):
    wl = W.config_small()
    uvw = wl.uvw.astype(np.float64)
    wmax = float(np.max(np.abs(uvw[:, 2])))
    dw = 2.0 * wmax / (layers - 1)
    return wl, uvw, dw


def _bank(api, torch, wl, layers, dw):
    return api.KernelBank("wstack", torch.from_numpy(wl.taps.astype(np.float32)).cuda(),
                          support=wl.support, layers=layers, inv_dw=1.0 / dw)


def test_indices_bit_exact(torch_cuda, api):
    torch = torch_cuda
    layers, dw, n, beta, S, scale = 5, 0.5, 256, 8, 7, 1.0
    rng = np.random.Generator(np.random.PCG64(17))
    nrec = 20000
    uv = rng.uniform(-n / 2, n / 2, (nrec, 2))
    w = rng.uniform(-2.0, 2.0, nrec)
    w[:200] = (np.arange(200) % (layers + 1) + 1 - layers / 2) * dw     # on boundaries
    uvw = np.concatenate([uv, w[:, None]], 1)
    spec = api.GridSpec(n, n, 1, beta, scale, scale)
    bank = api.KernelBank("wstack", torch.from_numpy(W.pswf_taps(S, beta).astype(np.float32)).cuda(),
                          support=S, layers=layers, inv_dw=1 / dw)
    got = api.compute_indices(spec, bank, torch.from_numpy(uvw).cuda())
    geom = oracle.Geometry(nu=n, nv=n, beta=beta, scale_u=scale, scale_v=scale, support=S)
    ref = oracle.index(geom, uvw)
    j = WS.layer_of(w, layers, 1 / dw)
    valid = ref["valid"].astype(bool)
    assert np.array_equal(got["valid"].cpu().numpy().astype(bool), valid)
    for k in ("k_lo_u", "o_u", "o_v"):
        assert np.array_equal(got[k].cpu().numpy()[valid], ref[k][valid]), k
    assert np.array_equal(got["k_lo_v"].cpu().numpy()[valid], (ref["k_lo_v"] + j * n)[valid])
    assert int(got["nskipped"].item()) == ref["nskipped"] > 0


def test_stacked_rows_at_the_16_bit_limit(torch_cuda, api):
    """8 layers of 8191 rows: stacked rows up to 65527, the top of the
    gridders' 16-bit cell halves; a random separable 7-tap kernel."""
    torch = torch_cuda
    layers, dw, nu, nv, beta, S = 8, 1.0, 64, 8191, 2, 7
    rng = np.random.Generator(np.random.PCG64(23))
    nrec = 20000
    u = rng.uniform(-nu / 2 - 3, nu / 2 + 3, nrec)
    v = rng.uniform(-nv / 2 - 3, nv / 2 + 3, nrec)
    w = rng.uniform(-layers / 2 - 1, layers / 2 + 1, nrec) * dw
    v[:2000] = rng.uniform(nv / 2 - 6, nv / 2, 2000)           # the top rows
    w[:2000] = rng.uniform(layers / 2 - 1, layers / 2, 2000) * dw   # of the top layer
    uvw = np.stack([u, v, w], 1)
    vis = (rng.standard_normal((nrec, 2)) + 1j * rng.standard_normal((nrec, 2)))
    taps = rng.uniform(-1.0, 1.0, beta * S + 1)
    spec = api.GridSpec(nu, nv, 2, beta, 1.0, 1.0)
    bank = api.KernelBank("wstack", torch.from_numpy(taps.astype(np.float32)).cuda(),
                          support=S, layers=layers, inv_dw=1 / dw)
    G = api.grid(spec, bank, torch.from_numpy(uvw).cuda(),
                 torch.from_numpy(vis.astype(np.complex64)).cuda())
    torch.cuda.synchronize()
    geom = oracle.Geometry(nu=nu, nv=nv, beta=beta, scale_u=1.0, scale_v=1.0, support=S)
    taps_q = taps.astype(np.float32).astype(np.float64)
    ref, sk = WS.grid_layers(geom, taps_q, uvw, vis, layers, 1 / dw)
    assert 0 < sk < nrec
    top = ref[:, layers - 1, nv - 8:, :]
    assert np.abs(top).max() > 0     # the top layer's top rows are reached
    err = H.rel_l2(G.cpu().numpy(), ref)
    print(f"[wstack] {layers} x {nv} stacked rows: rel-L2 {err:.2e}", flush=True)
    assert err < TOL


def test_grid_and_degrid_small_workload(torch_cuda, api):
    torch = torch_cuda
    layers = 8
    wl, uvw, dw = _small_wstack(layers)
    vis = W.vis_normal(wl.nrec, 4, seed=81)
    spec = H.grid_spec(wl)
    bank = _bank(api, torch, wl, layers, dw)
    uvw_d = torch.from_numpy(wl.uvw).cuda()
    vis_d = torch.from_numpy(vis).cuda()
    g1 = api.grid(spec, bank, uvw_d, vis_d)
    with api.Plan(spec, bank, uvw_d) as plan:
        g2 = plan.grid(vis_d)
        gin = W.vis_normal_torch(4 * layers * wl.n * wl.n, 1, 82, "cuda").reshape(
            4, layers, wl.n, wl.n)
        out = plan.degrid(gin)
        torch.cuda.synchronize()
    assert tuple(g1.shape) == (4, layers, wl.n, wl.n)
    taps = H.oracle_taps(wl)
    geom = H.oracle_geom(wl)
    ref, sk = WS.grid_layers(geom, taps, uvw, vis, layers, 1 / dw)
    for name, g in (("one-shot", g1), ("plan", g2)):
        err = H.rel_l2(g.cpu().numpy(), ref)
        print(f"[wstack] {name} grid, {layers} layers: rel-L2 {err:.2e}", flush=True)
        assert err < TOL
    j = WS.layer_of(uvw[:, 2], layers, 1 / dw)
    gh = gin.cpu().numpy()
    want = np.zeros((wl.nrec, 4), np.complex128)
    for lay in range(layers):
        sel = j == lay
        want[sel] = oracle.degrid(geom, taps, uvw[sel], gh[:, lay])[0]
    err = H.rel_l2(out.cpu().numpy(), want)
    print(f"[wstack] plan degrid: rel-L2 {err:.2e}", flush=True)
    assert err < TOL


def test_served_wstack_jobs_match_the_oracle(torch_cuda, api):
    """W-stacking jobs through the server, alongside a plain separable job on
    the same records: each served grid against the oracle."""
    torch = torch_cuda
    layers = 4
    wl, uvw, dw = _small_wstack(layers)
    vis = W.vis_normal(wl.nrec, 4, seed=84)
    spec = H.grid_spec(wl)
    uvw_d = torch.from_numpy(wl.uvw).cuda()
    vis_d = torch.from_numpy(vis).cuda()
    wbank = _bank(api, torch, wl, layers, dw)
    sbank = api.KernelBank("separable", torch.from_numpy(wl.taps.astype(np.float32)).cuda(),
                           support=wl.support)
    g_w = [torch.zeros(4, layers, wl.n, wl.n, dtype=torch.complex64, device="cuda")
           for _ in range(2)]
    g_s = torch.zeros(4, wl.n, wl.n, dtype=torch.complex64, device="cuda")
    with api.Server(16 << 30, max_slots=4, nstreams=3) as srv:
        ids = [srv.submit(spec, wbank, uvw_d, vis_d, g_w[0]),
               srv.submit(spec, sbank, uvw_d, vis_d, g_s),
               srv.submit(spec, wbank, uvw_d, vis_d, g_w[1])]
        for i in ids:
            srv.wait(i)
    torch.cuda.synchronize()
    taps = H.oracle_taps(wl)
    geom = H.oracle_geom(wl)
    ref_w, _ = WS.grid_layers(geom, taps, uvw, vis, layers, 1 / dw)
    ref_s, _ = oracle.grid(geom, taps, uvw, vis)
    for g in g_w:
        err = H.rel_l2(g.cpu().numpy(), ref_w)
        print(f"[wstack] served, {layers} layers: rel-L2 {err:.2e}", flush=True)
        assert err < TOL
    assert H.rel_l2(g_s.cpu().numpy(), ref_s) < TOL
    # more stacked rows than the 16-bit cell halves hold: refused at submit
    spec2 = api.GridSpec(16, 1024, 1, wl.beta, 1.0, 1.0)
    bank2 = _bank(api, torch, wl, 65, dw)
    u2 = torch.zeros(10, 3, dtype=torch.float64, device="cuda")
    v2 = torch.zeros(10, 1, dtype=torch.complex64, device="cuda")
    g2 = torch.zeros(1, 65, 1024, 16, dtype=torch.complex64, device="cuda")
    with api.Server(1 << 30, max_slots=1, nstreams=1) as srv:
        with pytest.raises(Exception, match="65535"):
            srv.submit(spec2, bank2, u2, v2, g2)


def test_image_small_workload(torch_cuda, api):
    torch = torch_cuda
    layers = 8
    wl, uvw, dw = _small_wstack(layers)
    vis = W.vis_normal(wl.nrec, 4, seed=83)
    bank = _bank(api, torch, wl, layers, dw)
    G = api.grid(H.grid_spec(wl), bank, torch.from_numpy(wl.uvw).cuda(),
                 torch.from_numpy(vis).cuda())
    t = torch.from_numpy(wl.taps.astype(np.float32)).cuda()
    h = api.corrector(wl.n, wl.beta, t, wl.beta)
    img = api.WStackImager(4, layers, wl.n, wl.n).image(G, h, h, wl.scale, wl.scale, dw)
    torch.cuda.synchronize()
    taps = H.oracle_taps(wl)
    ref_g, _ = WS.grid_layers(H.oracle_geom(wl), taps, uvw, vis, layers, 1 / dw)
    hr = IM.corrector(wl.n, wl.beta, taps, wl.beta)
    ref = WS.image(ref_g, hr, hr, wl.scale, wl.scale, dw)
    c = slice(wl.n // 4, 3 * wl.n // 4)
    got = img.cpu().numpy()
    err = H.rel_l2(got[:, c, c], ref[:, c, c])
    print(f"[wstack] image, {layers} layers: central half rel-L2 {err:.2e}", flush=True)
    assert err < TOL


def test_point_source_on_device(torch_cuda, api):
    torch = torch_cuda
    n, beta, S, fov, L, dw = 128, 8, 7, 0.2, 7, 60.0
    taps = W.pswf_taps(S, beta)
    rng = np.random.Generator(np.random.PCG64(9))
    nrec = 400
    xc = rng.integers(-40 * beta, 40 * beta, (nrec, 2)) / beta
    w = WS.layer_w(L, dw)[rng.integers(0, L, nrec)]
    u, v = xc[:, 0] / fov, xc[:, 1] / fov
    uvw = np.stack([u, v, w], 1)
    l0, m0 = -0.04, 0.025
    V = np.exp(-2j * np.pi * (u * l0 + v * m0 + w * (np.sqrt(1 - l0 ** 2 - m0 ** 2) - 1)))
    spec = api.GridSpec(n, n, 1, beta, fov, fov)
    t = torch.from_numpy(taps.astype(np.float32)).cuda()
    bank = api.KernelBank("wstack", t, support=S, layers=L, inv_dw=1 / dw)
    G = api.grid(spec, bank, torch.from_numpy(uvw).cuda(),
                 torch.from_numpy(V[:, None].astype(np.complex64)).cuda())
    h = api.corrector(n, beta, t, beta, False)
    img = api.WStackImager(1, L, n, n).image(G, h, h, fov, fov, dw)[0].cpu().numpy()
    lg = (np.arange(n) - n // 2) / n * fov
    Lg, Mg = np.meshgrid(lg, lg)
    truth = np.tensordot(V, np.exp(2j * np.pi * (
        np.multiply.outer(u, Lg) + np.multiply.outer(v, Mg)
        + np.multiply.outer(w, np.sqrt(1 - Lg ** 2 - Mg ** 2) - 1))), 1)
    c = slice(n // 4, 3 * n // 4)
    err = np.linalg.norm((img - truth)[c, c]) / np.linalg.norm(truth[c, c])
    print(f"[wstack] point source: rel-L2 {err:.2e}", flush=True)
    assert err < 1e-3
