"""Hybrid Gridding and column pruning on the GPU (through the C ABI) against
the FP64 oracle: the Hybrid Gridding Step at the small separable workload's
size and over geometry variants (supports 1..32, oversampling 2..16, 1-4
polarisations, FP16 taps, ties, non-finite and out-of-range records), at the
autograd workload's size on windows, the column pruner over (alpha, S_z)
and wrap-heavy shapes, and hybrid gridding followed by pruning with the
kernel itself against the convolutional gridder.  Bar: skipped counts exact,
values within relative L2 1e-5 of FP64."""
import numpy as np
import pytest

import oracle
from oracle import Geometry
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


def _edges(beta, nu, nv, scale):
    rows = []
    for q in range(-20, 20, 3):
        x = (q + 0.5) / beta + 2.0               # ties of the nearest-row rule
        rows.append([x / scale, x / scale, 0.0])
    rows += [[np.nan, 0, 0], [0, np.inf, 0], [nu / scale, 0, 0], [0, nv / scale, 0],
             [0, -(nv / 2 + 0.2) / scale, 0]]
    return np.array(rows)


def _hybrid_both(torch, api, geom, taps, uvw, vis, dtype="f32", plan=False):
    spec = api.GridSpec(geom.nu, geom.nv, vis.shape[1], geom.beta, geom.scale_u, geom.scale_v)
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    bank = api.KernelBank("separable", torch.from_numpy(taps).to(tdt).cuda(), support=geom.support)
    u = torch.from_numpy(np.ascontiguousarray(uvw)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(vis.astype(np.complex64))).cuda()
    nsk = torch.zeros(1, dtype=torch.int64, device="cuda")
    if plan:
        with api.HybridPlan(spec, bank, u) as hp:
            G = hp.grid(v)
            sk = hp.nskipped
    else:
        G = api.hybrid_grid(spec, bank, u, v, nskipped=nsk)
        torch.cuda.synchronize()
        sk = int(nsk.item())
    torch.cuda.synchronize()
    tq = H.quantise_taps(taps, dtype)
    ref, sk_ref = oracle.hybrid_grid(geom, tq, uvw, vis.astype(np.complex64).astype(np.complex128))
    assert sk == sk_ref
    return G.cpu().numpy(), ref


@pytest.mark.parametrize("plan", [False, True])
def test_hybrid_small_separable_workload(torch_cuda, api, plan):
    wl = W.config_small()
    geom = H.oracle_geom(wl)
    uvw = np.concatenate([wl.uvw, _edges(wl.beta, wl.n, wl.n, wl.scale)])
    vis = W.vis_normal(uvw.shape[0], 4, seed=51)
    G, ref = _hybrid_both(torch_cuda, api, geom, wl.taps, uvw, vis, plan=plan)
    err = H.rel_l2(G, ref)
    print(f"[hybrid] small workload, plan={plan}: rel-L2 {err:.2e}", flush=True)
    assert err < TOL


CASES = [  # nu, nv, beta, S, npol, dtype
    (300, 200, 2, 1, 2, "f32"),
    (257, 129, 4, 3, 3, "f32"),
    (256, 256, 16, 7, 4, "f32"),
    (200, 260, 8, 12, 1, "f32"),
    (400, 333, 4, 32, 4, "f32"),
    (300, 300, 4, 24, 4, "f16"),
    (128, 96, 6, 6, 4, "bf16"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-b{c[2]}-S{c[3]}-p{c[4]}-{c[5]}"
                                             for c in CASES])
def test_hybrid_geometry_variants(torch_cuda, api, case):
    nu, nv, beta, S, npol, dt = case
    rng = np.random.Generator(np.random.PCG64(nu + beta + S))
    nrec = 30000
    uvw = np.stack([rng.uniform(-nu / 2 - 3, nu / 2 + 3, nrec),
                    rng.uniform(-nv / 2 - 3, nv / 2 + 3, nrec), np.zeros(nrec)], 1)
    uvw[:60, 1] = (np.round(uvw[:60, 1] * beta) + 0.5) / beta
    vis = rng.standard_normal((nrec, npol)) + 1j * rng.standard_normal((nrec, npol))
    taps = rng.uniform(-1.0, 1.0, beta * S + 1)
    geom = Geometry(nu=nu, nv=nv, beta=beta, scale_u=1.0, scale_v=1.0, support=S)
    G, ref = _hybrid_both(torch_cuda, api, geom, taps, uvw, vis, dtype=dt)
    assert H.rel_l2(G, ref) < TOL


def test_hybrid_coherent_and_nonfinite(torch_cuda, api):
    """Every visibility 1 (coherent: fixed-point rounding of one sign would
    add up), then one NaN visibility: its tile commits in FP32 and exactly
    the cells of its footprint become NaN."""
    wl = W.config_small()
    geom = H.oracle_geom(wl)
    vis = np.ones((wl.nrec, 4), np.complex128)
    G, ref = _hybrid_both(torch_cuda, api, geom, wl.taps, wl.uvw, vis)
    assert H.rel_l2(G, ref) < TOL
    vis[777, 2] = np.nan
    G, ref = _hybrid_both(torch_cuda, api, geom, wl.taps, wl.uvw, vis)
    assert np.array_equal(np.isnan(G), np.isnan(ref)) and np.isnan(ref).any()
    fin = np.isfinite(ref)
    assert H.rel_l2(G[fin], ref[fin]) < TOL


@pytest.mark.parametrize("alpha,Sz,M,ncols", [(4, 14, 8192, 1024), (2, 6, 96, 300),
                                              (8, 16, 256, 17), (1, 2, 64, 513),
                                              (3, 4, 24, 256), (4, 8, 32, 40)])
def test_column_pruner(torch_cuda, api, alpha, Sz, M, ncols):
    torch = torch_cuda
    rng = np.random.Generator(np.random.PCG64(alpha * 100 + Sz))
    npol = 2 if M > 1000 else 3
    x = (rng.standard_normal((npol, M, ncols)) + 1j * rng.standard_normal((npol, M, ncols))
         ).astype(np.complex64)
    z = rng.standard_normal(alpha * Sz + 1).astype(np.float32)
    got = api.prune_columns(torch.from_numpy(x).cuda(), alpha, torch.from_numpy(z).cuda(), Sz)
    torch.cuda.synchronize()
    ref = oracle.prune_columns(x.astype(np.complex128), alpha, z.astype(np.float64), Sz)
    err = H.rel_l2(got.cpu().numpy(), ref)
    assert err < TOL, err


def test_hybrid_then_prune_equals_convolutional_gridder(torch_cuda, api):
    """Hybrid gridding then pruning with the gridding kernel itself (S_z = 2S,
    alpha = beta/2) on the GPU gives the convolutional grid on its even
    output rows: against the GPU gridder and the oracle."""
    torch = torch_cuda
    wl = W.config_small()
    spec = H.grid_spec(wl)
    bank = H.device_bank(wl)
    uvw = torch.from_numpy(wl.uvw).cuda()
    vis_h = W.vis_normal(wl.nrec, 4, seed=52)
    vis = torch.from_numpy(vis_h).cuda()
    hy = api.hybrid_grid(spec, bank, uvw, vis)
    z = torch.from_numpy(wl.taps.astype(np.float32)).cuda()
    pr = api.prune_columns(hy, wl.beta // 2, z, 2 * wl.support)
    conv = api.grid(spec, bank, uvw, vis)
    torch.cuda.synchronize()
    even = pr[:, ::2, :].cpu().numpy()
    assert H.rel_l2(even, conv.cpu().numpy()) < TOL
    ref, _ = oracle.grid(H.oracle_geom(wl), H.oracle_taps(wl), wl.uvw, vis_h)
    assert H.rel_l2(even, ref) < TOL


def test_hybrid_autograd_workload_windows(torch_cuda, api):
    """The 10,080,000-record autograd workload (2048^2, 7x7, beta 8) through a
    hybrid plan: four 64 x 256 windows of the 2048 x 16384 hybrid grid, each
    computed by the oracle over all records."""
    torch = torch_cuda
    wl = W.config_autograd()
    geom = H.oracle_geom(wl)
    spec = H.grid_spec(wl)
    vis_h = W.vis_normal(wl.nrec, 4, seed=53)
    with api.HybridPlan(spec, H.device_bank(wl), torch.from_numpy(wl.uvw).cuda()) as hp:
        G = hp.grid(torch.from_numpy(vis_h).cuda())
        torch.cuda.synchronize()
        assert hp.nskipped == 0
    n, rows = wl.n, wl.beta * wl.n
    r = np.hypot(wl.uvw[:, 0], wl.uvw[:, 1])
    order = np.argsort(r)
    wins = [(n // 2 - 32, rows // 2 - 128, 64, 256)]
    for q in (0.5, 0.9, 0.999):
        i = order[int(q * (len(order) - 1))]
        cu = int(wl.uvw[i, 0] * wl.scale + n // 2)
        cq = int((wl.uvw[i, 1] * wl.scale + n // 2) * wl.beta)
        wins.append((min(max(cu - 32, 0), n - 64), min(max(cq - 128, 0), rows - 256), 64, 256))
    taps = H.oracle_taps(wl)
    vis128 = vis_h.astype(np.complex128)
    for (u0, v0, wu, wv) in wins:
        ref, _ = oracle.hybrid_grid(geom, taps, wl.uvw, vis128, window=(u0, v0, wu, wv))
        got = G[:, v0:v0 + wv, u0:u0 + wu].cpu().numpy()
        err = H.rel_l2(got, ref)
        print(f"[hybrid] autograd workload window {(u0, v0, wu, wv)}: rel-L2 {err:.2e}", flush=True)
        assert np.linalg.norm(ref) > 0 and err < TOL
