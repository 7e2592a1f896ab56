"""GPU parity over geometry variants the workload generators do not reach:
non-square grids whose sides are not multiples of the tile, the largest
grid side (65535 cells) along u and along v, odd and large
oversampling factors, odd supports, S = 1, separable kernels of large
support (the block kernels' real-tap path), W-projection banks with odd
plane supports in every support class, FP16 banks, and records on and
beyond the grid edge.  Grid and degrid against the FP64 oracle; the tap
values are random (the map does not depend on them being a smooth kernel)."""
import numpy as np
import pytest

import oracle
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-5

# (name, kind, nu, nv, beta, supports, npol, tap dtype)
CASES = [
    ("sep-S1-b2", "sep", 300, 200, 2, [1], 2, "f32"),
    ("sep-S3-b4", "sep", 257, 129, 4, [3], 3, "f32"),
    ("sep-S6-b63", "sep", 256, 256, 63, [6], 4, "f32"),
    ("sep-S12-b128", "sep", 200, 260, 128, [12], 4, "f32"),
    ("sep-S20-b4", "sep", 400, 333, 4, [20], 4, "f32"),
    ("sep-S40-b2", "sep", 512, 300, 2, [40], 1, "f32"),
    ("sep-S24-b4-f16", "sep", 300, 300, 4, [24], 4, "f16"),
    ("wproj-odd-b2", "wproj", 300, 280, 2, [5, 9, 17, 33], 4, "f32"),
    ("wproj-b4-f16", "wproj", 260, 390, 4, [8, 14, 26, 50], 2, "f16"),
    # several planes per support class: tile-major plane groups and units
    # spanning planes of different supports
    ("wproj-groups", "wproj", 300, 260, 2, [6, 8, 10, 12, 16, 18, 24, 32, 34, 48], 4, "f32"),
    # supports out of order: every plane its own group, classes interleaved
    ("wproj-unordered", "wproj", 280, 300, 2, [40, 10, 20, 8, 12, 36], 3, "f32"),
    # every support of the 17..32 class in one group (each slot count 3..8 of
    # its two-wave teams, odd supports included), and the separable kernel
    # at the class's largest slot count
    ("wproj-class2-all", "wproj", 300, 300, 4, list(range(17, 33)), 4, "f32"),
    ("sep-S31-b2", "sep", 300, 290, 2, [31], 4, "f32"),
    # the largest grid side (cells up to 65534 in the packed 16-bit halves of
    # the gridders' cell words), along u and along v
    ("sep-S7-max-u", "sep", 65535, 40, 2, [7], 2, "f32"),
    ("wproj-max-v", "wproj", 48, 65535, 2, [5, 9, 17, 33], 2, "f32"),
]


def _case(kind, nu, nv, beta, supports, npol, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    nrec = 30000
    smax = max(supports)
    u = rng.uniform(-nu / 2 - 4, nu / 2 + 4, nrec)      # some beyond the edge
    v = rng.uniform(-nv / 2 - 4, nv / 2 + 4, nrec)
    w = rng.uniform(-len(supports) + 0.6, len(supports) - 0.6, nrec)
    # a few records exactly on cell and tie positions
    u[:50] = np.round(u[:50])
    v[50:100] = np.round(v[50:100] * beta) / beta + 0.5 / beta
    uvw = np.stack([u, v, w], 1)
    vis = (rng.standard_normal((nrec, npol)) + 1j * rng.standard_normal((nrec, npol)))
    if kind == "sep":
        S = supports[0]
        taps = rng.uniform(-1.0, 1.0, beta * S + 1)
        geom = oracle.Geometry(nu=nu, nv=nv, beta=beta, scale_u=1.0, scale_v=1.0, support=S)
        return uvw, vis, taps, geom, None
    sizes = [(beta * s + 1) ** 2 for s in supports]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    taps = rng.standard_normal(sum(sizes)) + 1j * rng.standard_normal(sum(sizes))
    taps /= np.abs(taps).max()
    geom = oracle.Geometry(nu=nu, nv=nv, beta=beta, scale_u=1.0, scale_v=1.0, kind="wproj",
                           plane_support=np.array(supports, np.int32), plane_offset=offs,
                           inv_dw=1.0)
    return uvw, vis, taps, geom, offs


@pytest.mark.parametrize("name,kind,nu,nv,beta,supports,npol,dtype", CASES,
                         ids=[c[0] for c in CASES])
def test_geometry_variant(name, kind, nu, nv, beta, supports, npol, dtype):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api
    uvw, vis, taps, geom, offs = _case(kind, nu, nv, beta, supports, npol, seed=len(name))
    taps_q = H.quantise_taps(taps, dtype)
    G_ref, sk = oracle.grid(geom, taps_q, uvw, vis)
    assert 0 < sk < len(uvw)
    spec = api.GridSpec(nu, nv, npol, beta, 1.0, 1.0)
    tdt = {"f32": torch.float32, "f16": torch.float16}[dtype]
    if kind == "sep":
        bank = api.KernelBank("separable", torch.from_numpy(taps).to(tdt).cuda(),
                              support=supports[0])
    else:
        if dtype == "f32":
            t = torch.from_numpy(taps.astype(np.complex64)).cuda()
        else:
            t = torch.from_numpy(np.stack([taps.real, taps.imag], -1)).to(tdt).cuda()
        bank = api.KernelBank("wproj", t, plane_support=list(supports),
                              plane_offset=offs.tolist(), inv_dw=1.0)
    uvw_d = torch.from_numpy(uvw).cuda()
    vis_d = torch.from_numpy(vis.astype(np.complex64)).cuda()
    nsk = torch.zeros(1, dtype=torch.int64, device="cuda")
    G = api.grid(spec, bank, uvw_d, vis_d, nskipped=nsk)
    torch.cuda.synchronize()
    assert int(nsk.item()) == sk
    assert H.rel_l2(G.cpu().numpy(), G_ref) < TOL

    rng = np.random.Generator(np.random.PCG64(5))
    Gin = (rng.standard_normal((npol, nv, nu)) + 1j * rng.standard_normal((npol, nv, nu))
           ).astype(np.complex64)
    V_ref, sk2 = oracle.degrid(geom, taps_q, uvw, Gin)
    V = api.degrid(spec, bank, uvw_d, torch.from_numpy(Gin).cuda())
    torch.cuda.synchronize()
    assert sk2 == sk
    assert H.rel_l2(V.cpu().numpy(), V_ref) < TOL
