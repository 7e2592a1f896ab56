"""GPU parity over seeded random geometries, beyond the hand-picked variants:
for each case a random grid (sides 64..700, not multiples of the tile), an
oversampling factor in 2..9, 1..4 polarisations, and either a separable
kernel of random support (1..48) or a W-projection bank of 2..6 planes with
random supports (1..64, in any order, so plane groups of every support class
mix; even where the oversampling factor is odd, since beta S must be even); records uniform over the grid and slightly beyond it, with runs of
records sharing a cell (as consecutive channels do) and a few on tie
positions.  Grid and degrid against the FP64 oracle at 1e-5 relative L2."""
import numpy as np
import pytest

import oracle
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-5
NCASES = 12


def _case(seed):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    nu, nv = (int(x) for x in rng.integers(64, 701, 2))
    beta = int(rng.integers(2, 10))
    npol = int(rng.integers(1, 5))
    kind = "sep" if seed % 3 == 0 else "wproj"
    if kind == "sep":
        supports = [int(rng.integers(1, 49))]
    else:
        supports = [int(x) for x in rng.integers(1, 65, int(rng.integers(2, 7)))]
    if beta % 2:   # beta * S must be even (the index rule's reading)
        supports = [s + s % 2 for s in supports]
    nrec = 20000
    u = rng.uniform(-nu / 2 - 3, nu / 2 + 3, nrec)
    v = rng.uniform(-nv / 2 - 3, nv / 2 + 3, nrec)
    # runs of records on one cell (different oversampling phases)
    u[1000:4000] = np.repeat(u[1000:1300], 10) + rng.uniform(0, 0.5, 3000)
    v[1000:4000] = np.repeat(v[1000:1300], 10)
    u[:40] = np.round(u[:40] * beta) / beta + 0.5 / beta      # ties
    w = rng.uniform(-len(supports) + 0.6, len(supports) - 0.6, nrec)
    uvw = np.stack([u, v, w], 1)
    vis = rng.standard_normal((nrec, npol)) + 1j * rng.standard_normal((nrec, npol))
    if kind == "sep":
        S = supports[0]
        taps = rng.uniform(-1.0, 1.0, beta * S + 1)
        geom = oracle.Geometry(nu=nu, nv=nv, beta=beta, scale_u=1.0, scale_v=1.0, support=S)
        return kind, nu, nv, beta, npol, supports, uvw, vis, taps, geom, None
    sizes = [(beta * s + 1) ** 2 for s in supports]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    taps = rng.standard_normal(sum(sizes)) + 1j * rng.standard_normal(sum(sizes))
    taps /= np.abs(taps).max()
    geom = oracle.Geometry(nu=nu, nv=nv, beta=beta, scale_u=1.0, scale_v=1.0, kind="wproj",
                           plane_support=np.array(supports, np.int32), plane_offset=offs,
                           inv_dw=1.0)
    return kind, nu, nv, beta, npol, supports, uvw, vis, taps, geom, offs


@pytest.mark.parametrize("seed", range(NCASES))
def test_random_geometry(seed):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api
    kind, nu, nv, beta, npol, supports, uvw, vis, taps, geom, offs = _case(seed)
    print(f"[random {seed}] {kind} {nu}x{nv} beta {beta} npol {npol} supports {supports}",
          flush=True)
    taps_q = H.quantise_taps(taps, "f32")
    G_ref, sk = oracle.grid(geom, taps_q, uvw, vis)
    spec = api.GridSpec(nu, nv, npol, beta, 1.0, 1.0)
    if kind == "sep":
        bank = api.KernelBank("separable", torch.from_numpy(taps.astype(np.float32)).cuda(),
                              support=supports[0])
    else:
        bank = api.KernelBank("wproj", torch.from_numpy(taps.astype(np.complex64)).cuda(),
                              plane_support=list(supports), plane_offset=offs.tolist(),
                              inv_dw=1.0)
    uvw_d = torch.from_numpy(uvw).cuda()
    vis_d = torch.from_numpy(vis.astype(np.complex64)).cuda()
    nsk = torch.zeros(1, dtype=torch.int64, device="cuda")
    G = api.grid(spec, bank, uvw_d, vis_d, nskipped=nsk)
    torch.cuda.synchronize()
    assert int(nsk.item()) == sk
    err = H.rel_l2(G.cpu().numpy(), G_ref)
    rng = np.random.Generator(np.random.PCG64(7 + seed))
    Gin = (rng.standard_normal((npol, nv, nu)) + 1j * rng.standard_normal((npol, nv, nu))
           ).astype(np.complex64)
    V_ref, _ = oracle.degrid(geom, taps_q, uvw, Gin)
    V = api.degrid(spec, bank, uvw_d, torch.from_numpy(Gin).cuda())
    torch.cuda.synchronize()
    err_d = H.rel_l2(V.cpu().numpy(), V_ref)
    print(f"[random {seed}] grid rel-L2 {err:.2e}, degrid rel-L2 {err_d:.2e}", flush=True)
    assert err < TOL
    assert err_d < TOL
