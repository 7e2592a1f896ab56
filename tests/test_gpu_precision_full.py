"""The precision workload at full size: 1,004,666,880 records (512 antennas
log-radial 20 m .. 5 km, 130816 baselines x 16 times x 480 channels) on a
16384^2 grid, W-projection with 32 planes, S 8 -> 64, oversampling 4, through
plans as the benchmark times them.

  * degrid a seeded N(0,1) grid with the FP32, FP16 and BF16 banks and check
    1,000,000 sampled records (seed 2115) against the FP64 oracle run with
    the same bank widened from its storage format (the error of the FP32
    arithmetic alone, bar 1e-5);
  * grid N(0,1) visibilities of every record and degrid the result: the
    adjoint identity <G x, G x> = <x, G^H G x>, a property that holds at any
    size, in FP64 sums of the FP32 results (bar 1e-5 relative)."""
import numpy as np
import pytest

import oracle
from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def c5():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api
    dev = torch.device("cuda:0")
    wl = W.config_wproj_device(dev, n_ant=512, n_times=16, n_chan=480, n=16384, nplanes=32,
                               s_min=8, s_max=64, beta=4, r_max_m=5000.0,
                               name="precision-16384-P32-S8to64-1.0G")
    print(f"[precision-full] {wl.name}: {wl.nrec} records", flush=True)
    yield api, dev, wl
    del wl
    torch.cuda.empty_cache()


def test_full_size_degrid_sampled_records(c5):
    import torch
    api, dev, wl = c5
    assert wl.nrec == 1_004_666_880
    n = wl.n
    spec = H.grid_spec(wl)
    gin = W.vis_normal_torch(4 * n * n, 1, W.SEED_NOISE, dev).reshape(4, n, n)
    gin_h = gin.cpu().numpy().astype(np.complex128)      # 17 GB, converted once
    idx = W.subsample(wl.nrec, 1_000_000, W.SEED_SUBSAMPLE)
    it = torch.from_numpy(idx).to(dev)
    uvw_s = wl.uvw[it].double().cpu().numpy()
    geom = H.oracle_geom(wl)
    for fmt in ("f32", "f16", "bf16"):
        with api.Plan(spec, H.device_bank(wl, fmt), wl.uvw) as plan:
            out = plan.degrid(gin)
            torch.cuda.synchronize()
            assert plan.nskipped == 0
            got = out[it].cpu().numpy()
            del out
        ref, sk = oracle.degrid(geom, H.quantise_taps(wl.bank.taps, fmt), uvw_s, gin_h)
        assert sk == 0
        err = H.rel_l2(got, ref)
        print(f"[precision-full] degrid {fmt} bank, {len(idx)} sampled records: rel-L2 "
              f"{err:.2e}", flush=True)
        assert err < TOL


def test_full_size_adjoint_identity(c5):
    import torch
    api, dev, wl = c5
    spec = H.grid_spec(wl)
    x = W.vis_normal_torch(wl.nrec, 4, W.SEED_VIS, dev)
    with api.Plan(spec, H.device_bank(wl, "f32"), wl.uvw) as plan:
        gx = plan.grid(x)
        ghgx = plan.degrid(gx)
        torch.cuda.synchronize()
    lhs = float((gx.abs().double() ** 2).sum())
    rhs = 0j
    step = 1 << 24
    for k in range(0, wl.nrec, step):
        a = x[k:k + step].to(torch.complex128)
        b = ghgx[k:k + step].to(torch.complex128)
        rhs += complex((b.conj() * a).sum())
    err = abs(lhs - rhs) / lhs
    print(f"[precision-full] <Gx,Gx> {lhs:.6e}, <x,GhGx> {rhs.real:.6e}{rhs.imag:+.2e}j: "
          f"relative difference {err:.2e}", flush=True)
    assert err < TOL
