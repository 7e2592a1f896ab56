"""Reduced-precision kernel banks at the precision workload's shape: a
1,000,000-record random subsample (seed 2115) of the 1.0e9-record
512-antenna array on a 16384^2 grid, W-projection with 32 planes, S 8 -> 64,
oversampling 4.

Per result (grid windows and degridded sampled records) and per tap format
(FP32, FP16, BF16), three relative-L2 errors are reported:
  total         GPU result vs the FP64 oracle with the FP64 bank
  accumulation  GPU result vs the FP64 oracle with the bank rounded to the
                tap format (what the FP32 arithmetic adds)
  quantisation  FP64 oracle with the rounded bank vs the FP64 bank
The bar: accumulation within 1e-5 in every format; total within twice the
format's unit roundoff (2^-24, 2^-11, 2^-8)."""
import numpy as np
import pytest

import oracle
from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def test_precision_report():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api
    dev = torch.device("cuda:0")
    wl = W.config_precision_sample()
    print(f"[precision] {wl.name}", flush=True)
    n = wl.n
    b = wl.bank
    geom = H.oracle_geom(wl)
    uvw64 = wl.uvw.astype(np.float64)
    vis = W.vis_normal(wl.nrec, 4, W.SEED_VIS)
    vis128 = vis.astype(np.complex128)
    r = np.hypot(uvw64[:, 0], uvw64[:, 1])
    order = np.argsort(r)
    wins = []
    for q in (0.0, 0.5, 0.9, 0.99):
        i = order[int(q * (len(order) - 1))]
        cu = int(uvw64[i, 0] * wl.scale + n // 2)
        cv = int(uvw64[i, 1] * wl.scale + n // 2)
        wins.append((min(max(cu - 32, 0), n - 64), min(max(cv - 32, 0), n - 64), 64, 64))

    def oracle_windows(taps):
        return [oracle.grid(geom, taps, uvw64, vis128, window=w)[0] for w in wins]

    idx = W.subsample(wl.nrec, 20000, W.SEED_SUBSAMPLE + 1)
    gin = W.vis_normal_torch(4 * n * n, 1, W.SEED_NOISE, dev).reshape(4, n, n)
    gin_h = gin.cpu().numpy().astype(np.complex128)   # converted once (17 GB)

    ref64_g = oracle_windows(b.taps)
    ref64_d = oracle.degrid(geom, b.taps, uvw64[idx], gin_h)[0]
    spec = H.grid_spec(wl)
    uvw_d = torch.from_numpy(wl.uvw).to(dev)
    vis_d = torch.from_numpy(vis).to(dev)
    grid = torch.empty(4, n, n, dtype=torch.complex64, device=dev)
    it = torch.from_numpy(idx).to(dev)
    rows = []
    for fmt in ("f32", "f16", "bf16"):
        taps_q = H.quantise_taps(b.taps, fmt)
        refq_g = oracle_windows(taps_q)
        refq_d = oracle.degrid(geom, taps_q, uvw64[idx], gin_h)[0]
        bank = H.device_bank(wl, fmt)
        grid.zero_()
        api.grid(spec, bank, uvw_d, vis_d, out=grid)
        vout = api.degrid(spec, bank, uvw_d, gin)
        torch.cuda.synchronize()
        got_g = np.concatenate([grid[:, v0:v0 + wv, u0:u0 + wu].cpu().numpy().ravel()
                                for (u0, v0, wu, wv) in wins])
        got_d = vout[it].cpu().numpy()
        cat = lambda xs: np.concatenate([x.ravel() for x in xs])
        for res, got, r64, rq in (("grid", got_g, cat(ref64_g), cat(refq_g)),
                                  ("degrid", got_d, ref64_d, refq_d)):
            tot, acc, qua = H.rel_l2(got, r64), H.rel_l2(got, rq), H.rel_l2(rq, r64)
            rows.append((res, fmt, tot, acc, qua))
            print(f"[precision] {res:6s} {fmt:4s} total {tot:.3e}  accumulation {acc:.3e}  "
                  f"quantisation {qua:.3e}  (unit roundoff {UNIT_ROUNDOFF[fmt]:.2e})", flush=True)
    for res, fmt, tot, acc, qua in rows:
        assert acc < 1e-5, (res, fmt, acc)
        assert tot < max(2 * UNIT_ROUNDOFF[fmt], 1e-5), (res, fmt, tot)
