"""Kernel generation on the GPU (mg_wkernel_bank through the C ABI) against
the oracle (oracle/wkernel.py), and the column-pruning aliasing experiment
(Section 7.6) through the device pruner and imager:

  * the W-projection bank of the 32-plane schedule (S 8 -> 64, oversampling
    4) and of an oversampling-8 schedule, FP32 / FP16 / BF16 outputs, entry
    by entry against the FP64 oracle bank (FP16/BF16: the oracle rounded the
    same way, one unit in the last place);
  * a point source observed with w terms, gridded on the device with the
    device-built bank and imaged on the device, against the direct Fourier
    sum with the W-term;
  * the pruning experiment: device pruner + imager against the FP64 oracle
    chain (RMS difference below 1e-5 of the input image's RMS, which the
    folded rows of amplitude a dominate), and the measured aliasing of the
    prolate spheroidal and the least-misfit pruning kernels in FP32."""
import numpy as np
import pytest

import oracle
from oracle import imaging as IM
from oracle import wkernel as WK
from paper_2111_04141_amd import kernels as K
from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("beta,nplanes,s_min,s_max,dw,fov", [(4, 32, 8, 64, 40.0, 0.05),
                                                              (8, 6, 8, 18, 25.0, 0.1)])
def test_bank_matches_oracle(torch_cuda, api, beta, nplanes, s_min, s_max, dw, fov):
    torch = torch_cuda
    sup = W.wproj_support_schedule(nplanes, s_min, s_max)
    ws = [p * dw for p in range(nplanes)]
    base = W.pswf_taps(7, beta)
    ref, offs = WK.wbank(base, beta, sup, ws, fov)
    bt = torch.from_numpy(base).cuda()
    for fmt in ("f32", "f16", "bf16"):
        bank, goffs = api.wkernel_bank(sup.tolist(), ws, beta, bt, fov, fmt)
        torch.cuda.synchronize()
        assert goffs == offs.tolist()
        if fmt == "f32":
            got = bank.cpu().numpy().astype(np.complex128)
            err = np.max(np.abs(got - ref))
            print(f"[kernels] beta {beta}, {nplanes} planes, f32: max |error| {err:.2e}",
                  flush=True)
            assert err < 2e-7                          # FP32 rounding of taps <= 1
        else:
            g = bank.float().cpu().numpy().astype(np.float64)
            got = g[:, 0] + 1j * g[:, 1]
            want = H.quantise_taps(ref, fmt)
            ulp = 2.0 ** (-10 if fmt == "f16" else -7)
            d = np.abs(got - want)
            assert np.all(d <= ulp * np.maximum(np.abs(want), 2.0 ** -14) + 1e-12), fmt


def test_point_source_with_device_bank(torch_cuda, api):
    torch = torch_cuda
    n, beta, fov = 128, 4, 0.2
    base = W.pswf_taps(7, beta)
    ws, sup = [0.0, 100.0, 200.0, 300.0], [8, 12, 16, 24]
    bank, offs = api.wkernel_bank(sup, ws, beta, torch.from_numpy(base).cuda(), fov)
    mx = max(np.max(np.abs(WK.wplane(base, beta, s, x, fov))) for s, x in zip(sup, ws))
    rng = np.random.Generator(np.random.PCG64(5))
    nrec = 300
    xc = rng.integers(-28 * beta, 28 * beta, (nrec, 2)) / beta
    p = rng.integers(0, 4, nrec)
    w = rng.choice([-1.0, 1.0], nrec) * np.array(ws)[p]
    u, v = xc[:, 0] / fov, xc[:, 1] / fov
    uvw = np.stack([u, v, w], 1)
    l0, m0 = 0.03, -0.02
    V = np.exp(-2j * np.pi * (u * l0 + v * m0 + w * (np.sqrt(1 - l0 ** 2 - m0 ** 2) - 1)))
    spec = api.GridSpec(n, n, 1, beta, fov, fov)
    kb = api.KernelBank("wproj", bank, plane_support=sup, plane_offset=offs, inv_dw=1 / 100.0)
    G = api.grid(spec, kb, torch.from_numpy(uvw).cuda(),
                 torch.from_numpy(V[:, None].astype(np.complex64)).cuda())
    h = api.corrector(n, beta, torch.from_numpy(base.astype(np.float32)).cuda(), beta, False)
    img = api.Imager(1, n, n).image(G, h, h)[0].cpu().numpy().astype(np.complex128) * mx
    lg = (np.arange(n) - n // 2) / n * fov
    L, M = np.meshgrid(lg, lg)
    truth = np.tensordot(V, np.exp(2j * np.pi * (
        np.multiply.outer(u, L) + np.multiply.outer(v, M)
        + np.multiply.outer(w, np.sqrt(1 - L ** 2 - M ** 2) - 1))), 1)
    c = slice(n // 4, 3 * n // 4)
    err = np.linalg.norm((img - truth)[c, c]) / np.linalg.norm(truth[c, c])
    print(f"[kernels] point source through the device bank: rel-L2 {err:.2e}", flush=True)
    assert err < 1e-3


def test_pruning_aliasing_experiment_on_device(torch_cuda, api):
    torch = torch_cuda
    alpha, nx, ny = 4, 256, 256
    kernels = {"pswf6": W.pswf_taps(6, alpha)}
    for S in (8, 10, 12, 14):
        kernels[f"lm{S}"] = K.least_misfit(S, 0.25, alpha, sampled=True).table
    rows = []
    ones = torch.ones(nx, dtype=torch.float32, device="cuda")
    for a in (0.5, 10.0, 100.0):
        img = WK.pruning_image(nx, ny, alpha, a)
        Y = img.shape[0]
        orig = img[Y // 2 - ny // 4: Y // 2 + ny // 4]
        G = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(img))) / img.size
        Gd = torch.from_numpy(G[None].astype(np.complex64)).cuda()
        # reference method: inverse transform of the whole grid, cut out
        ref = api.Imager(1, nx, Y).image(Gd, ones, torch.ones(ny // 2, device="cuda"),
                                         y0=Y // 2 - ny // 4, out_ny=ny // 2)
        ref_err = np.abs(ref[0].cpu().numpy() - orig).max()
        y = np.arange(ny // 2) - ny // 4
        for name, T in kernels.items():
            Sz = (T.size - 1) // alpha
            Td = torch.from_numpy(T.astype(np.float32)).cuda()
            P = api.prune_columns(Gd, alpha, Td, Sz)
            hy = api.corrector(ny, alpha, Td, alpha, False)[ny // 4: 3 * ny // 4].contiguous()
            out = api.Imager(1, nx, ny).image(P, ones, hy, y0=ny // 4, out_ny=ny // 2)
            got = out[0].cpu().numpy()
            # parity: the FP64 oracle chain with the same (FP32-rounded) table
            T32 = T.astype(np.float32).astype(np.float64)
            Pr = oracle.prune_columns(G[None], alpha, T32, Sz)[0]
            want = (IM.inverse_transform(Pr[None])[0]
                    * IM.corrector(ny, alpha, T32, alpha, nn_sinc=False)[:, None])
            want = want[ny // 4: 3 * ny // 4]
            # FP32 rounding scales with the whole input (the folded rows
            # carry amplitude a), not with the kept field
            par = np.sqrt(np.mean(np.abs(got - want) ** 2)) / np.sqrt(np.mean(img ** 2))
            assert par < 1e-5, (name, a, par)
            d = np.abs(got - orig)
            rows.append((a, name, d[y < 0].max(), d[y >= 0].max(), ref_err))
    print("[kernels] pruning experiment (FP32): a, kernel, max |error| aliasing region, "
          "zero region, reference method", flush=True)
    for r in rows:
        print(f"[kernels]   {r[0]:6.1f} {r[1]:6s} {r[2]:.2e} {r[3]:.2e} {r[4]:.2e}", flush=True)
    for a in (10.0, 100.0):
        ps = [r[2] for r in rows if r[0] == a and r[1] == "pswf6"][0]
        for r in rows:
            if r[0] == a and r[1] != "pswf6":
                assert r[2] < ps / 10, r
