"""Imaging chain on the GPU (origin shift, batched inverse FFT, correction;
mg_corrector and mg_imager_* through the C ABI) against the oracle's FP64
chain (oracle/imaging.py): correctors, the convolutional image of the small
separable workload, the hybrid image (hybrid gridding, column pruning, the
doubled field cut to its central half) and, with every record at one common
sub-cell offset, exact agreement with the direct Fourier sum."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import Geometry
from oracle import imaging as IM
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


def _central(a):
    n = a.shape[-1]
    m = a.shape[-2]
    return a[..., m // 4: 3 * m // 4, n // 4: 3 * n // 4]


def test_correctors(torch_cuda, api):
    torch = torch_cuda
    taps = W.pswf_taps(7, 8)
    t = torch.from_numpy(taps.astype(np.float32)).cuda()
    for n, phases, sinc in ((1024, 8, True), (1024, 4, True), (64, 8, False), (2048, 4, False)):
        got = api.corrector(n, 8, t, phases, sinc).cpu().numpy()
        ref = IM.corrector(n, 8, taps.astype(np.float32).astype(np.float64), phases, sinc)
        assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-6, (n, phases, sinc)


def test_convolutional_image_small_workload(torch_cuda, api):
    torch = torch_cuda
    wl = W.config_small()
    vis = W.vis_normal(wl.nrec, 4, seed=61)
    G = api.grid(H.grid_spec(wl), H.device_bank(wl), torch.from_numpy(wl.uvw).cuda(),
                 torch.from_numpy(vis).cuda())
    t = torch.from_numpy(wl.taps.astype(np.float32)).cuda()
    h = api.corrector(wl.n, wl.beta, t, wl.beta)
    im = api.Imager(4, wl.n, wl.n)
    img = im.image(G, h, h)
    torch.cuda.synchronize()
    taps = H.oracle_taps(wl)
    G_ref, _ = oracle.grid(H.oracle_geom(wl), taps, wl.uvw, vis)
    hr = IM.corrector(wl.n, wl.beta, taps, wl.beta)
    ref = IM.image_conv(G_ref, hr, hr)
    got = img.cpu().numpy()
    err_c = H.rel_l2(_central(got), _central(ref))
    err = H.rel_l2(got, ref)
    # the corrector grows without bound towards the edge of the field, where
    # it amplifies FP32 rounding: the central half is the usable image
    print(f"[imaging] convolutional image: central half rel-L2 {err_c:.2e}, whole {err:.2e}",
          flush=True)
    assert err_c < TOL


def test_hybrid_image_small_workload(torch_cuda, api):
    torch = torch_cuda
    wl = W.config_small()
    vis = W.vis_normal(wl.nrec, 4, seed=62)
    spec = H.grid_spec(wl)
    hy = api.hybrid_grid(spec, H.device_bank(wl), torch.from_numpy(wl.uvw).cuda(),
                         torch.from_numpy(vis).cuda())
    alpha, Sz = wl.beta // 2, 2 * wl.support
    t = torch.from_numpy(wl.taps.astype(np.float32)).cuda()
    pr = api.prune_columns(hy, alpha, t, Sz)
    hx = api.corrector(wl.n, wl.beta, t, wl.beta)
    hv = api.corrector(wl.n, wl.beta, t, alpha)
    im = api.Imager(4, wl.n, 2 * wl.n)
    img = im.image(pr, hx, hv, y0=wl.n // 2, out_ny=wl.n)
    torch.cuda.synchronize()
    taps = H.oracle_taps(wl)
    geom = H.oracle_geom(wl)
    hy_ref, _ = oracle.hybrid_grid(geom, taps, wl.uvw, vis)
    P_ref = oracle.prune_columns(hy_ref, alpha, taps, Sz)
    ref = IM.image_hybrid(P_ref, IM.corrector(wl.n, wl.beta, taps, wl.beta),
                          IM.corrector(wl.n, wl.beta, taps, alpha))
    got = img.cpu().numpy()
    err_c = H.rel_l2(_central(got), _central(ref))
    print(f"[imaging] hybrid image: central half rel-L2 {err_c:.2e}, whole "
          f"{H.rel_l2(got, ref):.2e}", flush=True)
    assert err_c < TOL


def test_equal_offsets_give_the_direct_sum(torch_cuda, api):
    torch = torch_cuda
    n, beta, S = 64, 4, 7
    rng = np.random.Generator(np.random.PCG64(63))
    nrec = 300
    du, dv = 1 / beta - 0.5, 2 / beta - 0.5
    pos = np.stack([rng.integers(8, n - 8, nrec) + du, rng.integers(8, n - 8, nrec) + dv],
                   1) - n // 2
    F = rng.standard_normal((nrec, 1)) + 1j * rng.standard_normal((nrec, 1))
    taps = W.pswf_taps(S, beta)
    uvw = np.concatenate([pos, np.zeros((nrec, 1))], 1)
    spec = api.GridSpec(n, n, 1, beta, 1.0, 1.0)
    bank = api.KernelBank("separable", torch.from_numpy(taps.astype(np.float32)).cuda(),
                          support=S)
    G = api.grid(spec, bank, torch.from_numpy(uvw).cuda(),
                 torch.from_numpy(F.astype(np.complex64)).cuda())
    l = (np.arange(n) - n // 2) / n
    t32 = taps.astype(np.float32).astype(np.float64)

    def lco(d):
        offs = [Fraction(m) - Fraction(d).limit_denominator(64) for m in range(-S - 1, S + 2)]
        offs = [o for o in offs if -Fraction(S, 2) < o <= Fraction(S, 2)]
        return sum(t32[int(beta * S // 2 + beta * o)] * np.exp(2j * np.pi * float(o) * l)
                   for o in offs)

    # the distortion l_co of a common offset is complex: the GPU chain runs
    # with unit correctors and the division by l_co is applied here
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    img = api.Imager(1, n, n).image(G, ones, ones)
    torch.cuda.synchronize()
    got = img[0].cpu().numpy() / lco(dv)[:, None] / lco(du)[None, :]
    want = oracle.dft(pos, F[:, 0], n, n)
    # exact in arithmetic; the division by l_co amplifies FP32 rounding
    # towards the edge of the field, so the central half carries the bar
    c = slice(n // 4, 3 * n // 4)
    err_c, err = H.rel_l2(got[c, c], want[c, c]), H.rel_l2(got, want)
    print(f"[imaging] equal offsets: central half rel-L2 {err_c:.2e}, whole {err:.2e}",
          flush=True)
    assert err_c < TOL and err < 1e-3
