"""Autograd wiring (CPU, FP64, with a dense stand-in for the plan) and the
GPU Functions against finite differences and the oracle's adjoint."""
import numpy as np
import pytest
import torch

import oracle
from paper_2111_04141_amd import autograd as AG
from paper_2111_04141_amd import workload as W
from tests import helpers as H


class DensePlan:
    """Test stand-in: an explicit complex matrix M (records*npol x cells)
    with the Plan's grid/degrid interface (grid = M^T vis, degrid = conj(M) g
    ... written as G and G^H of a random dense G)."""

    def __init__(self, G):
        self.G = G          # [cells, recs] complex128: grid = G @ vis

    def grid(self, vis):
        return (self.G @ vis.reshape(-1)).reshape(self.shape_g)

    def degrid(self, g):
        return (self.G.conj().T @ g.reshape(-1)).reshape(self.shape_v)


def test_autograd_wiring_gradcheck_cpu():
    torch.manual_seed(0)
    G = torch.randn(12, 10, dtype=torch.complex128)
    plan = DensePlan(G)
    plan.shape_g, plan.shape_v = (3, 4), (5, 2)
    g = torch.randn(3, 4, dtype=torch.complex128, requires_grad=True)
    v = torch.randn(5, 2, dtype=torch.complex128, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: AG.Degrid.apply(x, plan), (g,))
    assert torch.autograd.gradcheck(lambda x: AG.Grid.apply(x, plan), (v,))
    obs = torch.randn(5, 2, dtype=torch.complex128)
    assert torch.autograd.gradcheck(lambda x: AG.chi2(x, plan, obs, 0.1), (g,))


def _window_records(ix, w, S):
    """Records whose footprint reaches window w = (u0, v0, wu, wv)."""
    u0, v0, wu, wv = w
    ok = ix["valid"] == 1
    ku, kv = ix["k_lo_u"], ix["k_lo_v"]
    return np.nonzero(ok & (ku + S - 1 >= u0) & (ku < u0 + wu) & (kv + S - 1 >= v0) &
                      (kv < v0 + wv))[0]


@pytest.mark.gpu
def test_chi2_gradient_at_the_autograd_workload_size():
    """The differentiable workload: 10,080,000 records of the 64-antenna
    array on a 2048^2 grid (7x7, beta 8), V_obs = degrid(W_true) + 0.1 noise.
    At the model W = W_true / 2 the gradient of chi^2 = sum |V_obs - G^H W|^2
    / sigma^2 (the backward of Degrid, i.e. the gridder applied to the
    residual) is checked against the oracle's adjoint on four 64^2 windows,
    each computed over every record that reaches it, with the oracle's own
    V_obs (its degrid of W_true plus the same noise); and against central
    finite differences of the GPU loss on 16 sampled cells, real and
    imaginary parts separately (the major-cycle residual, Section 1.6)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api
    dev = "cuda"
    wl, W_true, noise = W.config_autograd_problem(dev)
    assert wl.nrec == 10_080_000 and wl.n == 2048
    sigma = 0.1
    print(f"[autograd] {wl.name}: {wl.nrec} records", flush=True)
    spec, bank = H.grid_spec(wl), H.device_bank(wl)
    uvw = torch.from_numpy(wl.uvw).to(dev)
    with api.Plan(spec, bank, uvw) as plan:
        vis_obs = plan.degrid(W_true) + noise
        Wm = (0.5 * W_true).detach().clone().requires_grad_(True)
        L = AG.chi2(Wm, plan, vis_obs, sigma)
        L.backward()
        grad = Wm.grad
        torch.cuda.synchronize()
        # the oracle's adjoint of the residual on four windows
        geom, taps = H.oracle_geom(wl), H.oracle_taps(wl)
        ix = oracle.index(geom, wl.uvw)
        Wt_h = W_true.cpu().numpy().astype(np.complex128)
        noise_h = noise.cpu().numpy().astype(np.complex128)
        n = wl.n
        r = np.hypot(wl.uvw[:, 0], wl.uvw[:, 1])
        order = np.argsort(r)
        wins = [(n // 2 - 32, n // 2 - 32, 64, 64)]
        for q in (0.3, 0.7, 0.95):
            i = order[int(q * (len(order) - 1))]
            cu = int(wl.uvw[i, 0] * wl.scale + n // 2)
            cv = int(wl.uvw[i, 1] * wl.scale + n // 2)
            wins.append((min(max(cu - 32, 0), n - 64), min(max(cv - 32, 0), n - 64), 64, 64))
        g_h = grad.cpu().numpy()
        for w in wins:
            sel = _window_records(ix, w, wl.support)
            u_s = wl.uvw[sel]
            obs_s = oracle.degrid(geom, taps, u_s, Wt_h)[0] + noise_h[sel]
            model_s = oracle.degrid(geom, taps, u_s, 0.5 * Wt_h)[0]
            res = -2.0 * (obs_s - model_s) / sigma ** 2
            ref, _ = oracle.grid(geom, taps, u_s, res, window=w)
            u0, v0, wu, wv = w
            got = g_h[:, v0:v0 + wv, u0:u0 + wu]
            err = H.rel_l2(got, ref)
            print(f"[autograd] window {w}: {len(sel)} records, gradient rel-L2 {err:.2e}",
                  flush=True)
            assert err < 1e-4, (w, err)
        # central finite differences on 16 cells with a large gradient
        rng = np.random.Generator(np.random.PCG64(12))
        g0 = np.abs(g_h[0])
        touched = np.argwhere(g0 > 0.1 * g0.max())
        cells = touched[rng.choice(len(touched), 16, replace=False)]
        for (y, x) in cells:
            gscale = float(np.abs(g_h[0, y, x])) + 1e-30
            for part, unit in (("re", 1.0), ("im", 1j)):
                eps = 1e-2 * max(1.0, float(np.abs(Wm[0, y, x].item())))
                Wp, Wn = Wm.detach().clone(), Wm.detach().clone()
                Wp[0, y, x] += eps * unit
                Wn[0, y, x] -= eps * unit
                Lp = AG.chi2(Wp, plan, vis_obs, sigma).item()
                Ln = AG.chi2(Wn, plan, vis_obs, sigma).item()
                fd = (Lp - Ln) / (2 * eps)
                an = g_h[0, y, x].real if part == "re" else g_h[0, y, x].imag
                assert abs(fd - an) <= 1e-3 * gscale, (y, x, part, fd, an)
        print(f"[autograd] finite differences agree on {len(cells)} cells", flush=True)
