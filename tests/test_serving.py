"""Serving (continuous batching): results alone == results in the mix, the
HBM budget is enforced, latencies are reported.  (GPU; the host-side
argument checks of the server API are in test_abi.py.)"""
import numpy as np
import pytest
import torch

from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api as A
    A.lib()
    return A


def _jobs(api):
    """Mixed jobs: separable and W-projection, different grid sizes and
    record counts (slices of two small record pools)."""
    sep = W.config_small()
    wp = W.config_wproj(n_ant=40, n_times=8, n_chan=16, n=1024, nplanes=16, s_min=8, s_max=32)
    vis = W.vis_normal(max(sep.nrec, wp.nrec), 4, seed=21)
    rng = np.random.Generator(np.random.PCG64(22))
    out = []
    for i in range(14):
        wl = sep if i % 2 == 0 else wp
        n = [256, 512, 1024][i % 3]
        nrec = int(rng.integers(1000, wl.nrec))
        s0 = int(rng.integers(0, wl.nrec - nrec + 1))
        smax = wl.support
        umax = float(np.abs(wl.uvw[:, :2]).max())
        scale = 0.5 * (n / 2 - smax) / umax
        spec = api.GridSpec(n, n, 4, wl.beta, scale, scale)
        bank = H.device_bank(wl)
        uvw = torch.from_numpy(np.ascontiguousarray(wl.uvw[s0:s0 + nrec])).cuda()
        v = torch.from_numpy(np.ascontiguousarray(vis[s0:s0 + nrec])).cuda()
        out.append((spec, bank, uvw, v))
    return out


def test_results_alone_equal_results_in_the_mix(api):
    jobs = _jobs(api)
    alone = []
    for spec, bank, uvw, v in jobs:
        g = api.grid(spec, bank, uvw, v)
        torch.cuda.synchronize()
        alone.append(g.cpu().numpy())
    grids = [torch.zeros(4, s.nv, s.nu, dtype=torch.complex64, device="cuda") for s, _, _, _ in jobs]
    with api.Server(16 << 30, max_slots=6, nstreams=4) as srv:
        ids = [srv.submit(s, b, u, v, g) for (s, b, u, v), g in zip(jobs, grids)]
        lat = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["max_running"] >= 2          # jobs overlapped on the device
    assert all(x > 0 for x in lat)
    for g, ref in zip(grids, alone):
        assert H.rel_l2(g.cpu().numpy(), ref) < 1e-5


def test_admission_respects_budget(api):
    jobs = _jobs(api)[:6]
    with api.Server(8 << 30, max_slots=64, nstreams=4) as srv:
        budget = srv.stats()["budget"]
        grids = [torch.zeros(4, s.nv, s.nu, dtype=torch.complex64, device="cuda") for s, _, _, _ in jobs]
        ids = [srv.submit(s, b, u, v, g) for (s, b, u, v), g in zip(jobs, grids)]
        for i in ids:
            srv.wait(i)
        st = srv.stats()
        assert st["bytes_peak"] <= budget
        assert st["bytes_in_use"] == 0
    # a job larger than the whole budget is refused at submission
    spec, bank, uvw, v = jobs[0]
    g = torch.zeros(4, spec.nv, spec.nu, dtype=torch.complex64, device="cuda")
    with api.Server(1 << 20, max_slots=4, nstreams=1) as srv:
        with pytest.raises(api.MigridError) as e:
            srv.submit(spec, bank, uvw, v, g)
        assert e.value.status == api.MG_ENOMEM


def test_one_slot_serialises(api):
    jobs = _jobs(api)[:4]
    grids = [torch.zeros(4, s.nv, s.nu, dtype=torch.complex64, device="cuda") for s, _, _, _ in jobs]
    with api.Server(16 << 30, max_slots=1, nstreams=4) as srv:
        ids = [srv.submit(s, b, u, v, g) for (s, b, u, v), g in zip(jobs, grids)]
        for i in ids:
            srv.wait(i)
        assert srv.stats()["max_running"] == 1
