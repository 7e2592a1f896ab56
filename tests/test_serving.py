"""Serving (continuous batching): every served job's grid against the FP64
oracle at the serving workload's shapes, each result the same alone and in
the mix, the HBM budget enforced, one slot serialising.  (GPU; the host-side
argument checks of the server API are in test_abi.py and its job state
transitions in test_serve_state.py.)"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api as A
    A.lib()
    return A


@pytest.fixture(scope="module")
def pools():
    """Record pools of the serving workload: the 64-antenna 1 km array
    (10,080,000 records, 7x7 prolate spheroidal, beta 8) and a log-radial
    array with a 16-plane W-projection bank, supports 8 -> 32, beta 4."""
    sep = W.config_autograd()
    wp = W.config_wproj(n_ant=64, n_times=32, n_chan=64, n=1024, nplanes=16, s_min=8,
                        s_max=32, beta=4, uvw_dtype=np.float32)
    return sep, wp


def _job_list(pools, njobs=14, seed=W.SEED_TRACE):
    """Jobs spanning the serving shapes: every grid side 512 .. 4096 with
    both kernels, records log-uniform in [1e4, 1e7] (capped by the pool)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = [512, 1024, 2048, 4096]
    out = []
    for i in range(njobs):
        kind = "sep" if i % 2 == 0 else "wproj"
        n = sides[(i // 2) % 4]
        wl = pools[0] if kind == "sep" else pools[1]
        nrec = int(round(math.exp(rng.uniform(math.log(1e4), math.log(1e7)))))
        if i == 0:
            nrec = 10_000_000          # the largest job size
        nrec = min(nrec, wl.nrec)
        s0 = int(rng.integers(0, wl.nrec - nrec + 1))
        out.append((kind, n, s0, nrec))
    return out


def _job_inputs(api, pools, job, vis_seed):
    kind, n, s0, nrec = job
    wl = pools[0] if kind == "sep" else pools[1]
    umax = float(np.abs(wl.uvw[:, :2]).max())
    scale = 0.5 * (n / 2 - wl.support) / umax
    spec = api.GridSpec(n, n, 4, wl.beta, scale, scale)
    uvw = np.ascontiguousarray(wl.uvw[s0:s0 + nrec])
    vis = W.vis_normal(nrec, 4, seed=vis_seed)
    if wl.kind == "separable":
        geom = oracle.Geometry(nu=n, nv=n, beta=wl.beta, scale_u=scale, scale_v=scale,
                               support=wl.support)
    else:
        b = wl.bank
        geom = oracle.Geometry(nu=n, nv=n, beta=wl.beta, scale_u=scale, scale_v=scale,
                               kind="wproj", plane_support=b.supports, plane_offset=b.offsets,
                               inv_dw=b.inv_dw)
    return spec, H.device_bank(wl), uvw, vis, geom, H.oracle_taps(wl)


def _windows(uvw, scale, n, size=64):
    r = np.hypot(uvw[:, 0], uvw[:, 1])
    order = np.argsort(r)
    wins = [(n // 2 - size // 2, n // 2 - size // 2, size, size)]
    for q in (0.5, 0.9, 0.999):
        i = order[int(q * (len(order) - 1))]
        cu = int(uvw[i, 0] * scale + n // 2)
        cv = int(uvw[i, 1] * scale + n // 2)
        wins.append((min(max(cu - size // 2, 0), n - size), min(max(cv - size // 2, 0), n - size),
                     size, size))
    return wins


def test_served_jobs_match_the_oracle_and_their_alone_runs(api, pools):
    jobs = _job_list(pools)
    inputs = [_job_inputs(api, pools, j, 100 + i) for i, j in enumerate(jobs)]
    dev = []
    for spec, bank, uvw, vis, _, _ in inputs:
        dev.append((spec, bank, torch.from_numpy(uvw).cuda(),
                    torch.from_numpy(vis).cuda()))
    alone = []
    for spec, bank, u, v in dev:
        g = api.grid(spec, bank, u, v)
        torch.cuda.synchronize()
        alone.append(g)
    grids = [torch.zeros(4, s.nv, s.nu, dtype=torch.complex64, device="cuda")
             for s, _, _, _ in dev]
    with api.Server(64 << 30, max_slots=8, nstreams=4) as srv:
        ids = [srv.submit(s, b, u, v, g) for (s, b, u, v), g in zip(dev, grids)]
        lat = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["max_running"] >= 2          # jobs overlapped on the device
    assert all(x > 0 for x in lat)
    torch.cuda.synchronize()
    for job, g, a in zip(jobs, grids, alone):
        # alone == in the mix
        assert H.rel_l2(g.cpu().numpy(), a.cpu().numpy()) < TOL, job
    for job, g, (spec, bank, uvw, vis, geom, taps) in zip(jobs, grids, inputs):
        kind, n, s0, nrec = job
        vis128 = vis.astype(np.complex128)
        if n <= 1024:
            ref, _ = oracle.grid_par(geom, taps, uvw, vis128)
            err = H.rel_l2(g.cpu().numpy(), ref)
            print(f"[serving] {kind} {n}^2 {nrec} records: full grid rel-L2 {err:.2e}", flush=True)
            assert err < TOL, job
        else:
            for w in _windows(uvw, spec.scale_u, n):
                u0, v0, wu, wv = w
                ref, _ = oracle.grid_par(geom, taps, uvw, vis128, window=w)
                got = g[:, v0:v0 + wv, u0:u0 + wu].cpu().numpy()
                err = H.rel_l2(got, ref)
                print(f"[serving] {kind} {n}^2 {nrec} records: window {w} rel-L2 {err:.2e}",
                      flush=True)
                if np.linalg.norm(ref) > 0:
                    assert err < TOL, (job, w)
                else:
                    assert np.abs(got).max() == 0.0, (job, w)


def _small_jobs(api, pools, k):
    jobs = [(["sep", "wproj"][i % 2], [512, 1024][i % 2], 1000 * i, 20000 + 5000 * i)
            for i in range(k)]
    out = []
    for i, j in enumerate(jobs):
        spec, bank, uvw, vis, _, _ = _job_inputs(api, pools, j, 200 + i)
        out.append((spec, bank, torch.from_numpy(uvw).cuda(), torch.from_numpy(vis).cuda()))
    return out


def test_admission_respects_budget(api, pools):
    jobs = _small_jobs(api, pools, 6)
    with api.Server(8 << 30, max_slots=64, nstreams=4) as srv:
        budget = srv.stats()["budget"]
        grids = [torch.zeros(4, s.nv, s.nu, dtype=torch.complex64, device="cuda") for s, _, _, _ in jobs]
        ids = [srv.submit(s, b, u, v, g) for (s, b, u, v), g in zip(jobs, grids)]
        for i in ids:
            srv.wait(i)
        st = srv.stats()
        assert st["bytes_peak"] <= budget
        assert st["bytes_in_use"] == 0
        # a waited job is released: its id is no longer known
        with pytest.raises(api.MigridError):
            srv.poll(ids[0])
    # a job larger than the whole budget is refused at submission
    spec, bank, uvw, v = jobs[0]
    g = torch.zeros(4, spec.nv, spec.nu, dtype=torch.complex64, device="cuda")
    with api.Server(1 << 20, max_slots=4, nstreams=1) as srv:
        with pytest.raises(api.MigridError) as e:
            srv.submit(spec, bank, uvw, v, g)
        assert e.value.status == api.MG_ENOMEM


def test_one_slot_serialises(api, pools):
    jobs = _small_jobs(api, pools, 4)
    grids = [torch.zeros(4, s.nv, s.nu, dtype=torch.complex64, device="cuda") for s, _, _, _ in jobs]
    with api.Server(16 << 30, max_slots=1, nstreams=4) as srv:
        ids = [srv.submit(s, b, u, v, g) for (s, b, u, v), g in zip(jobs, grids)]
        for i in ids:
            srv.wait(i)
        assert srv.stats()["max_running"] == 1


def test_inputs_produced_on_the_current_stream_are_waited_for(api, pools):
    """A job's visibilities written by torch on the current stream just
    before submission: the server's stream waits for them through the event
    recorded at submission (no host synchronisation)."""
    spec, bank, uvw, v = _small_jobs(api, pools, 1)[0]
    ref = api.grid(spec, bank, uvw, v)
    torch.cuda.synchronize()
    g = torch.zeros(4, spec.nv, spec.nu, dtype=torch.complex64, device="cuda")
    with api.Server(16 << 30, max_slots=4, nstreams=2) as srv:
        big = torch.randn(4096, 4096, device="cuda")
        vv = torch.zeros_like(v)
        for _ in range(20):                 # queue work ahead of the copy
            big = big @ big * 1e-3
        vv.copy_(v)
        jid = srv.submit(spec, bank, uvw, vv, g)
        srv.wait(jid)
    assert H.rel_l2(g.cpu().numpy(), ref.cpu().numpy()) < TOL
