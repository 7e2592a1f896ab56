"""Serving trace driver: a Poisson stream of gridding jobs of uneven sizes,
run through the continuous-batching server and, for comparison, one job at
a time.

The trace follows the serving workload: visibility counts log-uniform in
[1e4, 1e7], grids of 512^2 .. 4096^2 (uniform in the exponent), half of the
jobs with a 7x7 separable kernel (oversampling 8) and half with a
W-projection bank of 16 planes, supports 8 -> 32 (oversampling 4).  Record
coordinates are contiguous slices of two record pools (the 64-antenna 1 km
array and the 256-antenna log-radial array), visibilities slices of an
N(0, 1) pool.  Reported: p50/p99 latency (submission to completion seen by
the scheduler), aggregate Gridding Rate over the makespan, and the serial
rate of the same jobs.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List

import numpy as np
import torch

from . import api
from . import workload as W


@dataclasses.dataclass
class Job:
    kind: str            # "sep" | "wproj"
    n: int               # grid side
    start: int           # slice of the record pool
    nrec: int
    updates: int         # sum of S^2 over valid records
    arrival: float = 0.0


class TracePools:
    """Device-resident record pools shared by all jobs of a trace."""

    def __init__(self, device, max_rec: int = 10_000_000, seed: int = W.SEED_TRACE):
        self.device = device
        sep = W.config_autograd()                      # 10.08M records, 7x7, beta 8
        self.sep_uvw = torch.from_numpy(sep.uvw[:max_rec]).to(device)
        self.sep_taps = sep.taps
        self.sep_umax = float(np.abs(sep.uvw[:, :2]).max())
        wp = W.config_wproj_device(device, n_ant=128, n_times=32, n_chan=80, n=1024, nplanes=16,
                                   s_min=8, s_max=32, beta=4)
        self.wp_uvw = wp.uvw[:max_rec].contiguous()
        self.wp = wp
        self.wp_umax = float(wp.uvw[:, :2].abs().max())
        npool = max(self.sep_uvw.shape[0], self.wp_uvw.shape[0])
        self.vis = W.vis_normal_torch(npool, 4, seed, device)
        self._wp_prefix = None
        self._banks = {}

    def bank(self, kind: str):
        """The kernel bank of a job kind, resident on the device (one per
        kind: the tables do not depend on the grid size)."""
        if kind not in self._banks:
            if kind == "sep":
                t = torch.from_numpy(self.sep_taps.astype(np.float32)).to(self.device)
                self._banks[kind] = api.KernelBank("separable", t, support=7)
            else:
                # the bank's field of view follows the pool's 1024 grid; for
                # other grid sizes the same tables are used (the gridding cost
                # does not depend on the table values)
                b = self.wp.bank
                t = torch.from_numpy(b.taps.astype(np.complex64)).to(self.device)
                self._banks[kind] = api.KernelBank("wproj", t, plane_support=b.supports.tolist(),
                                                   plane_offset=b.offsets.tolist(),
                                                   inv_dw=b.inv_dw)
        return self._banks[kind]

    def spec_bank(self, kind: str, n: int, fill: float = 0.5):
        if kind == "sep":
            scale = fill * (n / 2 - 7) / self.sep_umax
            return api.GridSpec(n, n, 4, 8, scale, scale), self.bank(kind)
        scale = fill * (n / 2 - 32) / self.wp_umax
        return api.GridSpec(n, n, 4, 4, scale, scale), self.bank(kind)

    def wproj_updates_prefix(self):
        """Prefix sums of S_p^2 over the W-projection pool (all records fall
        inside every grid of the trace because uv are scaled per grid)."""
        if self._wp_prefix is None:
            spec, bank = self.spec_bank("wproj", 1024)
            ix = api.compute_indices(spec, bank, self.wp_uvw)
            sup = torch.tensor(self.wp.bank.supports, dtype=torch.int64, device=self.device)
            s2 = sup[ix["plane"].clamp(min=0).long()] ** 2 * ix["valid"].long()
            self._wp_prefix = torch.cat([torch.zeros(1, dtype=torch.int64, device=self.device),
                                         torch.cumsum(s2, 0)]).cpu().numpy()
        return self._wp_prefix


def make_trace(pools: TracePools, njobs: int, seed: int = W.SEED_TRACE,
               nrec_range=(1e4, 1e7)) -> List[Job]:
    rng = np.random.Generator(np.random.PCG64(seed))
    pre = pools.wproj_updates_prefix()
    jobs = []
    for _ in range(njobs):
        kind = "sep" if rng.random() < 0.5 else "wproj"
        n = int(2 ** rng.integers(9, 13))
        nrec = int(round(math.exp(rng.uniform(math.log(nrec_range[0]), math.log(nrec_range[1])))))
        pool = pools.sep_uvw if kind == "sep" else pools.wp_uvw
        nrec = min(nrec, pool.shape[0])
        start = int(rng.integers(0, pool.shape[0] - nrec + 1))
        upd = 49 * nrec if kind == "sep" else int(pre[start + nrec] - pre[start])
        jobs.append(Job(kind, n, start, nrec, upd))
    return jobs


def _job_inputs(pools: TracePools, j: Job):
    uvw = (pools.sep_uvw if j.kind == "sep" else pools.wp_uvw)[j.start:j.start + j.nrec]
    vis = pools.vis[j.start:j.start + j.nrec]
    spec, bank = pools.spec_bank(j.kind, j.n)
    return spec, bank, uvw, vis


class GridPool:
    """Output grids of the trace, reused round-robin per grid side (the
    trace measures time; the values of served results are checked by the
    serving tests, not here, so jobs may share an output grid: every commit
    is an atomic add)."""

    def __init__(self, device, per_side: int = 8):
        self.device, self.per_side = device, per_side
        self._grids = {}
        self._next = {}

    def get(self, n: int) -> torch.Tensor:
        lst = self._grids.setdefault(n, [])
        i = self._next.get(n, 0)
        self._next[n] = i + 1
        if len(lst) < self.per_side:
            lst.append(torch.zeros(4, n, n, dtype=torch.complex64, device=self.device))
        return lst[i % self.per_side]


def run_serial(pools: TracePools, jobs: List[Job], grids: "GridPool" = None) -> dict:
    """Each job alone: one-shot gridding, synchronised, one after the other."""
    grids = grids or GridPool(pools.device)
    inputs = [_job_inputs(pools, j) for j in jobs]
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for j, (spec, bank, uvw, vis) in zip(jobs, inputs):
        g = grids.get(j.n)
        a = time.perf_counter()
        api.grid(spec, bank, uvw, vis, out=g)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - a)
    total = time.perf_counter() - t0
    upd = sum(j.updates for j in jobs)
    busy = sum(times)
    return {"jobs": len(jobs), "busy_s": busy, "wall_s": total, "updates": upd,
            "rate_updates_per_s": upd / busy, "mean_service_s": busy / len(jobs)}


def run_served(pools: TracePools, jobs: List[Job], rho: float, mean_service_s: float,
               budget_bytes: int = 64 << 30, slots: int = 64, nstreams: int = 8,
               seed: int = W.SEED_TRACE + 1, grids: "GridPool" = None) -> dict:
    """Poisson arrivals at rate rho / mean_service_s; jobs are submitted at
    their arrival times and run through the server."""
    grids = grids or GridPool(pools.device)
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = rho / mean_service_s
    gaps = rng.exponential(1.0 / lam, len(jobs))
    arrivals = np.cumsum(gaps) - gaps[0]
    inputs = [_job_inputs(pools, j) for j in jobs]
    torch.cuda.synchronize()
    with api.Server(budget_bytes, slots, nstreams) as srv:
        t0 = time.perf_counter()
        ids = []
        for j, (spec, bank, uvw, vis), ta in zip(jobs, inputs, arrivals):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            ids.append(srv.submit(spec, bank, uvw, vis, grids.get(j.n)))
        lat = [srv.wait(i) for i in ids]
        makespan = time.perf_counter() - t0
        stats = srv.stats()
    upd = sum(j.updates for j in jobs)
    lat_ms = np.array(lat) * 1e3
    out = {"jobs": len(jobs), "rho": rho, "makespan_s": makespan,
           "rate_updates_per_s": upd / makespan,
           "latency_ms_p50": float(np.percentile(lat_ms, 50)),
           "latency_ms_p99": float(np.percentile(lat_ms, 99)),
           "latency_ms_mean": float(lat_ms.mean()),
           "max_running": stats["max_running"], "bytes_peak": stats["bytes_peak"],
           "budget": stats["budget"]}
    return out
