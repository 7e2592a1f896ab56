#!/usr/bin/env python3
"""Gridding Rate benchmark on one MI355X.

Workload (default): W-projection gridding of 133,693,440 four-polarisation
records (256-antenna log-radial array, 32640 baselines x 32 times x 128
channels, 1.2-1.6 GHz), 8192^2 complex64 grid per polarisation, 32 w-planes
with supports 8 -> 64, oversampling 4, FP32 kernel bank.  Inputs are seeded
and synthetic and are resident in HBM before timing starts.

A step is one one-shot gridding call (mg_grid): index rule + bucket sort +
chunk sort + gather + gridding kernels.  The metric is the Gridding Rate in
record x kernel-point updates per second: the sum over valid records of
S_p^2, divided by the step time.

Also printed: the dominant unit (the gridding kernels of a prepared plan,
timed with HIP events on the launch stream) against the FP32 vector roof;
degridding through the same plan; and the FP64 CPU oracle's rate on a
4,000,000-record sample of the same workload; and a serving trace
(Poisson arrivals of uneven jobs) through the continuous-batching server.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3      # MI355X published (packed FP32)
FP32_UNPACKED_TFLOPS = 78.6          # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBS = 8000.0

# HBM bytes of one plan.grid call (gather + gridding kernels) on the default
# workload: rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, summed over the
# call's dispatches and scaled by the reading of a plain device copy of known
# size.  Valid only for the kernel sources with this digest; any change to
# them makes the figure stale and it is then reported as null.
MEASURED_TRAFFIC = {"sources": "6abd30e3f95320dd", "bytes_per_call": 37043780241,
                    "profile": "profiles/grid_wproj8192_134M_hbm_traffic.txt"}
TRAFFIC_SOURCES = ("grid.hip", "plan.hip", "api.hip", "common.h", "internal.h")


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2111_04141_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def serving_leg(dev, njobs):
    """A Poisson trace of uneven gridding jobs through the serving API: the
    jobs one at a time, then at offered load 0.8 (latency) and as one burst
    (aggregate rate)."""
    from paper_2111_04141_amd import serving as SV
    t0 = time.time()
    pools = SV.TracePools(dev)
    jobs = SV.make_trace(pools, njobs)
    log(f"[bench] serving trace: {njobs} jobs, pools built in {time.time() - t0:.1f}s")
    SV.run_serial(pools, jobs[:4])                       # warm the allocator and kernels
    serial = SV.run_serial(pools, jobs)
    light = SV.run_served(pools, jobs, rho=0.8, mean_service_s=serial["mean_service_s"])
    burst = SV.run_served(pools, jobs, rho=1e6, mean_service_s=serial["mean_service_s"])
    log(f"[bench] serving: serial {serial['rate_updates_per_s']:.3e}/s, "
        f"rho 0.8 p50 {light['latency_ms_p50']:.2f} ms p99 {light['latency_ms_p99']:.2f} ms, "
        f"burst {burst['rate_updates_per_s']:.3e}/s (max running {burst['max_running']})")
    return {
        "trace": f"{njobs} jobs, Poisson arrivals, records log-uniform 1e4..1e7, grids "
                 "512^2..4096^2, half 7x7 separable (beta 8), half W-projection 16 planes "
                 "S 8->32 (beta 4), seed %d" % SV.W.SEED_TRACE,
        "updates": serial["updates"],
        "serial_rate_updates_per_s": serial["rate_updates_per_s"],
        "serial_mean_service_ms": 1e3 * serial["mean_service_s"],
        "rho0.8_latency_ms_p50": light["latency_ms_p50"],
        "rho0.8_latency_ms_p99": light["latency_ms_p99"],
        "rho0.8_rate_updates_per_s": light["rate_updates_per_s"],
        "burst_rate_updates_per_s": burst["rate_updates_per_s"],
        "burst_latency_ms_p50": burst["latency_ms_p50"],
        "burst_latency_ms_p99": burst["latency_ms_p99"],
        "burst_max_running": burst["max_running"],
        "burst_bytes_peak": burst["bytes_peak"],
        "budget_bytes": burst["budget"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--channels", type=int, default=128,
                    help="channels of the W-projection workload (128 = full size)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--serving-jobs", type=int, default=40,
                    help="jobs in the serving trace (0 = skip the serving measurement)")
    ap.add_argument("--no-reduced-precision", action="store_true",
                    help="skip timing the FP16 and BF16 banks")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2111_04141_amd import api
    from paper_2111_04141_amd import workload as W

    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    log(f"[bench] device {props.name}, {props.multi_processor_count} CUs, "
        f"{props.total_memory / 2**30:.0f} GiB")
    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 device copies of {nb} bytes")
        del src, dst
    t0 = time.time()
    wl = W.config_wproj_device(dev, n_chan=args.channels,
                               name=("wproj-8192-P32-S8to64-134M" if args.channels == 128
                                     else None))
    nrec = wl.nrec
    log(f"[bench] workload {wl.name}: {nrec} records, built in {time.time() - t0:.1f}s")
    vis = W.vis_normal_torch(nrec, 4, W.SEED_VIS, dev)
    b = wl.bank
    bank = api.KernelBank("wproj", torch.from_numpy(b.taps.astype(np.complex64)).to(dev),
                          plane_support=b.supports.tolist(), plane_offset=b.offsets.tolist(),
                          inv_dw=b.inv_dw)
    spec = api.GridSpec(wl.n, wl.n, 4, wl.beta, wl.scale, wl.scale)
    uvw = wl.uvw

    # algorithmic work: sum of S_p^2 over the valid records
    ix = api.compute_indices(spec, bank, uvw)
    sup = torch.tensor(b.supports, dtype=torch.int64, device=dev)
    valid = ix["valid"].bool()
    S = sup[ix["plane"].clamp(min=0).long()]
    updates = int(((S * S) * valid).sum().item())
    nvalid = int(valid.sum().item())
    del ix, S, valid
    log(f"[bench] valid records {nvalid}, updates per step {updates:.4e}")

    grid = torch.zeros(4, wl.n, wl.n, dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream(dev)

    # ---- the step: one-shot gridding ----
    for i in range(args.warmup):
        api.grid(spec, bank, uvw, vis, out=grid)
    torch.cuda.synchronize()
    log("[bench] warmup done")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for i in range(args.steps):
        api.grid(spec, bank, uvw, vis, out=grid)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = e0.elapsed_time(e1) / args.steps
    log(f"[bench] step {ms_step:.3f} ms (wall {1e3 * wall / args.steps:.3f} ms)")

    # ---- dominant unit: gridding kernels of a prepared plan ----
    eb0 = torch.cuda.Event(enable_timing=True)
    eb1 = torch.cuda.Event(enable_timing=True)
    eb0.record(stream)
    plan = api.Plan(spec, bank, uvw)
    eb1.record(stream)
    torch.cuda.synchronize()
    plan_ms = eb0.elapsed_time(eb1)
    plan.grid(vis, out=grid)
    torch.cuda.synchronize()
    ek0 = torch.cuda.Event(enable_timing=True)
    ek1 = torch.cuda.Event(enable_timing=True)
    ek0.record(stream)
    for i in range(args.steps):
        plan.grid(vis, out=grid)
    ek1.record(stream)
    torch.cuda.synchronize()
    grid_ms = ek0.elapsed_time(ek1) / args.steps
    vis_out = torch.empty_like(vis)
    plan.degrid(grid, out=vis_out)
    torch.cuda.synchronize()
    ed0 = torch.cuda.Event(enable_timing=True)
    ed1 = torch.cuda.Event(enable_timing=True)
    ed0.record(stream)
    for i in range(args.steps):
        plan.degrid(grid, out=vis_out)
    ed1.record(stream)
    torch.cuda.synchronize()
    degrid_ms = ed0.elapsed_time(ed1) / args.steps
    plan.close()
    log(f"[bench] plan build {plan_ms:.3f} ms, plan grid {grid_ms:.3f} ms, "
        f"plan degrid {degrid_ms:.3f} ms")

    # ---- reduced-precision banks on the same records (error vs FP64 is
    # measured by the precision test; here only their speed) ----
    reduced = {}
    if not args.no_reduced_precision:
        pairs = np.stack([b.taps.real, b.taps.imag], -1)
        for name, tdt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            bank_r = api.KernelBank("wproj", torch.from_numpy(pairs).to(tdt).to(dev),
                                    plane_support=b.supports.tolist(),
                                    plane_offset=b.offsets.tolist(), inv_dw=b.inv_dw)
            plan_r = api.Plan(spec, bank_r, uvw)
            plan_r.grid(vis, out=grid)
            plan_r.degrid(grid, out=vis_out)
            torch.cuda.synchronize()
            er = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            er[0].record(stream)
            for i in range(args.steps):
                plan_r.grid(vis, out=grid)
            er[1].record(stream)
            er[2].record(stream)
            for i in range(args.steps):
                plan_r.degrid(grid, out=vis_out)
            er[3].record(stream)
            torch.cuda.synchronize()
            g_ms = er[0].elapsed_time(er[1]) / args.steps
            d_ms = er[2].elapsed_time(er[3]) / args.steps
            plan_r.close()
            reduced[name] = {"plan_grid_ms": g_ms, "plan_grid_updates_per_s": updates / (g_ms * 1e-3),
                             "plan_degrid_ms": d_ms,
                             "plan_degrid_updates_per_s": updates / (d_ms * 1e-3)}
            log(f"[bench] {name} bank: plan grid {g_ms:.3f} ms, plan degrid {d_ms:.3f} ms")

    flops = 32.0 * updates            # 4 polarisations x complex multiply-add
    traffic = None
    if (MEASURED_TRAFFIC is not None and args.channels == 128
            and MEASURED_TRAFFIC["sources"] == sources_digest()):
        traffic = MEASURED_TRAFFIC["bytes_per_call"]
    achieved_tflops = flops / (grid_ms * 1e-3) / 1e12

    result = {
        "metric": "Gridding Rate (vis x kernel-pt updates/s)",
        "value": updates / (ms_step * 1e-3),
        "unit": "record x kernel-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded uvw by Earth-rotation synthesis, N(0,1) visibilities)",
        "config": {"workload": wl.name, "records": nrec, "valid_records": nvalid,
                   "grid": [4, wl.n, wl.n], "kernel": "W-projection, 32 planes, S 8->64, beta 4",
                   "uvw_dtype": "f32", "updates_per_step": updates},
        "gridding_rate_records_per_s": nvalid / (ms_step * 1e-3),
        "single_pol_updates_per_s": 4 * updates / (ms_step * 1e-3),
        "plan_build_ms": plan_ms,
        "plan_grid_ms": grid_ms,
        "plan_grid_updates_per_s": updates / (grid_ms * 1e-3),
        "plan_degrid_ms": degrid_ms,
        "plan_degrid_updates_per_s": updates / (degrid_ms * 1e-3),
        "reduced_precision_banks": reduced,
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": "one plan.grid call: gather + grid_window_kernel (S <= 32) + grid_block_kernel (S > 32)",
            "flops_per_launch": flops,
            "frac_of_unpacked_fp32": achieved_tflops / FP32_UNPACKED_TFLOPS,
        },
        "context_paper_p100": "Conv Gridder FP32 Npol=4 max 3.62 GRecs/s x 36 = 1.30e11 "
                              "updates/s (S=6 real kernel, no w-term; Tesla P100)",
    }

    if args.serving_jobs > 0:
        del plan, vis_out
        result["serving"] = serving_leg(dev, args.serving_jobs)

    if not args.no_cpu_baseline:
        import oracle
        idx = W.subsample(nrec, args.cpu_sample, W.SEED_SUBSAMPLE)
        it = torch.from_numpy(idx).to(dev)
        uvw_s = uvw[it].cpu().numpy().astype(np.float64)
        vis_s = vis[it].cpu().numpy()
        geom = oracle.Geometry(nu=wl.n, nv=wl.n, beta=wl.beta, scale_u=wl.scale,
                               scale_v=wl.scale, kind="wproj", plane_support=b.supports,
                               plane_offset=b.offsets, inv_dw=b.inv_dw)
        taps = b.taps.astype(np.complex64).astype(np.complex128)
        ixs = oracle.index(geom, uvw_s)
        upd_s = int((b.supports[ixs["plane"]].astype(np.int64) ** 2 * ixs["valid"]).sum())
        out = np.zeros((4, wl.n, wl.n), np.complex128)
        c0 = time.perf_counter()
        oracle.grid(geom, taps, uvw_s, vis_s, out=out)
        cpu_s = time.perf_counter() - c0
        result["cpu_baseline"] = {
            "value": upd_s / cpu_s, "unit": "record x kernel-point updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{len(idx)} records drawn with seed {W.SEED_SUBSAMPLE} from the "
                      f"{nrec}-record workload ({upd_s} updates, {cpu_s:.1f} s, FP64, 1 thread)",
        }
        log(f"[bench] cpu oracle {upd_s / cpu_s:.3e} updates/s over {cpu_s:.1f}s")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
