#!/usr/bin/env python3
"""Gridding Rate benchmark on one MI355X.

Workload (the headline line): W-projection gridding of 133,693,440
four-polarisation records (256-antenna log-radial array, 32640 baselines x
32 times x 128 channels, 1.2-1.6 GHz), 8192^2 complex64 grid per
polarisation, 32 w-planes with supports 8 -> 64, oversampling 4, FP32 kernel
bank.  Inputs are seeded and synthetic and are resident in HBM before timing
starts.

A step is one one-shot gridding call (mg_grid): index rule + bucket sort +
chunk sort + gather + gridding kernels.  The metric is the Gridding Rate in
record x kernel-point updates per second: the sum over valid records of
S_p^2, divided by the step time.

Also printed, as nested objects of the same JSON line:
  * the dominant unit (the gridding kernels of a prepared plan, 3 trials of
    20 calls timed with HIP events on the launch stream: the mean, which the
    roofline uses, the minimum trial mean, as the thesis reports, and the
    median call) against the FP32 vector roof, and degridding likewise;
  * FP16 and BF16 banks on the same records;
  * the small separable workload (100,800 records, 1024^2, 7x7, beta 8),
    the autograd workload (10,080,000 records, 2048^2) and the precision
    workload at full size (1,004,666,880 records, 16384^2, W-projection
    S 8 -> 64 with FP32, FP16 and BF16 banks), each against both roofs;
  * a serving trace (Poisson arrivals of uneven jobs) through the
    continuous-batching server at three offered loads, and as one burst;
  * the FP64 CPU oracle's rate (its band-parallel build on every host core)
    on a sample of the headline workload.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3      # MI355X published (packed FP32)
FP32_UNPACKED_TFLOPS = 78.6          # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6              # vector FP64
PAPER_P100 = ("Conv Gridder FP32 Npol=4 max 3.62 GRecs/s x 36 = 1.30e11 updates/s "
              "(S=6 real kernel, no w-term; Tesla P100)")

# HBM bytes of one plan.grid call (gather + gridding kernels) on the headline
# workload: rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, summed over the
# call's dispatches and scaled by the reading of a plain device copy of known
# size.  Valid only for the kernel sources with this digest; any change to
# them makes the figure stale and it is then reported as null.
MEASURED_TRAFFIC = {"sources": "9521dc875ade642d", "bytes_per_call": 32.57e9,
                    "read_bytes": 16.95e9, "written_bytes": 15.62e9,
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


class Timer:
    """HIP events on one stream: per-call durations and trial means."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def calls(self, fn, n):
        T = self.torch
        ev = [T.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        T.cuda.synchronize()
        ev[0].record(self.stream)
        for i in range(n):
            fn()
            ev[i + 1].record(self.stream)
        T.cuda.synchronize()
        return [ev[i].elapsed_time(ev[i + 1]) for i in range(n)]

    def protocol(self, fn, trials=3, calls=20):
        """The thesis's protocol: `trials` runs of `calls` back-to-back calls
        after one untimed call (which also builds any library plan, e.g. the
        FFT's); the minimum trial mean, plus the mean and median of all calls
        (ms)."""
        import numpy as np
        fn()
        per = [self.calls(fn, calls) for _ in range(trials)]
        flat = np.array([x for t in per for x in t])
        return {"mean_ms": float(flat.mean()), "min_trial_mean_ms": float(min(np.mean(t) for t in per)),
                "median_ms": float(np.median(flat)), "calls": int(flat.size)}


def count_updates(api, torch, spec, bank, uvw, supports, chunk=100_000_000):
    """Sum of S_p^2 over the valid records and the valid count (index rule on
    the device, in slices so the index arrays stay small)."""
    sup = torch.tensor(supports, dtype=torch.int64, device=uvw.device)
    upd, nval = 0, 0
    for s0 in range(0, uvw.shape[0], chunk):
        ix = api.compute_indices(spec, bank, uvw[s0:s0 + chunk])
        valid = ix["valid"].bool()
        S = sup[ix["plane"].clamp(min=0).long()]
        upd += int(((S * S) * valid).sum().item())
        nval += int(valid.sum().item())
        del ix, valid, S
    return upd, nval


def roofs(updates, nrec, touched_cells, npol, flop_per_update, t_ms, meta_bytes=8):
    """Both roofs of one gridding call: algorithmic HBM bytes (visibilities,
    per-record metadata, read-modify-write of the touched grid cells) and
    FP32 flops; fractions are roof time over measured time."""
    hbm_bytes = nrec * (8 * npol + meta_bytes) + 2 * 8 * npol * touched_cells
    flops = flop_per_update * updates
    t_hbm = hbm_bytes / (HBM_PEAK_GBS * 1e9)
    t_valu = flops / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
    t = t_ms * 1e-3
    return {"hbm_bytes": hbm_bytes, "flops": flops, "t_hbm_ms": 1e3 * t_hbm,
            "t_valu_ms": 1e3 * t_valu, "frac_hbm": t_hbm / t, "frac_valu": t_valu / t,
            "frac_binding": max(t_hbm, t_valu) / t,
            "frac_valu_unpacked": flops / (FP32_UNPACKED_TFLOPS * 1e12) / t}


def separable_leg(api, W, torch, dev, stream, wl, name, autograd=False):
    """A separable workload: one-shot and plan timings, both roofs; for the
    autograd workload also one chi^2 forward + backward."""
    import numpy as np
    timer = Timer(torch, stream)
    spec = api.GridSpec(wl.n, wl.n, 4, wl.beta, wl.scale, wl.scale)
    bank = api.KernelBank("separable", torch.from_numpy(wl.taps.astype(np.float32)).to(dev),
                          support=wl.support)
    uvw = torch.from_numpy(wl.uvw).to(dev)
    vis = W.vis_normal_torch(wl.nrec, 4, W.SEED_VIS, dev)
    upd, nval = count_updates(api, torch, spec, bank, uvw, [wl.support])
    grid = torch.zeros(4, wl.n, wl.n, dtype=torch.complex64, device=dev)
    api.grid(spec, bank, uvw, vis, out=grid)
    torch.cuda.synchronize()
    touched = int((grid[0] != 0).sum().item())
    one = timer.protocol(lambda: api.grid(spec, bank, uvw, vis, out=grid))
    b0 = timer.calls(lambda: api.Plan(spec, bank, uvw).close(), 3)
    plan = api.Plan(spec, bank, uvw)
    pg = timer.protocol(lambda: plan.grid(vis, out=grid))
    vout = torch.empty_like(vis)
    pd = timer.protocol(lambda: plan.degrid(grid, out=vout))
    out = {"workload": name, "records": wl.nrec, "valid_records": nval, "grid": [4, wl.n, wl.n],
           "kernel": f"separable {wl.support}x{wl.support}, beta {wl.beta}, FP32 taps",
           "updates": upd, "touched_cells": touched,
           "one_shot_grid": one, "plan_build_ms": float(np.median(b0)),
           "plan_grid": pg, "plan_degrid": pd,
           "plan_grid_updates_per_s": upd / (pg["mean_ms"] * 1e-3),
           "plan_degrid_updates_per_s": upd / (pd["mean_ms"] * 1e-3),
           "one_shot_updates_per_s": upd / (one["mean_ms"] * 1e-3),
           "plan_grid_roofs": roofs(upd, nval, touched, 4, 16, pg["mean_ms"]),
           "plan_degrid_roofs": roofs(upd, nval, touched, 4, 16, pd["mean_ms"]),
           "one_shot_roofs": roofs(upd, nval, touched, 4, 16, one["mean_ms"], meta_bytes=12)}
    if autograd:
        from paper_2111_04141_amd import autograd as AG
        model = (0.5 * grid).detach().clone()
        obs = vis

        def step():
            m = model.detach().requires_grad_(True)
            AG.chi2(m, plan, obs, 0.1).backward()
        st = timer.protocol(step, trials=3, calls=5)
        out["chi2_forward_backward"] = st
    plan.close()
    log(f"[bench] {name}: plan grid {pg['mean_ms']:.3f} ms, degrid {pd['mean_ms']:.3f} ms, "
        f"one-shot {one['mean_ms']:.3f} ms, plan build {out['plan_build_ms']:.3f} ms")
    del grid, vis, uvw, vout
    torch.cuda.empty_cache()
    return out


def hybrid_leg(api, W, torch, dev, stream, wl, name):
    """Hybrid Gridding against convolutional gridding on the same records
    (a separable workload): the Gridder Advantage (the ratio of the two
    gridders' rates, Section 3.5.5, records per second over a prepared plan),
    the column pruner (alpha = beta/2, S_z = 2S, the kernel's own taps as the
    pruning kernel) against the HBM roof, the Column Pruning Gain (inverse
    FFT of the hybrid grid over pruner plus inverse FFT of the pruned grid,
    Section 3.5.6; FFTs by the platform library through torch) and the
    Minimum Record Density D(co, hy) (Section 8.2.1) from these timings."""
    import numpy as np
    timer = Timer(torch, stream)
    spec = api.GridSpec(wl.n, wl.n, 4, wl.beta, wl.scale, wl.scale)
    bank = api.KernelBank("separable", torch.from_numpy(wl.taps.astype(np.float32)).to(dev),
                          support=wl.support)
    uvw = torch.from_numpy(wl.uvw).to(dev)
    vis = W.vis_normal_torch(wl.nrec, 4, W.SEED_VIS, dev)
    n, beta, S = wl.n, wl.beta, wl.support
    alpha = beta // 2
    conv = torch.zeros(4, n, n, dtype=torch.complex64, device=dev)
    hyg = torch.zeros(4, beta * n, n, dtype=torch.complex64, device=dev)
    cp = api.Plan(spec, bank, uvw)
    hp = api.HybridPlan(spec, bank, uvw)
    nval = wl.nrec - hp.nskipped
    tc = timer.protocol(lambda: cp.grid(vis, out=conv))
    th = timer.protocol(lambda: hp.grid(vis, out=hyg))
    z = torch.from_numpy(wl.taps.astype(np.float32)).to(dev)
    pruned = torch.empty(4, 2 * n, n, dtype=torch.complex64, device=dev)
    tp = timer.protocol(lambda: api.prune_columns(hyg, alpha, z, 2 * S, out=pruned))
    # the imaging chain of each grid (origin shifts, batched inverse FFT,
    # correction), through the library's imager
    ones_n = torch.ones(n, dtype=torch.float32, device=dev)
    im_hy = api.Imager(4, n, beta * n)
    im_pr = api.Imager(4, n, 2 * n)
    im_co = api.Imager(4, n, n)
    out_hy = torch.empty(4, beta * n, n, dtype=torch.complex64, device=dev)
    out_n = torch.empty(4, n, n, dtype=torch.complex64, device=dev)
    ones_bn = torch.ones(beta * n, dtype=torch.float32, device=dev)
    f_inp = timer.protocol(lambda: im_hy.image(hyg, ones_n, ones_bn, out=out_hy), trials=3, calls=5)
    f_out1 = timer.protocol(lambda: im_pr.image(pruned, ones_n, ones_n, y0=n // 2, out_ny=n,
                                                out=out_n), trials=3, calls=5)
    f_conv = timer.protocol(lambda: im_co.image(conv, ones_n, ones_n, out=out_n), trials=3, calls=5)
    for im in (im_hy, im_pr, im_co):
        im.close()
    cp.close()
    hp.close()
    rate_co = nval / (tc["mean_ms"] * 1e-3)
    rate_hy = nval / (th["mean_ms"] * 1e-3)
    fin_co = f_conv["mean_ms"] * 1e-3
    fin_hy = (tp["mean_ms"] + f_out1["mean_ms"]) * 1e-3
    denom = 1.0 / rate_co - 1.0 / rate_hy
    r_eq = (fin_hy - fin_co) / denom if denom > 0 else None
    nn = beta * n
    prune_bytes = 4 * 8 * (beta * n * n + 2 * n * n)
    out = {"workload": name, "records": wl.nrec, "valid_records": nval,
           "grid": [4, n, n], "hybrid_grid": [4, beta * n, n], "pruned_grid": [4, 2 * n, n],
           "kernel": f"separable {S}x{S}, beta {beta}; hybrid S x 1; pruning alpha {alpha}, "
                     f"S_z {2 * S}",
           "conv_plan_grid": tc, "hybrid_plan_grid": th,
           "conv_records_per_s": rate_co, "hybrid_records_per_s": rate_hy,
           "gridder_advantage": rate_hy / rate_co,
           "column_pruner": tp,
           "column_pruner_hbm_frac": prune_bytes / (HBM_PEAK_GBS * 1e9) / (tp["mean_ms"] * 1e-3),
           "image_hybrid_grid": f_inp, "image_pruned_grid": f_out1, "image_conv_grid": f_conv,
           "column_pruning_gain": f_inp["mean_ms"] / (tp["mean_ms"] + f_out1["mean_ms"]),
           "column_pruner_footprint": tp["mean_ms"] / (tp["mean_ms"] + f_out1["mean_ms"]),
           "min_record_density_co_hy_pct": (100.0 * r_eq / (nn * nn)) if r_eq is not None else None,
           "min_record_density_note": "D(co, hy) = R / N_nn^2 with fin(co) = imaging chain "
                                      "of the N x N grid, fin(hy) = pruner + imaging chain of "
                                      "the 2N x N grid (its central N rows kept)"}
    log(f"[bench] hybrid {name}: conv grid {tc['mean_ms']:.3f} ms, hybrid grid "
        f"{th['mean_ms']:.3f} ms (advantage {out['gridder_advantage']:.2f}x), pruner "
        f"{tp['mean_ms']:.3f} ms, imaging inp/out1/conv {f_inp['mean_ms']:.3f}/"
        f"{f_out1['mean_ms']:.3f}/{f_conv['mean_ms']:.3f} ms, pruning gain "
        f"{out['column_pruning_gain']:.2f}")
    del conv, hyg, pruned, vis, uvw
    torch.cuda.empty_cache()
    return out


def precision_leg(api, W, torch, dev, stream, steps):
    """The precision workload at full size, FP32, FP16 and BF16 banks."""
    import numpy as np
    t0 = time.time()
    wl = W.config_wproj_device(dev, n_ant=512, n_times=16, n_chan=480, n=16384, nplanes=32,
                               s_min=8, s_max=64, beta=4, r_max_m=5000.0,
                               name="precision-16384-P32-S8to64-1.0G")
    log(f"[bench] {wl.name}: {wl.nrec} records, built in {time.time() - t0:.1f}s")
    b = wl.bank
    spec = api.GridSpec(wl.n, wl.n, 4, wl.beta, wl.scale, wl.scale)
    bank32 = api.KernelBank("wproj", torch.from_numpy(b.taps.astype(np.complex64)).to(dev),
                            plane_support=b.supports.tolist(), plane_offset=b.offsets.tolist(),
                            inv_dw=b.inv_dw)
    upd, nval = count_updates(api, torch, spec, bank32, wl.uvw, b.supports)
    vis = W.vis_normal_torch(wl.nrec, 4, W.SEED_VIS, dev)
    grid = torch.zeros(4, wl.n, wl.n, dtype=torch.complex64, device=dev)
    timer = Timer(torch, stream)
    pairs = np.stack([b.taps.real, b.taps.imag], -1)
    out = {"workload": wl.name, "records": wl.nrec, "valid_records": nval,
           "grid": [4, wl.n, wl.n], "kernel": "W-projection, 32 planes, S 8->64, beta 4",
           "updates": upd, "banks": {}}
    touched = None
    for fmt in ("f32", "f16", "bf16"):
        if fmt == "f32":
            bank = bank32
        else:
            tdt = torch.float16 if fmt == "f16" else torch.bfloat16
            bank = api.KernelBank("wproj", torch.from_numpy(pairs).to(tdt).to(dev),
                                  plane_support=b.supports.tolist(),
                                  plane_offset=b.offsets.tolist(), inv_dw=b.inv_dw)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan = api.Plan(spec, bank, wl.uvw)
        e1.record(stream)
        torch.cuda.synchronize()
        build_ms = e0.elapsed_time(e1)
        grid.zero_()
        plan.grid(vis, out=grid)
        torch.cuda.synchronize()
        if touched is None:
            touched = int((grid[0] != 0).sum().item())
        g = timer.calls(lambda: plan.grid(vis, out=grid), steps)
        vout = torch.empty_like(vis)
        plan.degrid(grid, out=vout)
        d = timer.calls(lambda: plan.degrid(grid, out=vout), steps)
        del vout
        plan.close()
        gm, dm = float(np.mean(g)), float(np.mean(d))
        out["banks"][fmt] = {"plan_build_ms": build_ms, "plan_grid_ms": gm,
                             "plan_grid_min_ms": float(min(g)),
                             "plan_degrid_ms": dm, "plan_degrid_min_ms": float(min(d)),
                             "plan_grid_updates_per_s": upd / (gm * 1e-3),
                             "plan_degrid_updates_per_s": upd / (dm * 1e-3),
                             "plan_grid_roofs": roofs(upd, nval, touched, 4, 32, gm),
                             "plan_degrid_roofs": roofs(upd, nval, touched, 4, 32, dm)}
        log(f"[bench] precision {fmt}: plan build {build_ms:.2f} ms, grid {gm:.2f} ms, "
            f"degrid {dm:.2f} ms")
    out["touched_cells"] = touched
    del grid, vis, wl
    torch.cuda.empty_cache()
    return out


def imaging_leg(api, W, torch, dev, stream, wl, name):
    """The imaging chain on a convolutional grid of the workload: corrector
    vector, origin shifts fused around the platform library's batched C2C
    inverse FFT (one per polarisation) and the separable correction.  The
    fused shift-in and correct-out kernels stream the grid twice (read and
    write, 4 x 8 bytes per cell each); the FFT is the library's."""
    import numpy as np
    timer = Timer(torch, stream)
    n = wl.n
    G = W.vis_normal_torch(4 * n * n, 1, W.SEED_NOISE, dev).reshape(4, n, n)
    t = torch.from_numpy(wl.taps.astype(np.float32)).to(dev)
    h = api.corrector(n, wl.beta, t, wl.beta)
    im = api.Imager(4, n, n)
    out = torch.empty_like(G)
    chain = timer.protocol(lambda: im.image(G, h, h, out=out))
    fft = timer.protocol(lambda: torch.fft.ifft2(G))
    corr = timer.protocol(lambda: api.corrector(n, wl.beta, t, wl.beta))
    im.close()
    grid_bytes = 4 * 8 * n * n
    # the least traffic of the chain: shift-in, one FFT pass and the
    # correction each read and write the grid once
    r = {"workload": name, "grid": [4, n, n], "chain": chain, "library_fft_alone": fft,
         "corrector": corr,
         "chain_hbm_frac": 6 * grid_bytes / (HBM_PEAK_GBS * 1e9) / (chain["mean_ms"] * 1e-3),
         "note": "chain_hbm_frac: 6 x the grid bytes (three read-write passes) over the chain "
                 "time; torch.fft.ifft2 of the same grid timed alone for comparison"}
    log(f"[bench] imaging {name}: chain {chain['mean_ms']:.3f} ms, library FFT alone "
        f"{fft['mean_ms']:.3f} ms, corrector {corr['mean_ms']:.4f} ms")
    return r


def kernel_bank_leg(api, W, torch, dev, wl_wproj):
    """The W-projection bank of the 32-plane schedule (S 8 -> 64,
    oversampling 4, the W-projection and precision workloads' bank), built
    on the device in FP64 (taper, screen, batched Z2Z FFT per plane size,
    normalisation); the FP64 oracle's time for the same bank is part of the
    CPU baseline.  Timed on the host clock around a synchronised call (it
    includes the workspace allocation and about 160 launches), after a first
    call that creates the FFT plans; the FFT flops use 5 M^2 log2(M^2) per
    M x M plane."""
    import numpy as np
    b = wl_wproj.bank
    sup = [int(x) for x in b.supports]
    dw = 1.0 / b.inv_dw
    ws = [p * dw for p in range(len(sup))]
    base = W.pswf_taps(7, 4)
    bt = torch.from_numpy(base).to(dev)
    api.wkernel_bank(sup, ws, 4, bt, wl_wproj.scale)          # FFT plans made
    torch.cuda.synchronize()
    times = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.wkernel_bank(sup, ws, 4, bt, wl_wproj.scale)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
    flops = sum(5.0 * (8 * s) ** 2 * np.log2((8 * s) ** 2) for s in sup)
    r = {"schedule": "32 planes, S 8->64, beta 4, FP64 build, complex64 output",
         "device_ms_min": float(min(times)), "device_ms_median": float(np.median(times)),
         "fft_flops": flops,
         "fft_fp64_frac_at_min": flops / (FP64_PEAK_TFLOPS * 1e12) / (min(times) * 1e-3),
         "note": "launch-bound at this size: the whole bank is 32 planes of at most 512^2 "
                 "points"}
    log(f"[bench] kernel bank: device {min(times):.2f} ms (median {np.median(times):.2f})")
    return r


def wstack_leg(api, W, torch, dev, stream, wl, name, layers=16):
    """W-stacking on the workload's records: gridding onto `layers` layer
    grids (the plain gridder's kernels on the stacked grid) against gridding
    the same records onto one grid, and the W-stacking image (batched FFT of
    every layer and polarisation, screen-and-sum kernel that reads every
    layer once and writes the image)."""
    import numpy as np
    timer = Timer(torch, stream)
    n = wl.n
    wmax = float(np.max(np.abs(wl.uvw[:, 2])))
    dw = 2.0 * wmax / (layers - 1)
    spec = api.GridSpec(n, n, 4, wl.beta, wl.scale, wl.scale)
    t = torch.from_numpy(wl.taps.astype(np.float32)).to(dev)
    plain = api.KernelBank("separable", t, support=wl.support)
    ws = api.KernelBank("wstack", t, support=wl.support, layers=layers, inv_dw=1.0 / dw)
    uvw = torch.from_numpy(wl.uvw).to(dev)
    vis = W.vis_normal_torch(wl.nrec, 4, W.SEED_VIS, dev)
    pp = api.Plan(spec, plain, uvw)
    pw = api.Plan(spec, ws, uvw)
    g1 = torch.zeros(4, n, n, dtype=torch.complex64, device=dev)
    gl = torch.zeros(4, layers, n, n, dtype=torch.complex64, device=dev)
    tp = timer.protocol(lambda: pp.grid(vis, out=g1))
    tw = timer.protocol(lambda: pw.grid(vis, out=gl))
    nval = wl.nrec - pw.nskipped
    pp.close()
    pw.close()
    h = api.corrector(n, wl.beta, t, wl.beta)
    im = api.WStackImager(4, layers, n, n)
    img = torch.empty(4, n, n, dtype=torch.complex64, device=dev)
    ti = timer.protocol(lambda: im.image(gl, h, h, wl.scale, wl.scale, dw, out=img), calls=5)
    fft = timer.protocol(lambda: torch.fft.ifft2(gl), calls=5)
    im.close()
    upd = nval * wl.support ** 2
    layer_bytes = 4 * layers * 8 * n * n
    r = {"workload": name, "layers": layers, "layer_spacing_wavelengths": dw,
         "grid": [4, layers, n, n], "records": wl.nrec, "valid_records": nval,
         "plain_plan_grid": tp, "wstack_plan_grid": tw,
         "wstack_grid_updates_per_s": upd / (tw["mean_ms"] * 1e-3),
         "wstack_over_plain_grid_time": tw["mean_ms"] / tp["mean_ms"],
         "image": ti, "library_fft_alone": fft,
         "image_hbm_frac": (5 * layer_bytes + 4 * 8 * n * n) / (HBM_PEAK_GBS * 1e9)
                           / (ti["mean_ms"] * 1e-3),
         "note": "image_hbm_frac: the least traffic of the chain (shift-in and one FFT pass "
                 "read and write every layer, the screen-and-sum reads every layer and writes "
                 "the image) over the image time"}
    log(f"[bench] wstack {name}: {layers} layers, grid {tw['mean_ms']:.3f} ms (plain "
        f"{tp['mean_ms']:.3f} ms), image {ti['mean_ms']:.3f} ms (FFT alone {fft['mean_ms']:.3f})")
    return r


def serving_leg(dev, njobs):
    """A Poisson trace of uneven gridding jobs through the serving API: the
    jobs one at a time, then at offered loads 0.5, 0.8 and 0.95 (latency),
    and as one burst (aggregate rate)."""
    from paper_2111_04141_amd import serving as SV
    t0 = time.time()
    pools = SV.TracePools(dev)
    jobs = SV.make_trace(pools, njobs)
    grids = SV.GridPool(dev)
    log(f"[bench] serving trace: {njobs} jobs, pools built in {time.time() - t0:.1f}s")
    SV.run_serial(pools, jobs[:8], grids)              # warm the allocator and kernels
    serial = SV.run_serial(pools, jobs, grids)
    out = {
        "trace": f"{njobs} jobs, Poisson arrivals, records log-uniform 1e4..1e7, grids "
                 "512^2..4096^2, half 7x7 separable (beta 8), half W-projection 16 planes "
                 "S 8->32 (beta 4), seed %d" % SV.W.SEED_TRACE,
        "updates": serial["updates"],
        "serial_rate_updates_per_s": serial["rate_updates_per_s"],
        "serial_mean_service_ms": 1e3 * serial["mean_service_s"],
    }
    for rho in (0.5, 0.8, 0.95):
        r = SV.run_served(pools, jobs, rho=rho, mean_service_s=serial["mean_service_s"],
                          grids=grids)
        out[f"rho{rho}"] = {k: r[k] for k in ("latency_ms_p50", "latency_ms_p99",
                                              "latency_ms_mean", "rate_updates_per_s",
                                              "max_running")}
        log(f"[bench] serving rho {rho}: p50 {r['latency_ms_p50']:.2f} ms, "
            f"p99 {r['latency_ms_p99']:.2f} ms")
    burst = SV.run_served(pools, jobs, rho=1e6, mean_service_s=serial["mean_service_s"],
                          grids=grids)
    out["burst"] = {k: burst[k] for k in ("rate_updates_per_s", "latency_ms_p50",
                                          "latency_ms_p99", "max_running", "bytes_peak",
                                          "budget")}
    out["burst_over_serial"] = burst["rate_updates_per_s"] / serial["rate_updates_per_s"]
    log(f"[bench] serving: serial {serial['rate_updates_per_s']:.3e}/s, burst "
        f"{burst['rate_updates_per_s']:.3e}/s ({out['burst_over_serial']:.2f}x)")
    return out


def cpu_baseline_leg(api, W, torch, dev, wl, uvw, vis, b, nrec, per_thread):
    import numpy as np
    import oracle
    threads = oracle.max_threads()
    k = min(nrec, per_thread * threads)
    idx = W.subsample(nrec, k, W.SEED_SUBSAMPLE)
    it = torch.from_numpy(idx).to(dev)
    uvw_s = uvw[it].cpu().numpy().astype(np.float64)
    vis_s = vis[it].cpu().numpy()
    del it
    geom = oracle.Geometry(nu=wl.n, nv=wl.n, beta=wl.beta, scale_u=wl.scale,
                           scale_v=wl.scale, kind="wproj", plane_support=b.supports,
                           plane_offset=b.offsets, inv_dw=b.inv_dw)
    taps = b.taps.astype(np.complex64).astype(np.complex128)
    ixs = oracle.index(geom, uvw_s)
    upd_s = int((b.supports[ixs["plane"]].astype(np.int64) ** 2 * ixs["valid"]).sum())
    out = np.zeros((4, wl.n, wl.n), np.complex128)
    c0 = time.perf_counter()
    oracle.grid_par(geom, taps, uvw_s, vis_s, out=out)
    cpu_s = time.perf_counter() - c0
    log(f"[bench] cpu oracle {upd_s / cpu_s:.3e} updates/s over {cpu_s:.1f}s on {threads} threads")
    # the same workload's W-projection bank built by the FP64 oracle
    from oracle import wkernel as WK
    sup = [int(x) for x in b.supports]
    c0 = time.perf_counter()
    WK.wbank(W.pswf_taps(7, 4), 4, sup, [p / b.inv_dw for p in range(len(sup))], wl.scale)
    bank_ms = 1e3 * (time.perf_counter() - c0)
    return {
        "kernel_bank_oracle_ms": bank_ms,
        "value": upd_s / cpu_s, "unit": "record x kernel-point updates/s", "cores": threads,
        "kind": "oracle",
        "sample": f"{k} records drawn with seed {W.SEED_SUBSAMPLE} from the {nrec}-record "
                  f"workload ({upd_s} updates, {cpu_s:.1f} s, FP64 band-parallel oracle on "
                  f"{threads} threads; nproc {os.cpu_count()}, {cpu_model()})",
        "nproc": os.cpu_count(), "cpu_model": cpu_model(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-per-thread", type=int, default=2_000_000,
                    help="records of the CPU-baseline sample per host thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--channels", type=int, default=128,
                    help="channels of the W-projection workload (128 = full size)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--serving-jobs", type=int, default=1000,
                    help="jobs in the serving trace (0 = skip the serving measurement)")
    ap.add_argument("--no-reduced-precision", action="store_true",
                    help="skip timing the FP16 and BF16 banks on the headline workload")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the small, autograd and precision workload legs")
    ap.add_argument("--only-headline", action="store_true",
                    help="headline step and dominant unit only (profiling runs)")
    ap.add_argument("--only-leg", choices=["small", "autograd", "precision", "serving", "hybrid",
                                           "imaging", "wstack", "bank"],
                    help="run one of the other workloads alone (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)
    if args.only_headline:
        args.no_cpu_baseline = args.no_reduced_precision = args.no_legs = True
        args.serving_jobs = 0

    import numpy as np
    import torch

    from paper_2111_04141_amd import api
    from paper_2111_04141_amd import workload as W

    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    log(f"[bench] device {props.name}, {props.multi_processor_count} CUs, "
        f"{props.total_memory / 2**30:.0f} GiB")
    if args.only_leg:
        stream = torch.cuda.current_stream(dev)
        if args.only_leg == "small":
            r = separable_leg(api, W, torch, dev, stream, W.config_small(), "small-sep7-1024-100800")
        elif args.only_leg == "autograd":
            r = separable_leg(api, W, torch, dev, stream, W.config_autograd(),
                              "autograd-sep7-2048-10M", autograd=True)
        elif args.only_leg == "precision":
            r = precision_leg(api, W, torch, dev, stream, steps=args.steps)
        elif args.only_leg == "imaging":
            r = imaging_leg(api, W, torch, dev, stream, W.config_autograd(),
                            "autograd-sep7-2048-10M")
        elif args.only_leg == "wstack":
            r = wstack_leg(api, W, torch, dev, stream, W.config_autograd(),
                           "autograd-sep7-2048-10M")
        elif args.only_leg == "bank":
            r = kernel_bank_leg(api, W, torch, dev, W.config_wproj_device(
                dev, name="wproj-8192-P32-S8to64-134M"))
        elif args.only_leg == "hybrid":
            r = {"small": hybrid_leg(api, W, torch, dev, stream, W.config_small(),
                                     "small-sep7-1024-100800"),
                 "autograd": hybrid_leg(api, W, torch, dev, stream, W.config_autograd(),
                                        "autograd-sep7-2048-10M")}
        else:
            r = serving_leg(dev, args.serving_jobs)
        print(json.dumps(r), flush=True)
        return
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
    updates, nvalid = count_updates(api, torch, spec, bank, uvw, b.supports)
    log(f"[bench] valid records {nvalid}, updates per step {updates:.4e}")

    grid = torch.zeros(4, wl.n, wl.n, dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream(dev)
    timer = Timer(torch, stream)

    # ---- the step: one-shot gridding (W untimed, then exactly K timed) ----
    for i in range(args.warmup):
        api.grid(spec, bank, uvw, vis, out=grid)
    torch.cuda.synchronize()
    log("[bench] warmup done")
    w0 = time.perf_counter()
    step_ms = timer.calls(lambda: api.grid(spec, bank, uvw, vis, out=grid), args.steps)
    wall = time.perf_counter() - w0
    ms_step = float(np.mean(step_ms))
    log(f"[bench] step {ms_step:.3f} ms (min {min(step_ms):.3f}, median "
        f"{float(np.median(step_ms)):.3f}; wall {1e3 * wall / args.steps:.3f} ms)")

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
    pg = timer.protocol(lambda: plan.grid(vis, out=grid))
    grid_ms = pg["mean_ms"]
    vis_out = torch.empty_like(vis)
    plan.degrid(grid, out=vis_out)
    pd = timer.protocol(lambda: plan.degrid(grid, out=vis_out))
    degrid_ms = pd["mean_ms"]
    plan.close()
    log(f"[bench] plan build {plan_ms:.3f} ms, plan grid {grid_ms:.3f} ms (min trial "
        f"{pg['min_trial_mean_ms']:.3f}), plan degrid {degrid_ms:.3f} ms")

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
            g_ms = float(np.mean(timer.calls(lambda: plan_r.grid(vis, out=grid), 20)))
            d_ms = float(np.mean(timer.calls(lambda: plan_r.degrid(grid, out=vis_out), 20)))
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
    grid.zero_()
    plan2 = api.Plan(spec, bank, uvw)
    plan2.grid(vis, out=grid)
    torch.cuda.synchronize()
    touched = int((grid[0] != 0).sum().item())
    plan2.close()

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
                   "uvw_dtype": "f32", "updates_per_step": updates,
                   "accumulation": "FP32 arithmetic; supports <= 32 commit each unit's sums "
                                   "into a 32-bit fixed-point LDS region (rounded to nearest, "
                                   "per-unit power-of-two scale) flushed to the grid with FP32 "
                                   "atomics; supports > 32 accumulate in FP32 registers"},
        "step_ms_min": float(min(step_ms)),
        "step_ms_median": float(np.median(step_ms)),
        "gridding_rate_records_per_s": nvalid / (ms_step * 1e-3),
        "single_pol_updates_per_s": 4 * updates / (ms_step * 1e-3),
        "plan_build_ms": plan_ms,
        "plan_grid": pg,
        "plan_grid_ms": grid_ms,
        "plan_grid_updates_per_s": updates / (grid_ms * 1e-3),
        "plan_degrid": pd,
        "plan_degrid_ms": degrid_ms,
        "plan_degrid_updates_per_s": updates / (degrid_ms * 1e-3),
        "plan_grid_roofs": roofs(updates, nvalid, touched, 4, 32, grid_ms),
        "reduced_precision_banks": reduced,
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": "one plan.grid call: gather_units_kernel + grid_window_kernel "
                      "(S <= 32) + grid_block_kernel (S > 32)",
            "flops_per_launch": flops,
            "frac_of_unpacked_fp32": achieved_tflops / FP32_UNPACKED_TFLOPS,
        },
        "context_paper_p100": PAPER_P100,
    }
    del vis_out

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_leg(api, W, torch, dev, wl, uvw, vis, b, nrec,
                                                  args.cpu_per_thread)
    bank_wl = wl
    del grid, vis, uvw
    torch.cuda.empty_cache()

    if not args.no_legs:
        result["small_separable"] = separable_leg(api, W, torch, dev, stream, W.config_small(),
                                                  "small-sep7-1024-100800")
        result["autograd"] = separable_leg(api, W, torch, dev, stream, W.config_autograd(),
                                           "autograd-sep7-2048-10M", autograd=True)
        result["precision_full"] = precision_leg(api, W, torch, dev, stream, steps=3)
        result["hybrid"] = {
            "small": hybrid_leg(api, W, torch, dev, stream, W.config_small(),
                                "small-sep7-1024-100800"),
            "autograd": hybrid_leg(api, W, torch, dev, stream, W.config_autograd(),
                                   "autograd-sep7-2048-10M")}
        ag = W.config_autograd()
        result["imaging"] = imaging_leg(api, W, torch, dev, stream, ag, "autograd-sep7-2048-10M")
        result["wstack"] = wstack_leg(api, W, torch, dev, stream, ag, "autograd-sep7-2048-10M")
        result["kernel_bank"] = kernel_bank_leg(api, W, torch, dev, bank_wl)

    if args.serving_jobs > 0:
        result["serving"] = serving_leg(dev, args.serving_jobs)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
