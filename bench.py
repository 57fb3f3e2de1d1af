"""Throughput of complex-valued FSE on one MI355X, plain and warm-started.

A step conceals every lost block of a batch of eight synthetic 1920x1080
frames (804 isolated 16x16 losses per frame, 10% of the 16x16 grid, border
16 so each area is 48x48, 64x64 transform, rho 0.8, gamma 0.5): 6432 blocks,
inputs resident in HBM. Two legs are timed, each over the same number of
steps:
  plain  FSE with 100 iterations per block (persistent kernel);
  warm   the learned warm start: network inputs, forward pass, top-K
         candidate bins, transform kernel, restricted iterations (K, their
         count and step as chosen on validation frames);
and, with the same K, count and step, two warm starts whose candidates are
not learned (the initial spectrum's top K; the K lowest frequencies), which
show what the network adds.
PSNR over the lost pixels (against the undistorted frames) decides: the
reported value is the warm start's blocks/s if it loses at most 0.1 dB
against plain FSE, otherwise plain FSE's.

Prints one JSON line: blocks/s (value), both legs, the roofline of the
dominant kernel of the reported leg, and the FP64 CPU oracle timed on the
host's cores over a bounded sample of the same blocks. Each leg's steps are
timed twice: first with a HIP event pair around every kernel launch (the
kernel durations of the roofline; reported as instrumented_ms_per_step),
then plainly (value, ms_per_step), since the events cost dispatch time.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FSE blocks/s (16² loss, 64² FFT) plain vs warm-start at ≤0.1 dB PSNR loss"
PSNR_BAR_DB = 0.1
PEAK_FP32_TFLOPS = 157.3        # MI355X FP32 vector, published (counts packed FMA)
NONPACKED_FP32_TFLOPS = 78.6    # 256 CU x 64 lanes x 2 FLOP x 2.4 GHz, without packed FP32
NOMINAL_LDS_TBPS = 78.6         # 256 CU x 128 B/clk x 2.4 GHz (gfx950 measures about twice that)
PEAK_HBM_TBPS = 8.0
FLOP_PER_BIN_ITER = 11          # complex multiply-subtract (8) + |R|^2 (3), eq. (18) + eq. (12)
FLOP_PER_PIXEL_COEF = 4         # Re{c e^{j theta}}: two FMAs, the model on B
LDS_BYTES_PER_BIN_ITER = 24     # read R_w, read shifted W, write R_w (spectra resident on chip)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2204_14193_amd", "csrc", "fse_kernels.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, n_blocks, workload):
    """HBM bytes per launch of `kernel` from committed rocprofv3
    FETCH_SIZE/WRITE_SIZE counts, scaled by the copy-kernel calibration;
    None when the counters were taken on another version of the kernel
    source or another workload."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh).get(f"{kernel}@{workload}")
    except (OSError, ValueError):
        return None
    if not t or t.get("kernel_sha") != kernel_source_hash() or t.get("blocks") != n_blocks \
            or t.get("workload") != workload:
        return None
    return float(t["bytes_per_launch"])


def psnr_lost(frames, out, avail):
    """10 log10(255^2 / MSE) over the lost pixels, output clipped to [0, 255]."""
    lost = avail == 0
    err = np.clip(out[lost].astype(np.float64), 0.0, 255.0) - frames[lost].astype(np.float64)
    return float(10.0 * np.log10(255.0 ** 2 / np.mean(err ** 2)))


def time_steps(run, steps, stream):
    """Run `steps` steps bracketed by device synchronisation; returns wall
    ms per step and the mean of per-step HIP event durations."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        run()
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall * 1e3 / steps, float(np.mean([s.elapsed_time(e) for s, e in ev]))


def kernel_summary(batch, by_fft=False):
    """{kind: (launches, mean ms, F)} from the batch's timing records, or
    {(kind, F): ...} with by_fft."""
    acc = {}
    for kind, F, ms in batch.kernel_times():
        key = (kind, F) if by_fft else kind
        n, tot, _ = acc.get(key, (0, 0.0, F))
        acc[key] = (n + 1, tot + ms, F)
    return {k: (n, tot / n, F) for k, (n, tot, F) in acc.items()}


def _init_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _oracle_block(args):
    from oracle import cfse
    frames, avail, blk, rho, gamma, masked = args[:6]
    cand = args[6] if len(args) > 6 else None
    iters = args[7] if len(args) > 7 else None
    if cand is not None:
        F = int(blk["fft"])
        mask = np.zeros(F * F, dtype=bool)
        mask[np.asarray(cand, dtype=np.int64)] = True
        cand = mask.reshape(F, F)
    res = cfse.extrapolate_block(frames, avail, blk, rho, gamma, masked=masked, cand=cand, iters=iters)
    return None if res is None else (res["values"], res["lost"])


def fp32_error(wl, blocks, vals, out_gpu):
    """The GPU's FP32 result against the FP64 oracle's on the given blocks:
    largest pixel difference on B and PSNR over the blocks' lost pixels
    (each against the undistorted frames)."""
    ref, g, o, worst = [], [], [], 0.0
    for b, v in zip(blocks, vals):
        if v is None:
            continue
        f, y0, x0 = int(b["frame"]), int(b["y0"]), int(b["x0"])
        sl = (f, slice(y0, y0 + int(b["bh"])), slice(x0, x0 + int(b["bw"])))
        lost = v[1]
        gv = out_gpu[sl].astype(np.float64)[lost]
        ref.append(wl.frames[sl].astype(np.float64)[lost])
        g.append(gv)
        o.append(v[0][lost])
        worst = max(worst, float(np.abs(gv - v[0][lost]).max()))
    ref, g, o = np.concatenate(ref), np.concatenate(g), np.concatenate(o)
    lost = np.zeros(ref.shape, dtype=np.uint8)
    pg, po = psnr_lost(ref, g, lost), psnr_lost(ref, o, lost)
    return {"blocks": len(blocks), "max_abs_pixel_diff": worst, "psnr_gpu_db": pg, "psnr_oracle_db": po,
            "psnr_delta_db": pg - po}


def warm_error(wl, out_gpu, cand, args, n_sample=256, seed=6):
    """The warm leg's FP32 result against the FP64 oracle running the same
    restricted iterations (the GPU's candidates, count and step) on a
    seeded sample of blocks."""
    import multiprocessing as mp
    idx = np.sort(np.random.default_rng(seed).choice(len(wl.blocks), min(n_sample, len(wl.blocks)), replace=False))
    g = wl.gamma if args.gamma_r is None else args.gamma_r
    jobs = []
    for i in idx:
        b = wl.blocks[i].copy()
        f = int(b["frame"])
        b["frame"] = 0
        jobs.append((wl.frames[f:f + 1], wl.avail[f:f + 1], b, wl.rho, g, False, cand[i], args.ir))
    with mp.get_context("fork").Pool(len(os.sched_getaffinity(0)), initializer=_init_worker) as pool:
        vals = pool.map(_oracle_block, jobs, chunksize=1)
    return fp32_error(wl, wl.blocks[idx], vals, out_gpu)


def _spectral_block(args):
    from oracle import cfse, spectral
    frames, avail, blk, rho, gamma, masked = args
    s, A, B = cfse.area_of_block(frames, avail, blk, masked)
    w = cfse.weighting(*s.shape, rho, A)
    if w.sum() > 0:
        spectral.run(s, w, int(blk["fft"]), gamma, int(blk["iters"]))
    return 1


def cpu_baseline(wl, n_sample, seed=5, masked=False, out_gpu=None):
    """FP64 oracle, as it stands, over a seeded sample of the workload's
    blocks, one process per host core; with the GPU's output, the FP32
    error against the oracle on the same blocks."""
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0))
    idx = np.sort(np.random.default_rng(seed).choice(len(wl.blocks), n_sample, replace=False))
    # only the frames the sampled blocks touch are shipped to the workers
    jobs = []
    for i in idx:
        b = wl.blocks[i].copy()
        f = int(b["frame"])
        b["frame"] = 0
        jobs.append((wl.frames[f:f + 1], wl.avail[f:f + 1], b, wl.rho, wl.gamma, masked))
    with mp.get_context("fork").Pool(cores, initializer=_init_worker) as pool:
        pool.map(_oracle_block, jobs[:cores])            # warm the workers
        t0 = time.perf_counter()
        vals = pool.map(_oracle_block, jobs, chunksize=1)
        dt = time.perf_counter() - t0
        # the method in its frequency-domain form (FFTs and the spectral
        # update, FP64): the fair CPU speed reference, timed the same way
        pool.map(_spectral_block, jobs[:cores])
        t1 = time.perf_counter()
        pool.map(_spectral_block, jobs, chunksize=1)
        dt_fft = time.perf_counter() - t1
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except Exception:
        pass
    err = {} if out_gpu is None else {"fp32_error": fp32_error(wl, wl.blocks[idx], vals, out_gpu)}
    return {"value": n_sample / dt, "unit": "blocks/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_sample} seeded blocks of the same workload (FP64 direct projection, "
                      f"{int(wl.blocks[idx[0]]['iters'])} iterations each), {dt:.1f} s wall on {cpu}", **err,
            "fft_form": {"value": n_sample / dt_fft, "unit": "blocks/s", "cores": cores,
                         "kind": "FP64 frequency-domain form (oracle.spectral: FFTs, eq. (18) update)",
                         "seconds": dt_fft}}


def copy_calibration(args, rec, dev):
    """Three plain device copies of --copy-bytes bytes, the reference for
    scaling the FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    import torch
    if args.copy_bytes > 0:
        src = torch.randint(0, 255, (args.copy_bytes,), dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = args.copy_bytes


def _oracle_volume(args):
    from oracle import cfse3
    frames, avail, vol, rho, gamma = args
    cfse3.extrapolate_volume(frames, avail, vol, rho, gamma)
    return 1


def cpu_baseline_volumes(wl, n_sample, seed=5):
    """FP64 3-D oracle over a seeded sample of the clip's volumes, one
    process per host core."""
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0))
    idx = np.sort(np.random.default_rng(seed).choice(len(wl.blocks), n_sample, replace=False))
    jobs = []
    for i in idx:
        v = wl.blocks[i].copy()
        f0 = max(int(v["frame"]) - int(v["tborder"]), 0)
        f1 = min(int(v["frame"]) + int(v["bt"]) + int(v["tborder"]), len(wl.frames))
        v["frame"] -= f0
        jobs.append((wl.distorted[f0:f1], wl.avail[f0:f1], v, wl.rho, wl.gamma))
    with mp.get_context("fork").Pool(cores, initializer=_init_worker) as pool:
        pool.map(_oracle_volume, jobs[:cores])
        t0 = time.perf_counter()
        pool.map(_oracle_volume, jobs, chunksize=1)
        dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "volumes/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_sample} seeded volumes of the same clip (FP64 direct 3-D projection, "
                      f"{int(wl.blocks[idx[0]]['iters'])} iterations each), {dt:.1f} s wall"}


def bench_clip(args):
    """3-D (video) cFSE: lost 16x16x2 volumes of a 1920x1080x16 clip,
    plain (one kernel launch per step) and warm-started (network, top-K,
    restricted 3-D kernel); reported in volumes/s (not the blocks/s metric
    of the 2-D path): the warm leg's if it loses at most 0.1 dB."""
    import torch
    import paper_2204_14193_amd as fse
    from synth import workloads

    iters = 200 if args.iters == 100 else args.iters
    wl = workloads.clip_1080p_16x16x2(iters=iters)
    n = len(wl.blocks)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    out = img.to(torch.float32)
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    plan = fse.Plan(wl.rho, wl.gamma, iters)
    batch = fse.Batch3d(plan, wl.blocks, *wl.frames.shape)
    run = lambda: batch.run(img, av, out, status)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    # one launch per step: the step's HIP event pair brackets the kernel alone
    ms, ev_ms = time_steps(run, args.steps, stream)
    assert (status.cpu().numpy() == fse.BLOCK_OK).all()
    p_plain = psnr_lost(wl.frames, out.cpu().numpy(), wl.avail)
    legs = {"plain": {"volumes_per_s": n / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": ev_ms, "psnr_db": p_plain}}

    # learned warm start: the 2-D network's top-128 columns per volume, then
    # the 3-D iterations over those columns with every s
    from paper_2204_14193_amd import warm
    net = warm.Net(n, seed=0)
    net.load()
    ws = warm.WarmStart3d(net, batch, wl.blocks, plan)
    out_w = img.to(torch.float32)
    status_w = torch.zeros(n, dtype=torch.int32, device=dev)
    run_w = lambda: ws.run(img, av, out_w, status_w)
    for _ in range(args.warmup):
        run_w()
    torch.cuda.synchronize()
    ms_w, ev_w = time_steps(run_w, args.steps, stream)
    assert (status_w.cpu().numpy() == fse.BLOCK_OK).all() and int(ws.flags.sum().item()) == 0
    p_w = psnr_lost(wl.frames, out_w.cpu().numpy(), wl.avail)
    # the 3-D kernel alone (same candidates), for its roofline
    _, ev_k = time_steps(lambda: batch.run_warm(img, av, out_w, status_w, ws.cand, ws.flags), args.steps, stream)
    legs["warm"] = {"volumes_per_s": n / (ms_w * 1e-3), "ms_per_step": ms_w, "event_ms": ev_w,
                    "kernel_ms": ev_k, "psnr_db": p_w, "psnr_loss_db": p_plain - p_w,
                    "meets_bar": p_plain - p_w <= PSNR_BAR_DB, "speedup_vs_plain": ms / ms_w,
                    "candidates": "top-128 (k, l) of the 2-D network on the first lost frame, x 8 s"}
    ws.close()
    net.close()
    use_warm = legs["warm"]["meets_bar"]
    bins = 64 * 64 * 8
    lds_peak = fse.measure_lds_bandwidth() / 1e12
    vox = int(np.sum(wl.blocks["bt"].astype(np.int64) * wl.blocks["bh"] * wl.blocks["bw"]))
    if use_warm:
        kern, k_ms, rep_ms = "fse3d<warm>", ev_k, ms_w
        flop = n * iters * 1024 * FLOP_PER_BIN_ITER + vox * iters * FLOP_PER_PIXEL_COEF
    else:
        kern, k_ms, rep_ms = "fse3d", ev_ms, ms
        flop = n * iters * bins * FLOP_PER_BIN_ITER + vox * iters * FLOP_PER_PIXEL_COEF
    achieved = flop / (k_ms * 1e-3) / 1e12
    lds = n * iters * bins * 8 / (ev_ms * 1e-3) / 1e12      # plain kernel: the shifted W read, R_w in registers
    rec = {
        "metric": "3-D FSE volumes/s (16x16x2 loss, 64x64x8 FFT) plain vs warm-start at <=0.1 dB PSNR loss",
        "value": n / (rep_ms * 1e-3), "unit": "volumes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": rep_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "16x 1920x1080 synthetic frames (one image moving up to 3 px per frame), "
                               f"{n} lost 16x16x2 volumes (5% of the volume grid), border 16 px and 2 frames "
                               f"(48x48x6 area), 64x64x8 transform, rho 0.8, gamma 0.5, {iters} iterations",
                   "name": "clip-1080p", "volumes": n, "iters": iters,
                   "reported_leg": "warm" if use_warm else "plain"},
        "legs": legs,
        "mvoxel_per_s": vox / (rep_ms * 1e-3) / 1e6,
        "psnr_db": p_w if use_warm else p_plain,
        "roofline": {"bound": "alu", "kernel": kern, "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "frac_nonpacked": achieved / NONPACKED_FP32_TFLOPS, "kernel_ms": k_ms,
                     "traffic": measured_traffic(kern, n, "clip-1080p")},
        "lds_roofline": {"kernel": "fse3d", "achieved": lds, "peak": lds_peak, "peak_nominal": NOMINAL_LDS_TBPS,
                         "unit": "TB/s", "frac": lds / lds_peak,
                         "note": "plain kernel: algorithmic 8 B/bin/iteration (shifted W) against the measured LDS "
                                 "bandwidth"},
    }
    batch.close()
    plan.close()
    copy_calibration(args, rec, dev)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline_volumes(wl, min(args.cpu_sample, 48, n))
    print(json.dumps(rec), flush=True)


def _oracle_real_block(args):
    from oracle import rfse
    frames, avail, blk, rho, gamma = args
    rfse.extrapolate_block(frames, avail, blk, rho, gamma)
    return 1


def bench_real(args):
    """rFSE against cFSE at equal numbers of selected basis functions (the
    paper's runtime comparison, Section IV): the 6432 isolated 16x16 losses
    of eight 1080p frames, gamma 0.2; cFSE with n iterations, rFSE with n/2
    (each rFSE iteration adds a basis function and its conjugate), for n in
    50, 100, 200. One kernel launch per step; the step's HIP event pair
    brackets it."""
    import multiprocessing as mp
    import torch
    import paper_2204_14193_amd as fse
    from synth import workloads

    gamma = 0.2
    wl = workloads.random_1080p_16x16(seeds=tuple(range(99, 99 + args.frames)), iters=100)
    n = len(wl.blocks)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    stream = torch.cuda.current_stream()
    n_pix = int(wl.blocks["bh"].astype(np.int64) @ wl.blocks["bw"].astype(np.int64))

    def leg(iters, real):
        blocks = wl.blocks.copy()
        blocks["iters"] = iters
        out = img.to(torch.float32)
        status = torch.zeros(n, dtype=torch.int32, device=dev)
        plan = fse.Plan(wl.rho, gamma, iters, real=real)
        batch = fse.Batch(plan, blocks, *wl.frames.shape)
        run = lambda: batch.run(img, av, out, status)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        ms, ev_ms = time_steps(run, args.steps, stream)
        assert (status.cpu().numpy() == fse.BLOCK_OK).all()
        info = batch.launch_info(64)
        batch.close()
        plan.close()
        return {"iters": iters, "blocks_per_s": n / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": ev_ms,
                "us_per_block": ms * 1e3 / n, "psnr_db": psnr_lost(wl.frames, out.cpu().numpy(), wl.avail),
                "grid": info["grid"], "threads": info["threads"], "lds_bytes": info["lds_bytes"]}

    sweep = {}
    for nbf in (50, 100, 200):
        c, r, ri, rp = leg(nbf, False), leg(nbf // 2, True), leg(nbf // 2, "inloop"), leg(nbf // 2, "power")
        sweep[str(nbf)] = {"cfse": c, "rfse": r, "rfse_inloop": ri, "rfse_power": rp,
                           "rfse_over_cfse_time": r["ms_per_step"] / c["ms_per_step"],
                           "rfse_inloop_over_cfse_time": ri["ms_per_step"] / c["ms_per_step"],
                           "psnr_rfse_minus_cfse_db": r["psnr_db"] - c["psnr_db"],
                           "psnr_rfse_power_minus_cfse_db": rp["psnr_db"] - c["psnr_db"]}
    main_leg = sweep["100"]["rfse"]
    # 2112 half-plane bins per iteration: the pair update (8 FMA) and the
    # energy decrease (7 FLOP); 4 FLOP per pixel and iteration for the model
    flop = n * main_leg["iters"] * (2112 * 23) + n_pix * main_leg["iters"] * FLOP_PER_PIXEL_COEF
    achieved = flop / (main_leg["kernel_ms"] * 1e-3) / 1e12
    rec = {
        "metric": "rFSE blocks/s (16² loss, 64² FFT, 100 basis functions)", "value": main_leg["blocks_per_s"],
        "unit": "blocks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.frames}x 1920x1080 synthetic frames, 804 isolated 16x16 losses per frame, "
                               "border 16 (48x48 area), 64x64 transform, rho 0.8, gamma 0.2; rFSE with n/2 "
                               "iterations against cFSE with n, n = 50, 100, 200 basis functions",
                   "name": "rfse-1080p", "blocks": n},
        "sweep": sweep,
        "roofline": {"bound": "alu", "kernel": "fse_real64", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "frac_nonpacked": achieved / NONPACKED_FP32_TFLOPS, "kernel_ms": main_leg["kernel_ms"],
                     "traffic": measured_traffic("fse_real64", n, "rfse-1080p")},
    }
    copy_calibration(args, rec, dev)
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        m = min(args.cpu_sample, n)
        idx = np.sort(np.random.default_rng(5).choice(n, m, replace=False))
        jobs = []
        for i in idx:
            b = wl.blocks[i].copy()
            f = int(b["frame"])
            b["frame"] = 0
            b["iters"] = 50
            jobs.append((wl.distorted[f:f + 1], wl.avail[f:f + 1], b, wl.rho, gamma))
        with mp.get_context("fork").Pool(cores, initializer=_init_worker) as pool:
            pool.map(_oracle_real_block, jobs[:cores])
            t0 = time.perf_counter()
            pool.map(_oracle_real_block, jobs, chunksize=1)
            dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": m / dt, "unit": "blocks/s", "cores": cores, "kind": "oracle",
                               "sample": f"{m} seeded blocks of the same workload (FP64 rFSE by direct projection, "
                                         f"50 iterations each), {dt:.1f} s wall"}
    print(json.dumps(rec), flush=True)


def _oracle_fixed_block(args):
    from oracle import fixed
    frames, avail, blk, rho, gamma = args
    fixed.extrapolate_block(frames, avail, blk, rho, gamma)
    return 1


INT64_MAD_PEAK = 256 * 4 * 16 * 2.4e9 / 4   # 64-bit multiply-add, quarter rate (assumed)


def bench_fixed(args):
    """Fixed-point cFSE against the FP32 kernel on the 6432 isolated 16x16
    losses of eight 1080p frames (100 iterations, gamma 0.5). One kernel
    launch per step; the step's HIP event pair brackets it."""
    import multiprocessing as mp
    import torch
    import paper_2204_14193_amd as fse
    from synth import workloads

    wl = workloads.random_1080p_16x16(seeds=tuple(range(99, 99 + args.frames)), iters=args.iters)
    n = len(wl.blocks)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    stream = torch.cuda.current_stream()

    def leg(fixed_point):
        out = img.to(torch.float32)
        status = torch.zeros(n, dtype=torch.int32, device=dev)
        plan = fse.Plan(wl.rho, wl.gamma, args.iters, fixed=fixed_point)
        batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
        run = lambda: batch.run(img, av, out, status)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        ms, ev_ms = time_steps(run, args.steps, stream)
        assert (status.cpu().numpy() == fse.BLOCK_OK).all()
        info = batch.launch_info(64)
        batch.close()
        plan.close()
        return {"blocks_per_s": n / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": ev_ms,
                "psnr_db": psnr_lost(wl.frames, out.cpu().numpy(), wl.avail), **info}

    legs = {"float": leg(False), "fixed": leg(True)}
    fx = legs["fixed"]
    # 64-bit multiply-adds per launch: the two transform passes (4 per
    # complex term), 6 per bin and iteration (score 2, update 4), 2 per
    # pixel and iteration for the model
    M = N = 48
    mads = n * (4 * (M * N * 64 + 64 * 64 * M) + args.iters * 64 * 64 * 6 + args.iters * 256 * 2)
    achieved = mads / (fx["kernel_ms"] * 1e-3)
    rec = {
        "metric": "fixed-point cFSE blocks/s (16² loss, 64² FFT, 100 iterations)", "value": fx["blocks_per_s"],
        "unit": "blocks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": fx["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32/int64", "data": "synthetic",
        "config": {"workload": f"{args.frames}x 1920x1080 synthetic frames, 804 isolated 16x16 losses per frame, "
                               f"border 16 (48x48 area), 64x64 transform, rho 0.8, gamma 0.5, {args.iters} "
                               "iterations; fixed-point encoding against the FP32 kernel",
                   "name": "fixed-1080p", "blocks": n},
        "legs": legs, "psnr_fixed_minus_float_db": fx["psnr_db"] - legs["float"]["psnr_db"],
        "time_fixed_over_float": fx["ms_per_step"] / legs["float"]["ms_per_step"],
        "roofline": {"bound": "alu", "kernel": "fse_fixed64", "achieved": achieved / 1e12, "peak": INT64_MAD_PEAK / 1e12,
                     "unit": "T int64-MAD/s", "frac": achieved / INT64_MAD_PEAK, "kernel_ms": fx["kernel_ms"],
                     "traffic": measured_traffic("fse_fixed64", n, "fixed-1080p")},
    }
    copy_calibration(args, rec, dev)
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        m = min(args.cpu_sample, n)
        idx = np.sort(np.random.default_rng(5).choice(n, m, replace=False))
        jobs = []
        for i in idx:
            b = wl.blocks[i].copy()
            f = int(b["frame"])
            b["frame"] = 0
            jobs.append((wl.distorted[f:f + 1], wl.avail[f:f + 1], b, float(np.float32(wl.rho)),
                         float(np.float32(wl.gamma))))
        with mp.get_context("fork").Pool(cores, initializer=_init_worker) as pool:
            pool.map(_oracle_fixed_block, jobs[:cores])
            t0 = time.perf_counter()
            pool.map(_oracle_fixed_block, jobs, chunksize=1)
            dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": m / dt, "unit": "blocks/s", "cores": cores, "kind": "oracle",
                               "sample": f"{m} seeded blocks of the same workload (integer oracle, "
                                         f"{args.iters} iterations each), {dt:.1f} s wall"}
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--workload", default="random-1080p-16x16",
                    choices=["random-1080p-16x16", "random-1080p-8x8", "mixed-4k", "strokes-1080p", "clip-1080p",
                             "rfse-1080p", "fixed-1080p"],
                    help="the metric's workload (default) or one of the other configurations (plain only)")
    ap.add_argument("--kc", type=int, default=None, help="warm start: candidate bins per block "
                                                           "(default: the packaged network's operating point)")
    ap.add_argument("--ir", type=int, default=None, help="warm start: restricted iterations (default: as --kc)")
    ap.add_argument("--gamma-r", type=float, default=None, help="warm start: step of the restricted iterations "
                                                               "(default: as --kc; <= 0: the plan's gamma)")
    ap.add_argument("--no-ablation", action="store_true", help="skip the warm start's non-learned candidate legs")
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1024,
                    help="blocks timed on the FP64 oracle (about 20-30 s of CPU work; 3-D: at most 48 volumes)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the (untimed) autotuner")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run 3 plain device copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    from paper_2204_14193_amd import warm as _warm
    args.kc = _warm.KC if args.kc is None else args.kc
    args.ir = _warm.RESTRICTED_ITERS if args.ir is None else args.ir
    if args.gamma_r is None:
        args.gamma_r = _warm.RESTRICTED_GAMMA
    elif args.gamma_r <= 0:
        args.gamma_r = None
    if args.gpus != 1:
        print("this benchmark runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "clip-1080p":
        bench_clip(args)
        return
    if args.workload == "rfse-1080p":
        bench_real(args)
        return
    if args.workload == "fixed-1080p":
        bench_fixed(args)
        return

    import torch
    import paper_2204_14193_amd as fse
    from synth import workloads

    warm_ok = args.workload == "random-1080p-16x16" and not args.no_warm
    if args.workload == "random-1080p-16x16":
        wl = workloads.random_1080p_16x16(seeds=tuple(range(99, 99 + args.frames)), iters=args.iters)
        desc = (f"{args.frames}x 1920x1080 synthetic frames, 804 isolated 16x16 losses per frame (10%), "
                f"border 16 (48x48 area), 64x64 transform, rho 0.8, gamma 0.5; plain FSE {args.iters} iterations "
                f"vs learned warm start (top-{args.kc} candidates, {args.ir} restricted iterations, step "
                f"{0.5 if args.gamma_r is None else args.gamma_r})")
    elif args.workload == "random-1080p-8x8":
        wl = workloads.random_1080p_8x8(iters=200)
        desc = ("1920x1080 synthetic frame, 3240 isolated 8x8 losses (10%), border 16 (40x40 area), "
                "64x64 transform, rho 0.8, gamma 0.5, 200 iterations, plain FSE")
    elif args.workload == "strokes-1080p":
        nfr = min(args.frames, 3)
        wl = workloads.strokes_1080p(seeds=tuple(range(31, 31 + nfr)), iters=args.iters)
        desc = (f"{nfr}x 1920x1080 synthetic frames, scribble losses (6% of the pixels, strokes 2-7 px wide) "
                f"covered by 16x16 tiles, border 16 (48x48 area), 64x64 transform, rho 0.8, gamma 0.5, "
                f"{args.iters} iterations, plain FSE with mask-driven loss areas")
    else:
        wl = workloads.mixed_4k(seeds=tuple(range(2, 2 + args.frames)))
        desc = (f"{args.frames}x 3840x2160 synthetic frames, 305 losses each of 4, 8, 16, 32 px per frame (5%), "
                "border 8-16, transform 32/64/128, 50-500 iterations, plain FSE")
    masked = args.workload == "strokes-1080p"
    n = len(wl.blocks)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    stream = torch.cuda.current_stream()
    legs = {}

    # ---- plain FSE
    out = img.to(torch.float32)
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    plan = fse.Plan(wl.rho, wl.gamma, int(wl.blocks["iters"].max()), masked=masked)
    batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    tuning = batch.autotune(img, av, out, status, reps=2) if not args.no_tune else []
    classes = sorted(set(int(f) for f in wl.blocks["fft"]))
    info = {F: batch.launch_info(F) for F in classes}
    run_plain = lambda: batch.run(img, av, out, status)
    for _ in range(args.warmup):
        run_plain()
    torch.cuda.synchronize()
    # kernel times from a pass with an event pair around each launch, then
    # the reported time from the same number of steps without them (the
    # events cost dispatch time; the first pass also warms the clocks)
    batch.set_timing(len(classes) * args.steps)
    ms_ins, _ = time_steps(run_plain, args.steps, stream)
    kern = kernel_summary(batch, by_fft=True)
    batch.set_timing(0)
    ms, ev_ms = time_steps(run_plain, args.steps, stream)
    assert (status.cpu().numpy() == fse.BLOCK_OK).all()
    bin_iters = int(np.sum(wl.blocks["fft"].astype(np.int64) ** 2 * wl.blocks["iters"].astype(np.int64)))
    out_plain = out.cpu().numpy()
    legs["plain"] = {"blocks_per_s": n / (ms * 1e-3), "ms_per_step": ms, "event_ms": ev_ms,
                     "instrumented_ms_per_step": ms_ins,
                     "psnr_db": psnr_lost(wl.frames, out_plain, wl.avail),
                     "kernels": {f"fse_persistent<{F},{info[F]['threads']}>": {"ms": kern[("plain", F)][1], **info[F]}
                                 for F in classes},
                     "autotune_us": {f"{F}/{t}": round(us, 1) for F, t, us in tuning}}
    # one launch per transform size: the roofline counts all of them, over
    # their summed kernel time
    plain_roof = {"kernel": " + ".join(f"fse_persistent<{F},{info[F]['threads']}>" for F in classes),
                  "flop": FLOP_PER_BIN_ITER * bin_iters, "ms": sum(kern[("plain", F)][1] for F in classes)}
    batch.close()
    plan.close()

    # ---- learned warm start (restricted iterations only)
    warm_roof = None
    if warm_ok:
        from paper_2204_14193_amd import warm
        wblocks = wl.blocks.copy()
        wblocks["iters"] = 0
        out_w = img.to(torch.float32)
        status_w = torch.zeros(n, dtype=torch.int32, device=dev)
        plan_w = fse.Plan(wl.rho, wl.gamma, args.ir + args.iters)
        batch_w = fse.Batch(plan_w, wblocks, *wl.frames.shape)
        net = warm.Net(n, seed=0)
        net.load()
        ws = warm.WarmStart(net, batch_w, args.kc, args.ir, args.iters, args.gamma_r)
        run_warm = lambda: ws.run(img, av, out_w, status_w)
        for _ in range(args.warmup):
            run_warm()
        torch.cuda.synchronize()
        batch_w.set_timing(2 * args.steps)
        ms_w_ins, _ = time_steps(run_warm, args.steps, stream)
        kw = kernel_summary(batch_w)
        batch_w.set_timing(0)
        ms_w, ev_w = time_steps(run_warm, args.steps, stream)
        assert (status_w.cpu().numpy() == fse.BLOCK_OK).all()
        fallbacks = int(ws.flags.sum().item())
        out_warm = out_w.cpu().numpy()
        warm_cand = ws.cand.cpu().numpy()
        p_w = psnr_lost(wl.frames, out_warm, wl.avail)
        with open(warm.WEIGHTS, "rb") as fh:
            wsha = hashlib.sha256(fh.read()).hexdigest()[:16]
        legs["warm"] = {"blocks_per_s": n / (ms_w * 1e-3), "ms_per_step": ms_w, "event_ms": ev_w,
                        "instrumented_ms_per_step": ms_w_ins, "psnr_db": p_w,
                        "psnr_loss_db": legs["plain"]["psnr_db"] - p_w,
                        "meets_bar": legs["plain"]["psnr_db"] - p_w <= PSNR_BAR_DB,
                        "speedup_vs_plain": legs["plain"]["ms_per_step"] / ms_w, "fallbacks": fallbacks,
                        "kc": args.kc, "restricted_iters": args.ir,
                        "restricted_step": wl.gamma if args.gamma_r is None else args.gamma_r, "weights_sha": wsha,
                        "kernels": {("fse_restricted<%d>" % args.kc if k == "restricted" else
                                     "fse_persistent<64,512,%d,prep>" % args.kc): {"ms": v[1], "launches": v[0]}
                                    for k, v in kw.items()}}
        if not args.no_ablation:
            # what the network adds: the same warm start (K, restricted
            # iterations and step) with candidate sets that are not learned
            from paper_2204_14193_amd import operating_point as op
            cand = torch.empty_like(ws.cand)
            flg = torch.zeros_like(ws.flags)
            power = torch.empty((n, 4096), dtype=torch.float32, device=dev)
            low = torch.from_numpy(np.tile(op.lowfreq_bins(args.kc), (n, 1))).to(dev)
            props = {"spectrum": lambda: (warm.initial_power(batch_w, img, av, power),
                                          warm.topk(power, args.kc, cand, flg)),
                     "lowfreq": lambda: cand.copy_(low)}
            for name, propose in props.items():
                out_a = img.to(torch.float32)
                run_a = lambda: (propose(), warm.warm_extrapolate(batch_w, img, av, out_a, status_w, cand, flg,
                                                                  args.kc, args.ir, args.iters))
                for _ in range(args.warmup):
                    run_a()
                ms_a, _ = time_steps(run_a, args.steps, stream)
                assert (status_w.cpu().numpy() == fse.BLOCK_OK).all()
                p_a = psnr_lost(wl.frames, out_a.cpu().numpy(), wl.avail)
                legs["warm_" + name] = {
                    "candidates": {"spectrum": "top-K of |DFT(s w)|^2 (the first selection's criterion)",
                                   "lowfreq": "the K lowest frequencies, the same for every block"}[name],
                    "blocks_per_s": n / (ms_a * 1e-3), "ms_per_step": ms_a, "psnr_db": p_a,
                    "psnr_loss_db": legs["plain"]["psnr_db"] - p_a,
                    "meets_bar": legs["plain"]["psnr_db"] - p_a <= PSNR_BAR_DB,
                    "kc": args.kc, "restricted_iters": args.ir}
        try:
            with open(os.path.join(ROOT, "paper_2204_14193_amd", "weights", "operating_point.json")) as fh:
                opj = json.load(fh)
            legs["warm"]["operating_point"] = {
                "chosen": opj["chosen"], "rule": opj["rule"], "loss_target_db": opj["loss_target_db"],
                "validation_seeds": opj["validation_seeds"],
                "validation_loss_db": opj["validation_best"]["loss_db"],
                "is_default": (args.kc, args.ir) == (warm.KC, warm.RESTRICTED_ITERS)}
        except (OSError, ValueError, KeyError):
            pass
        n_pix = int(wl.blocks["bh"].astype(np.int64) @ wl.blocks["bw"].astype(np.int64))
        warm_roof = {"kernel": "fse_restricted<%d>" % args.kc,
                     "flop": n * args.ir * args.kc * FLOP_PER_BIN_ITER + n_pix * args.ir * FLOP_PER_PIXEL_COEF,
                     "ms": kw["restricted"][1], "prep_ms": kw["warm_prep"][1]}
        batch_w.close()
        plan_w.close()
        net.close()

    use_warm = warm_ok and legs["warm"]["meets_bar"]
    leg = legs["warm" if use_warm else "plain"]
    roof = warm_roof if use_warm else plain_roof
    achieved = roof["flop"] / (roof["ms"] * 1e-3) / 1e12
    if masked:
        lost_px = int(sum(int((wl.avail[int(b["frame"]), int(b["y0"]):int(b["y0"]) + int(b["bh"]),
                                        int(b["x0"]):int(b["x0"]) + int(b["bw"])] == 0).sum()) for b in wl.blocks))
    else:
        lost_px = int(wl.blocks["bh"].astype(np.int64) @ wl.blocks["bw"].astype(np.int64))
    rec = {
        "metric": METRIC, "value": leg["blocks_per_s"], "unit": "blocks/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "blocks": n, "reported_leg": "warm" if use_warm else "plain",
                   "fft": classes[0] if len(classes) == 1 else classes,
                   "iters": int(wl.blocks["iters"][0]) if len(set(wl.blocks["iters"].tolist())) == 1 else "mixed",
                   "rho": wl.rho, "gamma": wl.gamma},
        "legs": legs,
        # lost pixels concealed per second (each block's B; masked tiles count their lost pixels only)
        "mpixel_per_s": lost_px / (leg["ms_per_step"] * 1e-3) / 1e6,
        "roofline": {"bound": "alu", "kernel": roof["kernel"], "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "frac_nonpacked": achieved / NONPACKED_FP32_TFLOPS, "kernel_ms": roof["ms"],
                     "traffic": measured_traffic(roof["kernel"], n, args.workload)},
    }
    lds_peak = fse.measure_lds_bandwidth() / 1e12
    rec["lds_peak_measured"] = {"value": lds_peak, "unit": "TB/s", "nominal": NOMINAL_LDS_TBPS,
                                "how": "fse_measure_lds_bandwidth: conflict-free 16-byte LDS reads on every CU"}
    if not use_warm:
        lds_bytes = LDS_BYTES_PER_BIN_ITER * bin_iters
        rec["lds_roofline"] = {"achieved": lds_bytes / (roof["ms"] * 1e-3) / 1e12, "peak": lds_peak,
                               "peak_nominal": NOMINAL_LDS_TBPS,
                               "unit": "TB/s", "frac": lds_bytes / (roof["ms"] * 1e-3) / 1e12 / lds_peak,
                               "note": "algorithmic 24 B/bin/iteration (R_w read and written, shifted W read) "
                                       "against the measured LDS bandwidth; only the 8-B W read touches LDS, "
                                       "R_w stays in registers"}
    copy_calibration(args, rec, dev)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl, min(args.cpu_sample, n), masked=masked, out_gpu=out_plain)
        if use_warm:
            rec["cpu_baseline"]["warm_fp32_error"] = warm_error(wl, out_warm, warm_cand, args)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
