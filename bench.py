"""Throughput of complex-valued FSE on one MI355X.

A step conceals every lost block of a batch of eight synthetic 1920x1080
frames (804 isolated 16x16 losses per frame, 10% of the 16x16 grid, border
16 so each area is 48x48, 64x64 transform, rho 0.8, gamma 0.5, 100
iterations): 6432 blocks in one persistent launch, inputs resident in HBM.

Prints one JSON line: blocks/s (value), lost Mpixel/s, the roofline of the
dominant kernel, and the FP64 CPU oracle timed on the host's cores over a
bounded sample of the same blocks.
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
PEAK_FP32_TFLOPS = 157.3        # MI355X FP32 vector, published
NOMINAL_LDS_TBPS = 78.6         # 256 CU x 128 B/clk x 2.4 GHz
FLOP_PER_BIN_ITER = 11          # complex multiply-subtract (8) + |R|^2 (3), eq. (18) + eq. (12)
LDS_BYTES_PER_BIN_ITER = 24     # read R_w, read shifted W, write R_w (spectra resident on chip)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fse_persistent_64.json")


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2204_14193_amd", "csrc", "fse_kernels.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n_blocks, workload):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    counts, scaled by the copy-kernel calibration; None when the counters
    were taken on another version of the kernel."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_source_hash() or t.get("blocks") != n_blocks or t.get("workload") != workload:
        return None
    return float(t["bytes_per_launch"])


def _init_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _oracle_block(args):
    from oracle import cfse
    frames, avail, blk, rho, gamma = args
    cfse.extrapolate_block(frames, avail, blk, rho, gamma)
    return 1


def cpu_baseline(wl, n_sample, seed=5):
    """FP64 oracle, as it stands, over a seeded sample of the workload's
    blocks, one process per host core."""
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0))
    idx = np.sort(np.random.default_rng(seed).choice(len(wl.blocks), n_sample, replace=False))
    # only the frames the sampled blocks touch are shipped to the workers
    jobs = []
    for i in idx:
        b = wl.blocks[i].copy()
        f = int(b["frame"])
        b["frame"] = 0
        jobs.append((wl.frames[f:f + 1], wl.avail[f:f + 1], b, wl.rho, wl.gamma))
    with mp.get_context("fork").Pool(cores, initializer=_init_worker) as pool:
        pool.map(_oracle_block, jobs[:cores])            # warm the workers
        t0 = time.perf_counter()
        pool.map(_oracle_block, jobs, chunksize=1)
        dt = time.perf_counter() - t0
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except Exception:
        pass
    return {"value": n_sample / dt, "unit": "blocks/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_sample} seeded blocks of the same workload (FP64 direct projection, "
                      f"{int(wl.blocks[idx[0]]['iters'])} iterations each), {dt:.1f} s wall on {cpu}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--workload", default="random-1080p-16x16",
                    choices=["random-1080p-16x16", "random-1080p-8x8", "mixed-4k"],
                    help="the metric's workload (default) or one of the other configurations")
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the (untimed) autotuner")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run 3 plain device copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2204_14193_amd as fse
    from synth import workloads

    if args.workload == "random-1080p-16x16":
        wl = workloads.random_1080p_16x16(seeds=tuple(range(99, 99 + args.frames)), iters=args.iters)
        desc = (f"{args.frames}x 1920x1080 synthetic frames, 804 isolated 16x16 losses per frame (10%), "
                f"border 16 (48x48 area), 64x64 transform, rho 0.8, gamma 0.5, {args.iters} iterations, plain FSE")
    elif args.workload == "random-1080p-8x8":
        wl = workloads.random_1080p_8x8(iters=200)
        desc = ("1920x1080 synthetic frame, 3240 isolated 8x8 losses (10%), border 16 (40x40 area), "
                "64x64 transform, rho 0.8, gamma 0.5, 200 iterations, plain FSE")
    else:
        wl = workloads.mixed_4k(seeds=tuple(range(2, 2 + args.frames)))
        desc = (f"{args.frames}x 3840x2160 synthetic frames, 305 losses each of 4, 8, 16, 32 px per frame (5%), "
                "border 8-16, transform 32/64/128, 50-500 iterations, plain FSE")
    n = len(wl.blocks)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    out = img.to(torch.float32)
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    plan = fse.Plan(wl.rho, wl.gamma, int(wl.blocks["iters"].max()))
    batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    stream = torch.cuda.current_stream()
    tuning = batch.autotune(img, av, out, status, reps=2) if not args.no_tune else []
    classes = sorted(set(int(f) for f in wl.blocks["fft"]))
    info = {F: batch.launch_info(F) for F in classes}

    for _ in range(args.warmup):
        batch.run(img, av, out, status)
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == fse.BLOCK_OK).all()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        batch.run(img, av, out, status)
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = float(np.mean([s.elapsed_time(e) for s, e in ev]))
    ms_per_step = wall * 1e3 / args.steps

    blocks_per_s = n / (ms_per_step * 1e-3)
    lost_px = int(wl.blocks["bh"].astype(np.int64) @ wl.blocks["bw"].astype(np.int64))
    bin_iters = int(np.sum(wl.blocks["fft"].astype(np.int64) ** 2 * wl.blocks["iters"].astype(np.int64)))
    flop = FLOP_PER_BIN_ITER * bin_iters
    achieved = flop / (launch_ms * 1e-3) / 1e12
    lds_bytes = LDS_BYTES_PER_BIN_ITER * bin_iters
    rec = {
        "metric": METRIC, "value": blocks_per_s, "unit": "blocks/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "blocks": n,
                   "fft": classes[0] if len(classes) == 1 else classes,
                   "iters": int(wl.blocks["iters"][0]) if len(set(wl.blocks["iters"].tolist())) == 1 else "mixed",
                   "rho": wl.rho, "gamma": wl.gamma},
        "mpixel_per_s": lost_px / (ms_per_step * 1e-3) / 1e6,
        "launch": {"kernels": {f"fse_persistent<{F},{info[F]['threads']}>": info[F] for F in classes},
                   "avg_ms": launch_ms, "autotune_us": {f"{F}/{t}": round(us, 1) for F, t, us in tuning}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(n, args.workload)},
        "lds_roofline": {"achieved": lds_bytes / (launch_ms * 1e-3) / 1e12, "peak": NOMINAL_LDS_TBPS,
                         "unit": "TB/s", "frac": lds_bytes / (launch_ms * 1e-3) / 1e12 / NOMINAL_LDS_TBPS,
                         "note": "algorithmic 24 B/bin/iteration against the nominal LDS bandwidth"},
    }
    if args.copy_bytes > 0:
        src = torch.randint(0, 255, (args.copy_bytes,), dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = args.copy_bytes
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl, min(args.cpu_sample, n))
    batch.close()
    plan.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
