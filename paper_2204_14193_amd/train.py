"""Train the warm-start network on blocks concealed by plain FSE.

Data: synthetic 1920x1080 frames with 10% of the 16x16 grid lost
(non-adjacent), border 16 (48x48 areas). Each block's target is the set of
bins that plain FSE (64x64 transform, rho 0.8, gamma 0.5, 100 iterations,
this library's GPU kernels) selects. The network learns to score bins so
that its top-K set covers them (binary cross-entropy, positives weighted).
Forward, backward and Adam run in libfse; torch only holds the buffers.

    python -m paper_2204_14193_amd.train --blocks 1600000 --epochs 40
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

H, W = 1080, 1920


def _frame_job(seed):
    from synth import images, losses
    frame = images.synthetic_image(H, W, seed)
    blocks = losses.random_grid_losses(H, W, 16, 0.10, seed, 16, 64, 100)
    return frame, losses.blocks_to_array(blocks)


def make_frames(first_seed, n_frames, workers=16):
    """Frames and block lists for seeds first_seed ... (frame index f)."""
    seeds = list(range(first_seed, first_seed + n_frames))
    with mp.get_context("fork").Pool(min(workers, n_frames)) as pool:
        res = pool.map(_frame_job, seeds)
    frames = np.stack([r[0] for r in res])
    blocks = []
    for f, (_, b) in enumerate(res):
        b = b.copy()
        b["frame"] = f
        blocks.append(b)
    return frames, np.concatenate(blocks)


def targets_from_trace(trace, F=64):
    """Bit masks [n][128] (int32 view) of the bins each block selected."""
    bins = trace["u"].astype(np.int64) * F + trace["v"].astype(np.int64)      # [n, I]
    n = bins.shape[0]
    onehot = np.zeros((n, 4096), dtype=bool)
    np.put_along_axis(onehot, bins, True, axis=1)
    words = onehot.reshape(n, 128, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)
    return words.sum(axis=2).astype(np.uint32).view(np.int32)


def build_dataset(first_seed, n_blocks, dev, log=print):
    """Network inputs (GPU, BF16) and target bits (GPU, int32) for n_blocks
    blocks cut from consecutive seeds."""
    import torch
    from . import fse, warm
    from synth import losses
    n_frames = math.ceil(n_blocks / 804)
    t0 = time.time()
    frames, blocks = make_frames(first_seed, n_frames)
    log(f"frames: {n_frames} in {time.time() - t0:.1f} s, {len(blocks)} blocks")
    avail = losses.availability_mask(frames.shape, losses.array_to_blocks(blocks))
    img = torch.from_numpy(frames * avail).to(dev)
    av = torch.from_numpy(avail).to(dev)
    xs, bits = [], []
    chunk = 8 * 804
    out = torch.zeros(frames.shape, dtype=torch.float32, device=dev)
    for s in range(0, len(blocks), chunk):
        blk = blocks[s:s + chunk]
        plan = fse.Plan(0.8, 0.5, 100)
        batch = fse.Batch(plan, blk, *frames.shape)
        status = torch.zeros(len(blk), dtype=torch.int32, device=dev)
        tr = torch.zeros((len(blk), 100 * 16), dtype=torch.uint8, device=dev)
        batch.run(img, av, out, status, tr)
        x = torch.empty((len(blk), 48, 48, 2), dtype=torch.bfloat16, device=dev)
        warm.patches(batch, img, av, x)
        torch.cuda.synchronize()
        assert (status.cpu().numpy() == 0).all()
        trace = tr.cpu().numpy().view(fse.TRACE_DTYPE).reshape(len(blk), 100)
        bits.append(torch.from_numpy(targets_from_trace(trace)).to(dev))
        xs.append(x)
        batch.close()
        plan.close()
    x = torch.cat(xs)[:n_blocks]
    b = torch.cat(bits)[:n_blocks]
    log(f"dataset: {x.shape[0]} blocks, {time.time() - t0:.1f} s")
    return x, b


def train(x, bits, epochs, batch_size=256, lr=2e-3, pos_weight=4.0, seed=0, log=print):
    import torch
    from . import warm
    n = x.shape[0] // batch_size * batch_size
    net = warm.Net(batch_size, seed=seed)
    logits = torch.empty((batch_size, 4096), dtype=torch.float32, device=x.device)
    loss = torch.zeros(1, dtype=torch.float32, device=x.device)
    rng = np.random.default_rng(seed)
    steps_per_epoch = n // batch_size
    total = epochs * steps_per_epoch
    step = 0
    t0 = time.time()
    history = []
    for ep in range(epochs):
        loss.zero_()
        for bi in rng.permutation(steps_per_epoch):
            xb = x[bi * batch_size:(bi + 1) * batch_size]
            tb = bits[bi * batch_size:(bi + 1) * batch_size]
            net.forward(xb, logits, keep=True)
            net.backward(xb, logits, tb, pos_weight, loss)
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / total))
            net.adam(cur, 0.9, 0.999, 1e-8)
            step += 1
        torch.cuda.synchronize()
        mean = loss.item() / steps_per_epoch
        history.append(mean)
        log(f"epoch {ep}: loss {mean:.5f}, {time.time() - t0:.1f} s")
    return net, history


def psnr_lost(reference, reconstruction, avail):
    """10*log10(255^2 / MSE) over the lost pixels, reconstruction clipped to [0, 255]."""
    lost = avail == 0
    err = np.clip(reconstruction[lost].astype(np.float64), 0.0, 255.0) - reference[lost].astype(np.float64)
    return float(10.0 * np.log10(255.0 ** 2 / np.mean(err ** 2)))


def evaluate(net, seeds=tuple(range(99, 107)), configs=((384, 110), (512, 100), (512, 110)), plain_iters=100, reps=5,
             log=print):
    """PSNR over the lost pixels and blocks/s of plain FSE and of the warm
    start (restricted iterations only; (K, restricted iterations) per
    config) on held-out frames."""
    import torch
    from . import fse, warm
    from synth import workloads
    dev = torch.device("cuda:0")
    res = {}
    wl = workloads.random_1080p_16x16(seeds=tuple(seeds), iters=plain_iters)
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    n = len(wl.blocks)
    infer = warm.Net(n, seed=0)
    infer.set_params(net.get_params())
    modes = [("plain", None)] + [(f"warm_k{k}_ir{ir}", (k, ir)) for k, ir in configs]
    for mode, cfg in modes:
        blocks = wl.blocks.copy()
        if cfg is not None:
            blocks["iters"] = 0
        plan = fse.Plan(wl.rho, wl.gamma, 4096)
        batch = fse.Batch(plan, blocks, *wl.frames.shape)
        out = img.to(torch.float32)
        status = torch.zeros(n, dtype=torch.int32, device=dev)
        if cfg is None:
            batch.autotune(img, av, out, status, reps=2)
            run = lambda: batch.run(img, av, out, status)
        else:
            ws = warm.WarmStart(infer, batch, cfg[0], cfg[1], plain_iters)
            run = lambda: ws.run(img, av, out, status)
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        o = out.cpu().numpy()
        st = status.cpu().numpy()
        r = {"psnr": psnr_lost(wl.frames, o, wl.avail), "ms": ms, "blocks_per_s": n / (ms * 1e-3),
             "ok": int((st == 0).sum())}
        if cfg is not None:
            r["fallbacks"] = int(ws.flags.sum().item())
            r["psnr_loss_db"] = res["plain"]["psnr"] - r["psnr"]
            r["speedup"] = r["blocks_per_s"] / res["plain"]["blocks_per_s"]
        res[mode] = r
        log(f"{mode}: {r}")
        batch.close()
        plan.close()
    infer.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--blocks", type=int, default=1600000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--pos-weight", type=float, default=4.0)
    ap.add_argument("--first-seed", type=int, default=1000)
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None)
    ap.add_argument("--eval", default="384:110,512:100,512:110",
                    help="warm-start settings to evaluate, K:restricted_iters,...")
    args = ap.parse_args()
    import torch
    dev = torch.device("cuda:0")
    log = lambda m: print(m, flush=True)
    x, bits = build_dataset(args.first_seed, args.blocks, dev, log)
    net, hist = train(x, bits, args.epochs, args.batch, args.lr, args.pos_weight, log=log)
    if args.out:
        net.save(args.out)
        log(f"saved {args.out}")
    del x, bits
    configs = tuple(tuple(int(v) for v in c.split(":")) for c in args.eval.split(","))
    res = evaluate(net, configs=configs, log=log)
    res.update(blocks=args.blocks, epochs=args.epochs, batch=args.batch, lr=args.lr, pos_weight=args.pos_weight,
               loss_history=hist)
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(res, fh, indent=1)
    log(json.dumps({k: v for k, v in res.items() if k != "loss_history"}))


if __name__ == "__main__":
    main()
