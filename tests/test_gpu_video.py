"""GPU parity of 3-D (video) cFSE: libfse's 64x64x8 kernel against the FP64
oracle (oracle.cfse3), through the C ABI, with the same replay bars as the
2-D path (selections, accumulated coefficients, PSNR over the lost voxels).

Each test prints the case it runs before touching the GPU.
"""
import numpy as np
import pytest

from oracle import cfse3, metrics
from synth import losses, workloads
from tests import parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _run(frames_distorted, avail, vols, rho, gamma, trace=True):
    import torch
    import paper_2204_14193_amd as fse
    dev = torch.device("cuda:0")
    img = torch.from_numpy(frames_distorted).to(dev)
    av = torch.from_numpy(avail).to(dev)
    out, st, tr = fse.extrapolate3d(img, av, vols, rho, gamma, trace=trace)
    return out.cpu().numpy(), st, tr


def _check(wl, out, tr, idx):
    rows = []
    dist = wl.distorted
    for i in idx:
        v = wl.blocks[i]
        r = parity.replay_volume(dist, wl.avail, v, wl.rho, wl.gamma, tr[i])
        g = out[parity.volume_slices(v)].astype(np.float64)      # [t][y][x]
        r["pix_maxabs"] = float(np.abs(g - r["values"].transpose(2, 0, 1)).max())
        rows.append(r)
        assert r["gap_violations"] == 0, (i, r)
        assert r["coef_max"] <= parity.COEF_TOL and r["coef_l2"] <= parity.COEF_TOL, (i, r)
    return rows


def _psnr(wl, out, idx):
    """|PSNR(GPU) - PSNR(free-running oracle)| over the lost voxels of the
    volumes in idx."""
    ref = wl.distorted.astype(np.float64)
    mask = np.ones_like(wl.avail)
    for i in idx:
        v = wl.blocks[i]
        res = cfse3.extrapolate_volume(wl.distorted, wl.avail, v, wl.rho, wl.gamma)
        sl = parity.volume_slices(v)
        ref[sl] = res["values"].transpose(2, 0, 1)
        mask[sl] = 0
    pg = metrics.psnr_lost(wl.frames, out, mask)
    po = metrics.psnr_lost(wl.frames, ref, mask)
    return abs(pg - po), pg, po


def test_clip_256_full_parity():
    """51 lost 16x16x2 volumes in a 256x256x8 clip (48x48x6 areas, some cut
    by the clip's edges in space and time), 64x64x8 transform, I=40: every
    volume replayed; PSNR over the lost voxels within 0.01 dB; voxels outside
    every B untouched."""
    wl = workloads.clip_small()
    _say(f"case clip-256: {len(wl.blocks)} volumes 64x64x8 I=40")
    out, st, tr = _run(wl.distorted, wl.avail, wl.blocks, wl.rho, wl.gamma)
    assert (st == 0).all(), st
    idx = range(len(wl.blocks))
    rows = _check(wl, out, tr, idx)
    d, pg, po = _psnr(wl, out, idx)
    _say(f"ties={sum(r['ties'] for r in rows)} coef_max={max(r['coef_max'] for r in rows):.2e} "
         f"pix={max(r['pix_maxabs'] for r in rows):.2e} psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL
    lost = wl.avail == 0
    assert np.array_equal(out[~lost], wl.distorted[~lost].astype(np.float32))


def test_clip_1080p_sampled_parity():
    """The 1920x1080x16 clip with 16x16x2 volumes at 5% of the volume grid,
    I=200, in one launch: a seeded sample of 12 volumes replayed, PSNR of the
    sample within 0.01 dB."""
    wl = workloads.clip_1080p_16x16x2()
    _say(f"case clip-1080p: {len(wl.blocks)} volumes 64x64x8 I=200")
    out, st, tr = _run(wl.distorted, wl.avail, wl.blocks, wl.rho, wl.gamma)
    assert (st == 0).all()
    idx = np.sort(np.random.default_rng(5).choice(len(wl.blocks), 12, replace=False))
    rows = _check(wl, out, tr, idx)
    d, pg, po = _psnr(wl, out, idx)
    _say(f"ties={sum(r['ties'] for r in rows)} coef_max={max(r['coef_max'] for r in rows):.2e} "
         f"psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL


def test_clip_edge_cases():
    """Edge cases of the volume path: a volume with no support at all
    (status EMPTY_SUPPORT, B left as it was), one with iters = 0 (B set to
    0), a single-frame volume (bt = 1, tborder = 0) next to the first frame,
    and an empty volume list."""
    import torch
    import paper_2204_14193_amd as fse
    wl = workloads.clip_small()
    vols = np.zeros(4, dtype=losses.VOLUME_DTYPE)
    base = dict(bt=2, bh=16, bw=16, border=16, tborder=2, fft=64, fft_t=8, iters=12)
    for v, (f, y, x) in zip(vols, ((2, 96, 96), (4, 32, 160), (0, 176, 48), (6, 200, 200))):
        for k, val in base.items():
            v[k] = val
        v["frame"], v["y0"], v["x0"] = f, y, x
    vols[1]["iters"] = 0
    vols[2]["bt"], vols[2]["tborder"] = 1, 0
    av = losses.volume_availability(wl.frames.shape, vols)
    av[0:6, 80:128, 80:128] = 0                       # the first volume's whole area
    dist = (wl.frames * av).astype(np.uint8)
    _say("case clip-edges: empty support, iters=0, bt=1, empty list")
    out, st, tr = _run(dist, av, vols, 0.8, 0.5)
    assert st[0] == fse.BLOCK_EMPTY_SUPPORT and (st[1:] == 0).all(), st
    assert np.array_equal(out[parity.volume_slices(vols[0])], np.zeros((2, 16, 16), np.float32))
    assert np.array_equal(out[parity.volume_slices(vols[1])], np.zeros((2, 16, 16), np.float32))
    sub = workloads.Workload("edges", wl.frames, av, vols, 0.8, 0.5)
    _check(sub, out, tr, [2, 3])
    out2, st2, tr2 = _run(dist, av, np.zeros(0, dtype=losses.VOLUME_DTYPE), 0.8, 0.5)
    assert len(st2) == 0 and np.array_equal(out2, dist.astype(np.float32))


def test_clip_mixed_volume_sizes():
    """Volumes of other shapes in one launch: 8x8x1 (border 8, 1 frame),
    24x24x4 (border 12 and 2: a 48x48x8 area, 2304 voxels, more than one
    per thread), 16x16x2 with border 24 (a 64x64x6 area, the largest that
    fits), each replayed against the oracle."""
    wl = workloads.clip_small()
    vols = np.zeros(3, dtype=losses.VOLUME_DTYPE)
    spec = [(1, 8, 8, 8, 0, 3, 40), (4, 24, 24, 12, 2, 2, 100), (2, 16, 16, 24, 2, 4, 180)]
    for v, (bt, bh, bw, bd, td, f, pos) in zip(vols, spec):
        v["frame"], v["y0"], v["x0"] = f, pos, pos
        v["bt"], v["bh"], v["bw"], v["border"], v["tborder"] = bt, bh, bw, bd, td
        v["fft"], v["fft_t"], v["iters"] = 64, 8, 30
    av = losses.volume_availability(wl.frames.shape, vols)
    dist = (wl.frames * av).astype(np.uint8)
    _say("case clip-mixed: 8x8x1, 24x24x4, 16x16x2 border 24")
    out, st, tr = _run(dist, av, vols, 0.8, 0.5)
    assert (st == 0).all(), st
    sub = workloads.Workload("mixed", wl.frames, av, vols, 0.8, 0.5)
    rows = _check(sub, out, tr, range(3))
    _say(f"coef_max={max(r['coef_max'] for r in rows):.2e} pix={max(r['pix_maxabs'] for r in rows):.2e}")


def _run_warm(wl, iters=None, trace=True):
    """Warm-started 3-D: the 2-D network's top-128 columns per volume."""
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    dev = torch.device("cuda:0")
    vols = wl.blocks.copy()
    if iters is not None:
        vols["iters"] = iters
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, int(vols["iters"].max()))
    batch = fse.Batch3d(plan, vols, *wl.frames.shape)
    net = warm.Net(len(vols), seed=0)
    net.load()
    ws = warm.WarmStart3d(net, batch, vols, plan)
    out = (img * (av != 0)).to(torch.float32)
    status = torch.full((len(vols),), -1, dtype=torch.int32, device=dev)
    tbuf = torch.zeros((len(vols), batch.max_iters * 16), dtype=torch.uint8, device=dev) if trace else None
    ws.run(img, av, out, status, tbuf)
    torch.cuda.synchronize()
    tr = None if tbuf is None else tbuf.cpu().numpy().view(fse.TRACE_DTYPE).reshape(len(vols), batch.max_iters)
    res = out.cpu().numpy(), status.cpu().numpy(), tr, ws.cand.cpu().numpy(), ws.flags.cpu().numpy(), vols
    ws.close()
    net.close()
    batch.close()
    plan.close()
    return res


def test_clip_warm_start_parity():
    """Warm-started 3-D on the 256x256x8 clip (I = 40): every volume
    replayed against the oracle restricted to the same candidate columns
    (selections, coefficients); PSNR within 0.01 dB of the restricted
    oracle."""
    wl = workloads.clip_small()
    _say(f"case clip-256 warm: {len(wl.blocks)} volumes, 128 columns x 8")
    out, st, tr, cand, flags, vols = _run_warm(wl)
    assert (flags == 0).all() and (st == 0).all(), st
    assert all((np.diff(c.astype(np.int64)) > 0).all() for c in cand)
    ref = wl.distorted.astype(np.float64)
    mask = np.ones_like(wl.avail)
    rows = []
    for i, v in enumerate(vols):
        cmask = parity.volume_candidates(cand[i])
        r = parity.replay_volume(wl.distorted, wl.avail, v, wl.rho, wl.gamma, tr[i], cand=cmask)
        assert r["gap_violations"] == 0, (i, r)
        assert r["coef_max"] <= parity.COEF_TOL and r["coef_l2"] <= parity.COEF_TOL, (i, r)
        rows.append(r)
        free = cfse3.extrapolate_volume(wl.distorted, wl.avail, v, wl.rho, wl.gamma, cand=cmask)
        sl = parity.volume_slices(v)
        ref[sl] = free["values"].transpose(2, 0, 1)
        mask[sl] = 0
    pg, po = metrics.psnr_lost(wl.frames, out, mask), metrics.psnr_lost(wl.frames, ref, mask)
    _say(f"ties={sum(r['ties'] for r in rows)} coef_max={max(r['coef_max'] for r in rows):.2e} "
         f"psnr gpu={pg:.4f} oracle={po:.4f}")
    assert abs(pg - po) <= parity.PSNR_TOL


def test_clip_warm_start_quality_1080p():
    """On the 1080p clip (3216 volumes, I = 200) the warm start loses at
    most 0.1 dB against plain 3-D FSE over the lost voxels."""
    import torch
    import paper_2204_14193_amd as fse
    wl = workloads.clip_1080p_16x16x2()
    _say(f"case clip-1080p warm vs plain: {len(wl.blocks)} volumes")
    out_w, st_w, _, _, flags, _ = _run_warm(wl, trace=False)
    out_p, st_p, _ = _run(wl.distorted, wl.avail, wl.blocks, wl.rho, wl.gamma, trace=False)
    assert (flags == 0).all() and (st_w == 0).all() and (st_p == 0).all()
    pw, pp = metrics.psnr_lost(wl.frames, out_w, wl.avail), metrics.psnr_lost(wl.frames, out_p, wl.avail)
    _say(f"psnr warm={pw:.4f} plain={pp:.4f}")
    assert pw >= pp - 0.1
