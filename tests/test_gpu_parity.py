"""GPU parity: libfse (FP32, HIP) against the FP64 oracle, through the C ABI.

Each test prints the case it runs before touching the GPU.
"""
import numpy as np
import pytest

from synth import losses, workloads
from tests import parity

pytestmark = pytest.mark.gpu


def _run(wl, trace=True, rho=None, gamma=None, masked=False):
    import torch
    import paper_2204_14193_amd as fse
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    out, status, tr = fse.extrapolate_batch(img, av, wl.blocks, wl.rho if rho is None else rho,
                                            wl.gamma if gamma is None else gamma, trace=trace, masked=masked)
    return out.cpu().numpy(), status, tr


def _say(msg):
    print(msg, flush=True)


def test_isolated_256_full_parity():
    """64 isolated 16x16 losses in a 256x256 frame, F=64, I=100: every block
    replayed against the oracle; frame PSNR within 0.01 dB."""
    wl = workloads.isolated_256()
    _say(f"case isolated-256: {len(wl.blocks)} blocks F=64 I=100")
    out, st, tr = _run(wl)
    assert (st == 0).all()
    rows = parity.check_blocks(wl.frames, wl.avail, wl.blocks, wl.rho, wl.gamma, tr, out)
    d, pg, po, pb = parity.psnr_delta(wl.frames, wl.avail, wl.blocks, wl.rho, wl.gamma, out)
    _say(f"ties={sum(r['ties'] for r in rows)} coef_max={max(r['coef_max'] for r in rows):.2e} "
         f"pix={max(r['pix_maxabs'] for r in rows):.2e} psnr gpu={pg:.4f} oracle={po:.4f} between={pb:.1f}")
    assert d <= parity.PSNR_TOL
    # pixels outside every B are untouched
    lost = wl.avail == 0
    assert np.array_equal(out[~lost], wl.distorted[~lost].astype(np.float32))


def test_random_1080p_8x8_subset_parity():
    """1080p, 3240 non-adjacent 8x8 losses (40x40 areas), F=64, I=200: the
    whole frame runs in one launch; a seeded sample of 96 blocks is replayed."""
    wl = workloads.random_1080p_8x8()
    _say(f"case random-1080p-8x8: {len(wl.blocks)} blocks F=64 I=200")
    out, st, tr = _run(wl)
    assert (st == 0).all()
    idx = np.random.default_rng(7).choice(len(wl.blocks), 96, replace=False)
    parity.check_blocks(wl.frames, wl.avail, wl.blocks, wl.rho, wl.gamma, tr, out, idx)
    sub = wl.blocks[np.sort(idx)]
    d, pg, po, _ = parity.psnr_delta(wl.frames, wl.avail, sub, wl.rho, wl.gamma, out)
    _say(f"sample psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL


def test_random_1080p_16x16_sampled_parity_8_frames():
    """Eight 1080p frames, 804 16x16 losses each (6432 blocks, F=64, I=100),
    in the launch configuration of the benchmark; 48 sampled blocks replayed,
    all blocks checked for status and finite, bounded output."""
    wl = workloads.random_1080p_16x16(seeds=tuple(range(99, 107)))
    _say(f"case random-1080p-16x16 x8: {len(wl.blocks)} blocks F=64 I=100")
    out, st, tr = _run(wl, trace=True)
    assert (st == 0).all()
    lost = wl.avail == 0
    assert np.isfinite(out[lost]).all() and np.abs(out[lost]).max() < 1e4
    idx = np.random.default_rng(11).choice(len(wl.blocks), 48, replace=False)
    rows = parity.check_blocks(wl.frames, wl.avail, wl.blocks, wl.rho, wl.gamma, tr, out, idx)
    sub = wl.blocks[np.sort(idx)]
    d, pg, po, _ = parity.psnr_delta(wl.frames, wl.avail, sub, wl.rho, wl.gamma, out, processes=8)
    _say(f"sample pix={max(r['pix_maxabs'] for r in rows):.2e} psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL


def _ragged_workload():
    """Small frames with ragged geometry: non-square blocks, odd sizes, areas
    crossing every frame edge, all three transform sizes, I in {0, 1, 2, 37}."""
    frames = np.stack([__import__("synth").synthetic_image(96, 130, 31),
                       __import__("synth").synthetic_image(96, 130, 32)])
    B = losses.Block
    blocks = [
        B(0, 0, 0, 5, 11, 7, 32, 37),        # top-left corner, 19x25 area
        B(0, 90, 120, 6, 10, 9, 32, 2),      # bottom-right corner
        B(0, 40, 60, 16, 16, 16, 64, 37),    # interior, paper geometry
        B(1, 3, 100, 13, 7, 16, 64, 1),      # top edge, 45x39 area
        B(1, 50, 0, 32, 30, 16, 128, 37),    # left edge, 64x62 area in F=128
        B(1, 60, 70, 9, 9, 0, 32, 37),       # no border: empty support
        B(0, 20, 30, 4, 4, 8, 32, 0),        # zero iterations
    ]
    arr = losses.blocks_to_array(blocks)
    avail = losses.availability_mask(frames.shape, blocks)
    return workloads.Workload("ragged", frames, avail, arr, 0.8, 0.5)


def test_ragged_edges_and_degenerate_blocks():
    wl = _ragged_workload()
    _say(f"case ragged: {len(wl.blocks)} blocks F=32/64/128")
    out, st, tr = _run(wl)
    assert st.tolist() == [0, 0, 0, 0, 0, 1, 0]
    # empty support: B untouched (stays the distorted value 0)
    b = wl.blocks[5]
    assert (out[1, 60:69, 70:79] == 0).all()
    # zero iterations: model is zero on B
    assert (out[0, 20:24, 30:34] == 0).all()
    idx = [0, 1, 2, 3, 4]
    rows = parity.check_blocks(wl.frames, wl.avail, wl.blocks, wl.rho, wl.gamma, tr, out, idx)
    for r in rows:
        _say(f"  block {r['index']} F={wl.blocks['fft'][r['index']]}: coef_max={r['coef_max']:.2e} "
             f"pix_maxabs={r['pix_maxabs']:.2e}")
    # frame PSNR per transform size (F = 32: blocks 0, 1; 64: 2, 3; 128: 4)
    for sel in ([0, 1], [2, 3], [4]):
        d, pg, po, _ = parity.psnr_delta(wl.frames, wl.avail, wl.blocks[sel], wl.rho, wl.gamma, out)
        _say(f"  blocks {sel}: psnr gpu={pg:.4f} oracle={po:.4f}")
        assert d <= parity.PSNR_TOL, sel


def test_gamma_zero_gives_zero_model():
    wl = workloads.subset(workloads.isolated_256(iters=20), np.arange(8))
    _say("case gamma=0")
    out, st, _ = _run(wl, trace=False, gamma=0.0)
    assert (st == 0).all()
    for b in wl.blocks:
        assert (out[0, b["y0"]:b["y0"] + 16, b["x0"]:b["x0"] + 16] == 0).all()


def test_batch_invariance_and_determinism():
    """A block's output and selections do not depend on its batch companions
    or on the run: alone, in a batch, and twice in a row give identical bits."""
    wl = workloads.isolated_256(iters=60)
    _say("case batch invariance")
    out_all, _, tr_all = _run(wl)
    out_again, _, tr_again = _run(wl)
    assert np.array_equal(out_all, out_again) and np.array_equal(tr_all, tr_again)
    for i in (0, 17, 63):
        sub = workloads.subset(wl, [i])
        out1, _, tr1 = _run(sub)
        b = wl.blocks[i]
        sl = (0, slice(b["y0"], b["y0"] + 16), slice(b["x0"], b["x0"] + 16))
        assert np.array_equal(out1[sl], out_all[sl])
        assert np.array_equal(tr1[0], tr_all[i])


def _run_batch(wl, variants=None, trace=True):
    """Run through the Batch API with optional forced variants {F: threads}."""
    import torch
    import paper_2204_14193_amd as fse
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, int(wl.blocks["iters"].max()))
    batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    for F, nt in (variants or {}).items():
        batch.set_variant(F, nt)
    out = (img * (av != 0)).to(torch.float32)
    status = torch.full((len(wl.blocks),), -1, dtype=torch.int32, device=dev)
    tb = torch.zeros((len(wl.blocks), batch.max_iters * 16), dtype=torch.uint8, device=dev) if trace else None
    batch.run(img, av, out, status, tb)
    torch.cuda.synchronize()
    res = (out.cpu().numpy(), status.cpu().numpy(), None if tb is None else tb.cpu().numpy())
    batch.close()
    plan.close()
    return res


@pytest.mark.parametrize("F,shapes", [(64, [256, 128, 512]), (32, [64, 128, 256]), (128, [1024, 512])])
def test_every_variant_is_bit_identical(F, shapes):
    """Each compiled workgroup shape computes identical bits (same per-bin
    arithmetic, exact argmax), so the autotuner may pick any of them."""
    wl = _ragged_workload() if F != 64 else workloads.isolated_256(iters=50)
    _say(f"case variants F={F}: {shapes}")
    ref = _run_batch(wl, {F: shapes[0]})
    for shp in shapes[1:]:
        got = _run_batch(wl, {F: shp})
        assert np.array_equal(got[1], ref[1]), shp
        assert np.array_equal(got[0], ref[0]), shp
        assert np.array_equal(got[2], ref[2]), shp


def test_autotune_picks_a_variant_and_keeps_results():
    import torch
    import paper_2204_14193_amd as fse
    wl = workloads.isolated_256(iters=50)
    _say("case autotune")
    ref = _run_batch(wl)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, 50)
    batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    out = (img * (av != 0)).to(torch.float32)
    status = torch.zeros(len(wl.blocks), dtype=torch.int32, device=dev)
    rows = batch.autotune(img, av, out, status, reps=2)
    assert {r[0] for r in rows} == {64} and len(rows) >= 2
    best = min(rows, key=lambda r: r[2])
    info = batch.launch_info(64)
    assert info["threads"] == best[1]
    out.copy_((img * (av != 0)).to(torch.float32))
    batch.run(img, av, out, status)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref[0])


def test_autotune_cache(tmp_path):
    """The tuner's decision cache: a first call times every shape of each
    class and appends one line per class; a second batch of the same shape
    takes the decisions from the file without timing and keeps results
    bit-identical; a cached shape that is not compiled is ignored (timed
    again)."""
    import torch
    import paper_2204_14193_amd as fse
    wl = _ragged_workload()
    _say("case autotune cache")
    ref = _run_batch(wl)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    cache = tmp_path / "tune.txt"
    classes = sorted({int(f) for f in wl.blocks["fft"]})

    def tuned():
        plan = fse.Plan(wl.rho, wl.gamma, int(wl.blocks["iters"].max()))
        batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
        out = (img * (av != 0)).to(torch.float32)
        status = torch.zeros(len(wl.blocks), dtype=torch.int32, device=dev)
        rows = batch.autotune(img, av, out, status, reps=1, cache=str(cache))
        chosen = {F: batch.launch_info(F)["threads"] for F in classes}
        out.copy_((img * (av != 0)).to(torch.float32))
        batch.run(img, av, out, status)
        torch.cuda.synchronize()
        res = out.cpu().numpy()
        batch.close()
        plan.close()
        return rows, chosen, res

    rows1, chosen1, out1 = tuned()
    assert all(r[2] is not None for r in rows1) and {r[0] for r in rows1} == set(classes)
    lines = cache.read_text().splitlines()
    assert len(lines) == len(classes)
    assert all(line.split()[0].split("/")[2] in {f"F{F}" for F in classes} for line in lines), lines
    rows2, chosen2, out2 = tuned()
    assert sorted(rows2) == [(F, chosen1[F], None) for F in classes], rows2
    assert chosen2 == chosen1
    assert np.array_equal(out1, ref[0]) and np.array_equal(out2, ref[0])
    assert len(cache.read_text().splitlines()) == len(classes)  # nothing timed, nothing appended
    # a decision naming a shape that is not compiled: that class is timed again
    key = lines[0].split()[0]
    with open(cache, "a") as fh:
        fh.write(f"{key} 96 1.0\n")
    rows3, chosen3, _ = tuned()
    F0 = int(key.split("/")[2][1:])
    assert any(r[0] == F0 and r[2] is not None for r in rows3), rows3
    assert all(r[2] is None for r in rows3 if r[0] != F0), rows3


def _mixed_4k(n_frames=2):
    return workloads.mixed_4k(seeds=tuple(range(2, 2 + n_frames)))


def test_mixed_4k_uneven_batch_parity():
    """Two 3840x2160 frames with 305 losses each of 4, 8, 16 and 32 pixels
    (borders 8..16, F in {32, 64, 128}, I in {50, 100, 200, 500}) in one
    call; a stratified seeded sample (3 blocks per loss size and transform
    size) replayed against the oracle, with per-stratum FP32 error printed."""
    wl = _mixed_4k()
    _say(f"case mixed-4k x2: {len(wl.blocks)} blocks, F classes {sorted(set(wl.blocks['fft'].tolist()))}")
    out, st, tr = _run(wl)
    assert (st == 0).all()
    lost = wl.avail == 0
    assert np.isfinite(out[lost]).all()
    rng = np.random.default_rng(3)
    idx = []
    for bs in (4, 8, 16, 32):
        for F in (32, 64, 128):
            cand = np.flatnonzero((wl.blocks["bh"] == bs) & (wl.blocks["fft"] == F))
            if len(cand):
                # prefer short runs for the oracle's sake, but include one long one
                cand = cand[np.argsort(wl.blocks["iters"][cand], kind="stable")]
                pick = list(rng.choice(cand[:max(3, len(cand) // 2)], min(2, len(cand)), replace=False))
                pick.append(cand[-1])
                idx += [int(i) for i in pick]
    rows = parity.check_blocks(wl.frames, wl.avail, wl.blocks, wl.rho, wl.gamma, tr, out, idx)
    for r in rows:
        b = wl.blocks[r["index"]]
        _say(f"  size {b['bh']:2d} F={b['fft']:3d} I={b['iters']:3d}: coef_max={r['coef_max']:.2e} "
             f"coef_l2={r['coef_l2']:.2e} pix_maxabs={r['pix_maxabs']:.2e} ties={r['ties']}")
    # PSNR of the sample per transform size against the free-running oracle
    idx = np.array(sorted(idx))
    for F in (32, 64, 128):
        sel = idx[wl.blocks["fft"][idx] == F]
        d, pg, po, _ = parity.psnr_delta(wl.frames, wl.avail, wl.blocks[sel], wl.rho, wl.gamma, out, processes=8)
        _say(f"  F={F}: {len(sel)} blocks, psnr gpu={pg:.4f} oracle={po:.4f}")
        assert d <= parity.PSNR_TOL, F


def test_graph_capture_replays_match_eager():
    """The launch is capture-safe: replaying a captured call several times,
    with eager work in between, reproduces the eager result bit for bit."""
    import torch
    import paper_2204_14193_amd as fse
    wl = _mixed_4k(1)
    _say(f"case graph capture: {len(wl.blocks)} blocks")
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, 500)
    batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    base = (img * (av != 0)).to(torch.float32)
    out = base.clone()
    status = torch.zeros(len(wl.blocks), dtype=torch.int32, device=dev)
    batch.run(img, av, out, status)
    torch.cuda.synchronize()
    eager = out.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    out.copy_(base)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        batch.run(img, av, out, status, stream=s)
    for rep in range(3):
        out.copy_(base)
        status.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert (status == 0).all(), rep
        assert torch.equal(out, eager), rep
        _ = (img.float() * 2).sum().item()          # unrelated eager work between replays
    del g
    batch.close()
    plan.close()


def test_masked_loss_areas_parity():
    """Arbitrary loss shapes: scribble losses in a 256x256 frame covered by
    16x16 tiles (border 16, F=64, I=60), each block concealing only its
    tile's lost pixels. Every block replayed against the oracle's
    mask-driven loss area; frame PSNR within 0.01 dB; received pixels,
    including those inside the tiles, untouched."""
    wl = workloads.strokes_256()
    part = sum(1 for b in wl.blocks
               if (wl.avail[0, b["y0"]:b["y0"] + b["bh"], b["x0"]:b["x0"] + b["bw"]] != 0).any())
    _say(f"case strokes-256 masked: {len(wl.blocks)} blocks ({part} partly received) F=64 I=60")
    assert part > len(wl.blocks) // 2
    out, st, tr = _run(wl, masked=True)
    assert (st == 0).all()
    rows = parity.check_blocks(wl.frames, wl.avail, wl.blocks, wl.rho, wl.gamma, tr, out, masked=True)
    d, pg, po, pb = parity.psnr_delta(wl.frames, wl.avail, wl.blocks, wl.rho, wl.gamma, out, masked=True)
    _say(f"ties={sum(r['ties'] for r in rows)} coef_max={max(r['coef_max'] for r in rows):.2e} "
         f"pix={max(r['pix_maxabs'] for r in rows):.2e} psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL
    assert max(r["pix_maxabs"] for r in rows) < 0.05
    recv = wl.avail != 0
    assert np.array_equal(out[recv], wl.distorted[recv].astype(np.float32))


def test_masked_plan_on_rectangular_losses_is_bitwise_plain():
    """When every pixel of each rectangle is lost, the mask-driven plan is
    the rectangular one: same selections, coefficients and output bits."""
    wl = workloads.isolated_256(iters=40)
    _say("case isolated-256 masked vs rectangular")
    o1, s1, t1 = _run(wl)
    o2, s2, t2 = _run(wl, masked=True)
    assert (s1 == 0).all() and np.array_equal(s1, s2)
    assert np.array_equal(o1, o2) and np.array_equal(t1, t2)


def test_warm_start_refuses_masked_plans():
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    wl = workloads.subset(workloads.isolated_256(iters=0), [0, 1])
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, 4096, masked=True)
    batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    out = img.to(torch.float32)
    st = torch.zeros(2, dtype=torch.int32, device=dev)
    cand = torch.zeros((2, 256), dtype=torch.int16, device=dev)
    flags = torch.zeros(2, dtype=torch.int32, device=dev)
    with pytest.raises(fse.FseError) as e:
        warm.warm_extrapolate(batch, img, av, out, st, cand, flags, 256, 10, 10)
    assert e.value.code == -2
