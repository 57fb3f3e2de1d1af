"""GPU parity of fixed-point cFSE (plan flag FSE_PLAN_FIXED) against the
integer oracle (oracle.fixed): integer work, so the bar is bit-exact —
every selection, every coefficient and every output value.

Each test prints the case it runs before touching the GPU.
"""
import numpy as np
import pytest

from oracle import fixed, metrics
from synth import losses, workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _f32(x):
    """The plan holds rho and gamma in FP32; the oracle takes the same values."""
    return float(np.float32(x))


def _run(distorted, avail, blocks, rho, gamma, trace=True, fixed_point=True):
    import torch
    import paper_2204_14193_amd as fse
    dev = torch.device("cuda:0")
    img = torch.from_numpy(distorted).to(dev)
    av = torch.from_numpy(avail).to(dev)
    out, st, tr = fse.extrapolate_batch(img, av, blocks, rho, gamma, trace=trace, fixed=fixed_point)
    return out.cpu().numpy(), st, tr


def _exact(distorted, avail, blocks, rho, gamma, out, tr, idx):
    """Every selection, coefficient and B pixel equal to the oracle's."""
    for i in idx:
        b = blocks[i]
        ref = fixed.extrapolate_block(distorted, avail, b, _f32(rho), _f32(gamma))
        I = int(b["iters"])
        rec = tr[i][:I]
        seq = (rec["u"].astype(np.int64) * 64 + rec["v"]).tolist()
        assert seq == ref["seq"], (i, next(j for j in range(I) if seq[j] != ref["seq"][j]))
        c = np.stack([rec["c_re"].astype(np.float64) * 65536, rec["c_im"].astype(np.float64) * 65536], 1)
        assert np.array_equal(c, np.array(ref["c"], dtype=np.float64).reshape(-1, 2)), i
        f, y0, x0 = int(b["frame"]), int(b["y0"]), int(b["x0"])
        g = out[f, y0:y0 + int(b["bh"]), x0:x0 + int(b["bw"])]
        assert np.array_equal(g, ref["values"].astype(np.float32)), i


def test_fixed_isolated_256_bit_exact():
    """64 isolated 16x16 losses in a 256x256 frame, F = 64, I = 100: every
    block bit-exact against the integer oracle."""
    wl = workloads.isolated_256()
    _say(f"case fixed isolated-256: {len(wl.blocks)} blocks F=64 I=100")
    out, st, tr = _run(wl.distorted, wl.avail, wl.blocks, wl.rho, wl.gamma)
    assert (st == 0).all(), st
    _exact(wl.distorted, wl.avail, wl.blocks, wl.rho, wl.gamma, out, tr, range(len(wl.blocks)))
    lost = wl.avail == 0
    assert np.array_equal(out[~lost], wl.distorted[~lost].astype(np.float32))


def test_fixed_1080p_sampled_bit_exact_and_quality():
    """One 1080p frame, 804 random 16x16 losses, I = 100: a seeded sample of
    48 blocks bit-exact; over all blocks the PSNR is within 0.05 dB of the
    FP32 GPU path (no error build-up without divisions in the loop)."""
    wl = workloads.random_1080p_16x16(seeds=(99,), iters=100)
    _say(f"case fixed random-1080p-16x16: {len(wl.blocks)} blocks F=64 I=100")
    out, st, tr = _run(wl.distorted, wl.avail, wl.blocks, wl.rho, wl.gamma)
    assert (st == 0).all()
    idx = np.sort(np.random.default_rng(11).choice(len(wl.blocks), 48, replace=False))
    _exact(wl.distorted, wl.avail, wl.blocks, wl.rho, wl.gamma, out, tr, idx)
    out_f, st_f, _ = _run(wl.distorted, wl.avail, wl.blocks, wl.rho, wl.gamma, trace=False, fixed_point=False)
    p_fixed = metrics.psnr_lost(wl.frames, out, wl.avail)
    p_float = metrics.psnr_lost(wl.frames, out_f, wl.avail)
    _say(f"psnr fixed={p_fixed:.4f} float={p_float:.4f}")
    assert abs(p_fixed - p_float) <= 0.05


def test_fixed_edge_cases():
    """No support (EMPTY_SUPPORT, B untouched), I = 0 (B = 0), a constant
    area (DC every iteration, exact), a corner block, and F = 32 refused."""
    import paper_2204_14193_amd as fse
    H = W = 128
    frame = np.full((1, H, W), 77, dtype=np.uint8)
    frame[0, :, 64:] = (np.arange(64)[None, :] * 3 % 251).astype(np.uint8)
    blist = [losses.Block(0, 16, 16, 16, 16, 16, 64, 10), losses.Block(0, 16, 80, 16, 16, 16, 64, 0),
             losses.Block(0, 80, 16, 16, 16, 16, 64, 6), losses.Block(0, 0, 112, 16, 16, 16, 64, 12)]
    blocks = losses.blocks_to_array(blist)
    av = losses.availability_mask(frame.shape, blist)
    av[0, 0:48, 0:48] = 0
    dist = (frame * av).astype(np.uint8)
    _say("case fixed edges: empty support, iters=0, constant area, corner")
    out, st, tr = _run(dist, av, blocks, 0.8, 0.5)
    assert st.tolist() == [fse.BLOCK_EMPTY_SUPPORT, 0, 0, 0], st
    assert np.array_equal(out[0, 16:32, 16:32], np.zeros((16, 16), np.float32))
    assert np.array_equal(out[0, 16:32, 80:96], np.zeros((16, 16), np.float32))
    assert (tr[2][:6]["u"] == 0).all() and (tr[2][:6]["v"] == 0).all()
    _exact(dist, av, blocks, 0.8, 0.5, out, tr, [2, 3])
    bad = blocks.copy()
    bad[1]["fft"] = 32
    bad[1]["border"] = 8
    with pytest.raises(fse.FseError):
        _run(dist, av, bad, 0.8, 0.5)


def test_fixed_mixed_block_sizes_bit_exact():
    """8x8 (border 16), 32x32 (border 16: a 64x64 area, the encoding's
    largest) and 16x16 (border 8) blocks in one launch, bit-exact."""
    frames = workloads.synthetic_image(192, 192, 77)[None]
    blist = [losses.Block(0, 24, 24, 8, 8, 16, 64, 40), losses.Block(0, 96, 16, 32, 32, 16, 64, 40),
             losses.Block(0, 40, 120, 16, 16, 8, 64, 40)]
    blocks = losses.blocks_to_array(blist)
    av = losses.availability_mask(frames.shape, blist)
    dist = (frames * av).astype(np.uint8)
    _say("case fixed mixed sizes: 8x8/b16, 32x32/b16, 16x16/b8")
    out, st, tr = _run(dist, av, blocks, 0.8, 0.5)
    assert (st == 0).all(), st
    _exact(dist, av, blocks, 0.8, 0.5, out, tr, range(3))
