"""GPU parity of real-valued FSE (plan flag FSE_PLAN_REAL) against the FP64
rFSE oracle (oracle.rfse), through the C ABI: selections (near ties within
1e-6), accumulated coefficients (1e-4), PSNR over the lost pixels (0.01 dB).

Each test prints the case it runs before touching the GPU.
"""
import numpy as np
import pytest

from oracle import metrics, rfse
from synth import losses, workloads
from tests import parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _run(distorted, avail, blocks, rho, gamma, trace=True, real=True):
    import torch
    import paper_2204_14193_amd as fse
    dev = torch.device("cuda:0")
    img = torch.from_numpy(distorted).to(dev)
    av = torch.from_numpy(avail).to(dev)
    out, st, tr = fse.extrapolate_batch(img, av, blocks, rho, gamma, trace=trace, real=real)
    return out.cpu().numpy(), st, tr


def _check(frames, avail, blocks, rho, gamma, out, tr, idx, selection="decrease"):
    rows = []
    for i in idx:
        b = blocks[i]
        r = parity.replay_real_block(frames * avail, avail, b, rho, gamma, tr[i], selection)
        f, y0, x0 = int(b["frame"]), int(b["y0"]), int(b["x0"])
        g = out[f, y0:y0 + int(b["bh"]), x0:x0 + int(b["bw"])].astype(np.float64)
        r["pix_maxabs"] = float(np.abs(g - r["values"]).max())
        rows.append(r)
        assert r["gap_violations"] == 0, (i, r)
        assert r["coef_max"] <= parity.COEF_TOL and r["coef_l2"] <= parity.COEF_TOL, (i, r)
        assert r["pix_maxabs"] < parity.PIX_TOL, (i, r["pix_maxabs"])
    return rows


def _psnr(frames, avail, blocks, rho, gamma, out, idx, selection="decrease"):
    ref = (frames * avail).astype(np.float64)
    mask = np.ones_like(avail)
    for i in idx:
        b = blocks[i]
        f, y0, x0 = int(b["frame"]), int(b["y0"]), int(b["x0"])
        sl = (f, slice(y0, y0 + int(b["bh"])), slice(x0, x0 + int(b["bw"])))
        ref[sl] = rfse.extrapolate_block(frames * avail, avail, b, rho, gamma, selection=selection)["values"]
        mask[sl] = 0
    pg, po = metrics.psnr_lost(frames, out, mask), metrics.psnr_lost(frames, ref, mask)
    return abs(pg - po), pg, po


def test_rfse_isolated_256_full_parity():
    """64 isolated 16x16 losses in a 256x256 frame, F = 64, 50 rFSE
    iterations (100 basis functions): every block replayed; PSNR within
    0.01 dB; pixels outside every B untouched."""
    wl = workloads.isolated_256()
    blocks = wl.blocks.copy()
    blocks["iters"] = 50
    _say(f"case rfse isolated-256: {len(blocks)} blocks F=64 I=50")
    out, st, tr = _run(wl.distorted, wl.avail, blocks, wl.rho, wl.gamma)
    assert (st == 0).all(), st
    idx = range(len(blocks))
    rows = _check(wl.frames, wl.avail, blocks, wl.rho, wl.gamma, out, tr, idx)
    d, pg, po = _psnr(wl.frames, wl.avail, blocks, wl.rho, wl.gamma, out, idx)
    _say(f"ties={sum(r['ties'] for r in rows)} coef_max={max(r['coef_max'] for r in rows):.2e} "
         f"pix={max(r['pix_maxabs'] for r in rows):.2e} psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL
    lost = wl.avail == 0
    assert np.array_equal(out[~lost], wl.distorted[~lost].astype(np.float32))


def test_rfse_inloop_variant_parity():
    """The form that recomputes the pair constants in every iteration
    (FSE_PLAN_REAL_INLOOP) meets the same bars on the 256x256 case."""
    wl = workloads.isolated_256()
    blocks = wl.blocks.copy()
    blocks["iters"] = 50
    _say(f"case rfse-inloop isolated-256: {len(blocks)} blocks F=64 I=50")
    out, st, tr = _run(wl.distorted, wl.avail, blocks, wl.rho, wl.gamma, real="inloop")
    assert (st == 0).all(), st
    idx = range(len(blocks))
    rows = _check(wl.frames, wl.avail, blocks, wl.rho, wl.gamma, out, tr, idx)
    d, pg, po = _psnr(wl.frames, wl.avail, blocks, wl.rho, wl.gamma, out, idx)
    _say(f"ties={sum(r['ties'] for r in rows)} coef_max={max(r['coef_max'] for r in rows):.2e} "
         f"psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL


@pytest.mark.parametrize("gamma", [0.2, 0.5])
def test_rfse_power_selection_parity(gamma):
    """The other selection reading (FSE_PLAN_REAL_POWER: the pair holding
    the largest |R_w|^2) against the oracle with that reading: every block
    of the 256x256 case, 50 iterations."""
    wl = workloads.isolated_256()
    blocks = wl.blocks.copy()
    blocks["iters"] = 50
    _say(f"case rfse-power isolated-256: {len(blocks)} blocks F=64 I=50 gamma={gamma}")
    out, st, tr = _run(wl.distorted, wl.avail, blocks, wl.rho, gamma, real="power")
    assert (st == 0).all(), st
    idx = range(len(blocks))
    rows = _check(wl.frames, wl.avail, blocks, wl.rho, gamma, out, tr, idx, "power")
    d, pg, po = _psnr(wl.frames, wl.avail, blocks, wl.rho, gamma, out, idx, "power")
    _say(f"ties={sum(r['ties'] for r in rows)} coef_max={max(r['coef_max'] for r in rows):.2e} "
         f"psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL


def test_rfse_1080p_sampled_parity():
    """One 1080p frame, 804 random 16x16 losses, 50 rFSE iterations, gamma
    0.2 (the paper's comparison setting): a seeded sample of 32 blocks
    replayed, PSNR of the sample within 0.01 dB."""
    wl = workloads.random_1080p_16x16(seeds=(99,), iters=50)
    _say(f"case rfse random-1080p-16x16: {len(wl.blocks)} blocks F=64 I=50 gamma=0.2")
    out, st, tr = _run(wl.distorted, wl.avail, wl.blocks, wl.rho, 0.2)
    assert (st == 0).all()
    idx = np.sort(np.random.default_rng(3).choice(len(wl.blocks), 32, replace=False))
    rows = _check(wl.frames, wl.avail, wl.blocks, wl.rho, 0.2, out, tr, idx)
    d, pg, po = _psnr(wl.frames, wl.avail, wl.blocks, wl.rho, 0.2, out, idx)
    _say(f"ties={sum(r['ties'] for r in rows)} coef_max={max(r['coef_max'] for r in rows):.2e} "
         f"psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL


def test_rfse_edge_cases():
    """No support (status EMPTY_SUPPORT, B untouched), iters = 0 (B = 0), a
    constant area (the DC pair, a self-conjugate bin, reproduces it) and a
    block at the frame corner; F = 32 blocks are refused."""
    import paper_2204_14193_amd as fse
    H = W = 128
    frame = np.full((1, H, W), 77, dtype=np.uint8)
    frame[0, :, 64:] = (np.arange(64)[None, :] * 3 % 251).astype(np.uint8)
    blist = [losses.Block(0, 16, 16, 16, 16, 16, 64, 10), losses.Block(0, 16, 80, 16, 16, 16, 64, 0),
             losses.Block(0, 80, 16, 16, 16, 16, 64, 6), losses.Block(0, 0, 112, 16, 16, 16, 64, 12)]
    blocks = losses.blocks_to_array(blist)
    av = losses.availability_mask(frame.shape, blist)
    av[0, 0:48, 0:48] = 0                        # the first block's whole area
    dist = (frame * av).astype(np.uint8)
    _say("case rfse edges: empty support, iters=0, constant area, corner")
    out, st, tr = _run(dist, av, blocks, 0.8, 0.5)
    assert st.tolist() == [fse.BLOCK_EMPTY_SUPPORT, 0, 0, 0], st
    assert np.array_equal(out[0, 16:32, 16:32], np.zeros((16, 16), np.float32))
    assert np.array_equal(out[0, 16:32, 80:96], np.zeros((16, 16), np.float32))
    # constant 77 around the third block: gamma 0.5 per iteration on the DC pair
    np.testing.assert_allclose(out[0, 80:96, 16:32], 77.0 * (1 - 0.5 ** 6), rtol=1e-5)
    _check(frame, av, blocks, 0.8, 0.5, out, tr, [2, 3])
    bad = blocks.copy()
    bad["fft"] = 64
    bad[1]["fft"] = 32
    bad[1]["border"] = 8
    with pytest.raises(fse.FseError):
        _run(dist, av, bad, 0.8, 0.5)


def test_rfse_mixed_block_sizes():
    """8x8 (border 16), 32x32 (border 16: a 64x64 area, the largest) and
    16x16 (border 8) blocks in one launch, every block replayed."""
    frames = workloads.synthetic_image(192, 192, 77)[None]
    blist = [losses.Block(0, 24, 24, 8, 8, 16, 64, 30), losses.Block(0, 96, 16, 32, 32, 16, 64, 30),
             losses.Block(0, 40, 120, 16, 16, 8, 64, 30)]
    blocks = losses.blocks_to_array(blist)
    av = losses.availability_mask(frames.shape, blist)
    dist = (frames * av).astype(np.uint8)
    _say("case rfse mixed sizes: 8x8/b16, 32x32/b16, 16x16/b8")
    out, st, tr = _run(dist, av, blocks, 0.8, 0.5)
    assert (st == 0).all(), st
    _check(frames, av, blocks, 0.8, 0.5, out, tr, range(3))
