"""GPU tests of the learned warm start: network kernels against the FP64
network oracle, candidate selection, and warm-started FSE against the FP64
FSE oracle (through the C ABI)."""
import numpy as np
import pytest

from oracle import cfse, cnn
from synth import losses, workloads
from tests import parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def bf16(x):
    """Round to BF16 (nearest even), returned as float32."""
    u = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32)


def _relfro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _cos(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))


def _setup(n_blocks=16, seed=0):
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    wl = workloads.subset(workloads.isolated_256(iters=30), np.arange(n_blocks))
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, 4096)
    batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    x = torch.empty((n_blocks, 48, 48, 2), dtype=torch.bfloat16, device=dev)
    warm.patches(batch, img, av, x)
    torch.cuda.synchronize()
    return wl, img, av, plan, batch, x


def test_patches_match_definition():
    wl, img, av, plan, batch, x = _setup()
    _say("case cnn patches")
    got = x.float().cpu().numpy()
    for i, blk in enumerate(wl.blocks):
        s, A, B = cfse.area_of_block(wl.frames, wl.avail, blk)
        mu = s[A].mean()
        ch0 = np.where(A, (s - mu) / 64.0, 0.0)
        assert np.array_equal(got[i, :, :, 1], A.astype(np.float32))
        assert np.abs(got[i, :, :, 0] - ch0).max() <= 2.0 ** -8 * np.abs(ch0).max() + 1e-6


def _oracle_forward_bf16(params, x):
    """The oracle's layers with every activation rounded to BF16, as the
    GPU stores them."""
    p = cnn.unflatten(params.astype(np.float64))
    h = x.astype(np.float64)
    for i in range(4):
        h = bf16(np.maximum(cnn.conv_forward(h, p[f"conv{i + 1}.w"], p[f"conv{i + 1}.b"]), 0.0)).astype(np.float64)
    feat = h.reshape(h.shape[0], -1)
    return feat @ p["head.w"].T + p["head.b"]


def _oracle_backward_bf16(p, x, target, pos_weight):
    """The oracle's gradients with the GPU's storage precision: activations
    stored in BF16 after each ReLU, and the operands of every backward
    product (dL/dlogits, dL/dz of each layer) rounded to BF16 as the GPU
    rounds them before its MFMA products; bias gradients from the unrounded
    values. Returns (logits, flat gradient)."""
    acts, pre = [x], []
    h = x
    for i in range(4):
        z = cnn.conv_forward(h, p[f"conv{i + 1}.w"], p[f"conv{i + 1}.b"])
        pre.append(z)
        h = bf16(np.maximum(z, 0.0)).astype(np.float64)
        acts.append(h)
    feat = h.reshape(h.shape[0], -1)
    logits = feat @ p["head.w"].T + p["head.b"]
    _, dl = cnn.bce_loss(logits, target, pos_weight)
    dlb = bf16(dl).astype(np.float64)
    g = {"head.w": dlb.T @ feat, "head.b": dl.sum(axis=0)}
    dh = (dlb @ p["head.w"]).reshape(acts[4].shape)
    for i in reversed(range(4)):
        dz = dh * (pre[i] > 0)
        dzb = bf16(dz).astype(np.float64)
        dx, dw, _ = cnn.conv_backward(acts[i], p[f"conv{i + 1}.w"], dzb)
        g[f"conv{i + 1}.w"], g[f"conv{i + 1}.b"] = dw, dz.sum(axis=(0, 1, 2))
        dh = dx
    return logits, cnn.flatten_grads(g)


def test_forward_matches_oracle():
    import torch
    from paper_2204_14193_amd import warm
    wl, img, av, plan, batch, x = _setup()
    _say("case cnn forward")
    params = cnn.init_params(7).astype(np.float32)
    params[cnn.n_params() - 4096:] = np.random.default_rng(1).normal(0, 0.1, 4096)   # nonzero head bias
    net = warm.Net(64, seed=0)
    net.set_params(params)
    logits = torch.empty((x.shape[0], 4096), dtype=torch.float32, device=x.device)
    net.forward(x, logits)
    torch.cuda.synchronize()
    got = logits.cpu().numpy()
    ref = _oracle_forward_bf16(bf16(params), x.float().cpu().numpy())
    _say(f"  logits relfro={_relfro(got, ref):.2e} cos={_cos(got, ref):.6f}")
    assert _relfro(got, ref) <= 5e-3 and _cos(got, ref) >= 0.9999
    net.close()


@pytest.mark.parametrize("case", ["256", "1080p-300"])
def test_forward_from_frames_equals_patches_then_forward(case):
    """fse_cnn_forward_blocks builds the inputs in LDS; its logits are the
    bits of fse_cnn_patches followed by fse_cnn_forward: a batch with frame
    edges in a non-trivial block order, and 300 blocks of a 1080p frame
    (ragged row tiles of the head product, spread over the XCDs)."""
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    _say(f"case forward from frames {case}")
    if case == "256":
        wl = workloads.subset(workloads.isolated_256(iters=30), np.arange(64)[::-1].copy())
    else:
        full = workloads.random_1080p_16x16(seeds=(100,), iters=0)
        wl = workloads.subset(full, np.arange(0, len(full.blocks), 2)[:300])
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, 4096)
    batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    n = len(wl.blocks)
    net = warm.Net(n)
    net.load()
    x = torch.empty((n, 48, 48, 2), dtype=torch.bfloat16, device=dev)
    warm.patches(batch, img, av, x)
    a = torch.empty((n, 4096), dtype=torch.float32, device=dev)
    b = torch.full((n, 4096), float("nan"), dtype=torch.float32, device=dev)
    net.forward(x, a)
    net.forward_blocks(batch, img, av, b)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    net.close()


def test_backward_matches_oracle_and_adam_step():
    import torch
    from paper_2204_14193_amd import warm
    wl, img, av, plan, batch, x = _setup()
    _say("case cnn backward")
    rng = np.random.default_rng(5)
    params = (cnn.init_params(9) * 0.7).astype(np.float32)
    net = warm.Net(64, seed=0)
    net.set_params(params)
    B = x.shape[0]
    tgt = rng.random((B, 4096)) < 0.03
    bits = np.packbits(tgt.reshape(B, 128, 32)[:, :, ::-1], axis=-1, bitorder="big").view(">u4").astype(np.uint32)
    bits = np.ascontiguousarray(bits.reshape(B, 128)).view(np.int32)
    tbits = torch.from_numpy(bits).to(x.device)
    logits = torch.empty((B, 4096), dtype=torch.float32, device=x.device)
    loss = torch.zeros(1, dtype=torch.float32, device=x.device)
    net.forward(x, logits, keep=True)
    net.backward(x, logits, tbits, 4.0, loss)
    torch.cuda.synchronize()
    _, g = net.get_params(grads=True)
    xin = x.float().cpu().numpy().astype(np.float64)
    pq = cnn.unflatten(bf16(params).astype(np.float64))
    lo, gref = _oracle_backward_bf16(pq, xin, tgt.astype(float), 4.0)
    l_ref, _ = cnn.bce_loss(lo, tgt.astype(float), 4.0)
    _say(f"  loss gpu={loss.item():.6f} oracle={l_ref:.6f}")
    assert abs(loss.item() - l_ref) <= 2e-3 * abs(l_ref)
    o = 0
    for name, shp in cnn.param_shapes():
        n = int(np.prod(shp))
        a, b = g[o:o + n], gref[o:o + n]
        _say(f"  {name:8s} relfro={_relfro(a, b):.2e} cos={_cos(a, b):.6f}")
        assert _relfro(a, b) <= 1e-2 and _cos(a, b) >= 0.9999, name
        o += n
    # one Adam step from zero moments: w -= lr * g / (|g| + eps)
    lr, eps = 1e-3, 1e-8
    net.adam(lr, 0.9, 0.999, eps)
    torch.cuda.synchronize()
    p1, g1 = net.get_params(grads=True)
    expect = params - lr * g / (np.abs(g) + eps)
    assert np.allclose(p1, expect, rtol=1e-5, atol=1e-7)
    assert not g1.any()
    net.close()


def test_topk_exact_with_ties_and_nan():
    import torch
    from paper_2204_14193_amd import warm
    _say("case topk")
    rng = np.random.default_rng(3)
    B, K = 6, 256
    lg = rng.normal(size=(B, 4096)).astype(np.float32)
    lg[1] = np.round(lg[1] * 2) / 2          # many exact ties
    lg[2, :] = 1.5                           # all equal
    lg[3, 100:600] = 7.0                     # ties across the threshold
    lg[4, 17] = np.nan                       # non-finite row
    lg[5] = -np.abs(lg[5])
    lg[5, ::7] = 0.0
    lg[5, 3::7] = -0.0                       # -0 ties with +0
    dev = torch.device("cuda:0")
    t = torch.from_numpy(lg).to(dev)
    cand = torch.full((B, K), -1, dtype=torch.int16, device=dev)
    flags = torch.full((B,), -1, dtype=torch.int32, device=dev)
    warm.topk(t, K, cand, flags)
    torch.cuda.synchronize()
    c, f = cand.cpu().numpy(), flags.cpu().numpy()
    assert f.tolist() == [0, 0, 0, 0, 1, 0]
    for b in (0, 1, 2, 3, 5):
        order = np.lexsort((np.arange(4096), -lg[b].astype(np.float64)))
        assert np.array_equal(c[b], np.sort(order[:K])), b


def test_topk_when_the_sample_misses_the_threshold():
    """Rows whose sampled bins (one per thread: bin 16 t + ((t ^ (t >> 4)) & 15))
    hold the largest values, so that the sample's bracket misses the K-th
    key and the selection falls back to a bisection over all keys; K values
    over the whole accepted range."""
    import torch
    from paper_2204_14193_amd import warm
    _say("case topk fallback")
    rng = np.random.default_rng(11)
    t = np.arange(256)
    sample_bins = 16 * t + ((t ^ (t >> 4)) & 15)
    dev = torch.device("cuda:0")
    for K in (1, 17, 255, 256, 300, 1000, 4095, 4096):
        lg = rng.normal(size=(4, 4096)).astype(np.float32)
        lg[0, sample_bins] = 10.0 + rng.random(256).astype(np.float32)   # sample far above the rest
        lg[1, sample_bins] = -10.0 - rng.random(256).astype(np.float32)  # far below
        lg[2, sample_bins] = 3.0                                         # tied block of the sample
        t_ = torch.from_numpy(lg).to(dev)
        cand = torch.full((4, K), -1, dtype=torch.int16, device=dev)
        flags = torch.full((4,), -1, dtype=torch.int32, device=dev)
        warm.topk(t_, K, cand, flags)
        torch.cuda.synchronize()
        c = cand.cpu().numpy()
        assert flags.cpu().numpy().tolist() == [0, 0, 0, 0]
        for b in range(4):
            order = np.lexsort((np.arange(4096), -lg[b].astype(np.float64)))
            assert np.array_equal(c[b], np.sort(order[:K])), (K, b)


def _warm_case(ir=30, iters=20, fb=40, kc=256, n_blocks=12, extra_iters=None):
    """Warm-started FSE on n_blocks isolated blocks with synthetic candidate
    sets; block 3 is flagged (plain fallback). extra_iters: append one more
    block with that iteration count (a batch whose largest count is then
    > 0 runs the single-kernel form)."""
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    idx = list(np.arange(0, 64, 64 // n_blocks)[:n_blocks])
    if extra_iters is not None:
        idx.append(63)
    wl = workloads.subset(workloads.isolated_256(iters=iters), idx)
    if extra_iters is not None:
        wl.blocks["iters"][-1] = extra_iters
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, 4096)
    batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    rng = np.random.default_rng(11)
    # candidate sets: low frequencies plus random bins, ascending
    cands = []
    for i in range(len(wl.blocks)):
        k = np.arange(4096)
        low = np.flatnonzero((np.minimum(k // 64, 64 - k // 64) < 6) & (np.minimum(k % 64, 64 - k % 64) < 6))
        rest = rng.choice(np.setdiff1d(k, low), kc - len(low), replace=False)
        cands.append(np.sort(np.concatenate([low, rest])))
    cands = np.stack(cands).astype(np.int16)
    flags = np.zeros(len(wl.blocks), np.int32)
    flags[3] = 1
    out = (img * (av != 0)).to(torch.float32)
    status = torch.full((len(wl.blocks),), -1, dtype=torch.int32, device=dev)
    stride = warm.trace_stride(batch, ir, fb)
    tr = torch.zeros((len(wl.blocks), stride * 16), dtype=torch.uint8, device=dev)
    warm.warm_extrapolate(batch, img, av, out, status, torch.from_numpy(cands).to(dev),
                          torch.from_numpy(flags).to(dev), kc, ir, fb, trace=tr)
    torch.cuda.synchronize()
    trace = tr.cpu().numpy().view(fse.TRACE_DTYPE).reshape(len(wl.blocks), stride)
    return wl, out.cpu().numpy(), status.cpu().numpy(), trace, cands, flags


def test_warm_fse_replays_against_oracle():
    ir, iters, fb = 30, 20, 40
    wl, out, st, trace, cands, flags = _warm_case(ir, iters, fb)
    _say(f"case warm fse: {len(wl.blocks)} blocks, ir={ir} I={iters} fallback={fb}")
    assert (st == 0).all()
    for i, blk in enumerate(wl.blocks):
        if flags[i]:
            continue
        r = parity.replay_warm_block(wl.frames, wl.avail, blk, wl.rho, wl.gamma, trace[i], cands[i], ir, iters)
        for ph in ("restricted", "full"):
            assert r[ph]["gap_violations"] == 0, (i, ph, r[ph])
            assert r[ph]["coef_max"] <= parity.COEF_TOL and r[ph]["coef_l2"] <= parity.COEF_TOL, (i, ph, r[ph])
        g = out[0, blk["y0"]:blk["y0"] + 16, blk["x0"]:blk["x0"] + 16]
        _say(f"  block {i}: restricted coef {r['restricted']['coef_max']:.1e}, full coef {r['full']['coef_max']:.1e}, "
             f"pix {np.abs(g - r['values']).max():.1e}")
        assert np.abs(g - r["values"]).max() < 0.05


def test_warm_fallback_is_plain_fse_bitwise():
    """A block flagged by candidate selection runs exactly plain FSE."""
    import torch
    import paper_2204_14193_amd as fse
    ir, iters, fb = 30, 20, 40
    wl, out, st, trace, cands, flags = _warm_case(ir, iters, fb)
    _say("case warm fallback")
    i = int(np.flatnonzero(flags)[0])
    sub = workloads.subset(wl, [i])
    sub.blocks["iters"] = fb
    dev = torch.device("cuda:0")
    img = torch.from_numpy(sub.distorted).to(dev)
    av = torch.from_numpy(sub.avail).to(dev)
    o2, s2, t2 = fse.extrapolate_batch(img, av, sub.blocks, sub.rho, sub.gamma, trace=True)
    b = wl.blocks[i]
    sl = (0, slice(b["y0"], b["y0"] + 16), slice(b["x0"], b["x0"] + 16))
    assert np.array_equal(o2.cpu().numpy()[sl], out[sl])
    assert np.array_equal(t2[0, :fb], trace[i, :fb])


def test_split_warm_replays_against_oracle():
    """Restricted iterations only (block iteration count 0): the transform
    kernel and the restricted kernel."""
    ir, fb = 40, 30
    for kc in (128, 256, 512):
        wl, out, st, trace, cands, flags = _warm_case(ir, 0, fb, kc=kc)
        _say(f"case split warm fse: kc={kc}, {len(wl.blocks)} blocks, ir={ir} fallback={fb}")
        assert (st == 0).all()
        for i, blk in enumerate(wl.blocks):
            if flags[i]:
                continue
            r = parity.replay_warm_block(wl.frames, wl.avail, blk, wl.rho, wl.gamma, trace[i], cands[i], ir, 0)
            rr = r["restricted"]
            assert rr["gap_violations"] == 0, (kc, i, rr)
            assert rr["coef_max"] <= parity.COEF_TOL and rr["coef_l2"] <= parity.COEF_TOL, (kc, i, rr)
            g = out[0, blk["y0"]:blk["y0"] + 16, blk["x0"]:blk["x0"] + 16]
            assert np.abs(g - r["values"]).max() < 0.05, (kc, i)


def test_warm_restricted_step_replays_against_oracle():
    """A restricted step other than the plan's gamma (fse_warm_set_restricted_gamma):
    the restricted phase replays against the oracle run with that step, in
    the two-kernel and the single-kernel form (whose full iterations keep
    the plan's gamma), and both forms give the same bits."""
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    ir, fb = 30, 20
    outs = []
    for iters in (0, 6):
        wl = workloads.subset(workloads.isolated_256(iters=iters), np.arange(0, 64, 6))
        n = len(wl.blocks)
        _say(f"case restricted step 1.0: {n} blocks, ir={ir}, full iterations {iters}")
        dev = torch.device("cuda:0")
        img = torch.from_numpy(wl.distorted).to(dev)
        av = torch.from_numpy(wl.avail).to(dev)
        plan = fse.Plan(wl.rho, wl.gamma, 4096)
        batch = fse.Batch(plan, wl.blocks, *wl.frames.shape)
        rng = np.random.default_rng(17)
        cands = np.stack([np.sort(rng.choice(4096, 256, replace=False)) for _ in range(n)]).astype(np.int16)
        flags = np.zeros(n, np.int32)
        warm.warm_prepare(batch, 256, ir, fb)
        warm.set_restricted_gamma(batch, 1.0)
        out = (img * (av != 0)).to(torch.float32)
        st = torch.full((n,), -1, dtype=torch.int32, device=dev)
        stride = warm.trace_stride(batch, ir, fb)
        tr = torch.zeros((n, stride * 16), dtype=torch.uint8, device=dev)
        warm.warm_extrapolate(batch, img, av, out, st, torch.from_numpy(cands).to(dev),
                              torch.from_numpy(flags).to(dev), 256, ir, fb, trace=tr)
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == 0).all()
        trace = tr.cpu().numpy().view(fse.TRACE_DTYPE).reshape(n, stride)
        o = out.cpu().numpy()
        for i, blk in enumerate(wl.blocks):
            r = parity.replay_warm_block(wl.frames, wl.avail, blk, wl.rho, wl.gamma, trace[i], cands[i], ir, iters,
                                         gamma_r=1.0)
            for ph in ("restricted", "full"):
                assert r[ph]["gap_violations"] == 0, (iters, i, ph, r[ph])
                assert r[ph]["coef_max"] <= parity.COEF_TOL and r[ph]["coef_l2"] <= parity.COEF_TOL, (iters, i, ph)
            g = o[0, blk["y0"]:blk["y0"] + 16, blk["x0"]:blk["x0"] + 16]
            assert np.abs(g - r["values"]).max() < parity.PIX_TOL, (iters, i)
        outs.append((o, trace[:, :ir]))
        batch.close()
        plan.close()
    # restricted selections and coefficients agree between the two forms
    assert np.array_equal(outs[0][1], outs[1][1])


def test_split_warm_equals_single_kernel_bitwise():
    """The two-kernel form computes the same bits as the single-kernel form
    (which a batch takes when some block also has full iterations)."""
    ir, fb = 40, 30
    for kc in (256, 512):
        _say(f"case split vs single kernel: kc={kc}")
        wl1, out1, st1, tr1, c1, f1 = _warm_case(ir, 0, fb, kc=kc)
        wl2, out2, st2, tr2, c2, f2 = _warm_case(ir, 0, fb, kc=kc, extra_iters=5)
        n = len(wl1.blocks)
        assert np.array_equal(c1, c2[:n]) and np.array_equal(st1, st2[:n])
        assert (st1 == 0).all()
        for i, blk in enumerate(wl1.blocks):
            sl = (0, slice(blk["y0"], blk["y0"] + 16), slice(blk["x0"], blk["x0"] + 16))
            assert np.array_equal(out1[sl], out2[sl]), (kc, i)
            m = fb if f1[i] else ir
            assert np.array_equal(tr1[i, :m], tr2[i, :m]), (kc, i)


def test_warm_start_quality_bar_and_timing_hook():
    """The packaged network at the package's operating point (chosen on
    validation frames) loses at most 0.1 dB of PSNR over the lost pixels
    against plain FSE with 100 iterations, on the eight benchmark frames;
    what the network adds: the same K, restricted iterations and step with
    candidates from the initial spectrum instead of the network, and plain
    FSE given about the warm step's time (45 iterations), both at least
    0.5 dB below it; the timing hook records both kernels of the split form."""
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    _say(f"case warm quality bar: K={warm.KC}, ir={warm.RESTRICTED_ITERS}, step={warm.RESTRICTED_GAMMA}")
    wl = workloads.random_1080p_16x16(seeds=tuple(range(99, 107)), iters=100)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    n = len(wl.blocks)
    out_p = img.to(torch.float32)
    st_p = torch.zeros(n, dtype=torch.int32, device=dev)
    plan = fse.Plan(wl.rho, wl.gamma, 4096)
    bp = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    bp.set_timing(4)
    bp.run(img, av, out_p, st_p)
    recs = bp.kernel_times()
    assert [(k, F) for k, F, _ in recs] == [("plain", 64)] and recs[0][2] > 0
    wb = wl.blocks.copy()
    wb["iters"] = 0
    bw = fse.Batch(plan, wb, *wl.frames.shape)
    net = warm.Net(n)
    net.load()
    ws = warm.WarmStart(net, bw)
    out_w = img.to(torch.float32)
    st_w = torch.zeros(n, dtype=torch.int32, device=dev)
    bw.set_timing(2)
    ws.run(img, av, out_w, st_w)
    ws.run(img, av, out_w, st_w)          # beyond the two records: untimed
    recs = bw.kernel_times()
    assert [(k, F) for k, F, _ in recs] == [("warm_prep", 64), ("restricted", 64)]
    assert all(ms > 0 for _, _, ms in recs)
    torch.cuda.synchronize()
    assert (st_p.cpu().numpy() == 0).all() and (st_w.cpu().numpy() == 0).all()
    assert int(ws.flags.sum().item()) == 0
    # the same warm start with candidates from the initial spectrum
    power = torch.empty((n, 4096), dtype=torch.float32, device=dev)
    cand = torch.empty_like(ws.cand)
    flags = torch.empty_like(ws.flags)
    warm.initial_power(bw, img, av, power)
    warm.topk(power, warm.KC, cand, flags)
    out_s = img.to(torch.float32)
    warm.warm_extrapolate(bw, img, av, out_s, st_w, cand, flags, warm.KC, warm.RESTRICTED_ITERS, 100)
    torch.cuda.synchronize()
    assert (st_w.cpu().numpy() == 0).all()

    def psnr(o):
        lost = wl.avail == 0
        e = np.clip(o[lost].astype(np.float64), 0, 255) - wl.frames[lost]
        return 10 * np.log10(255.0 ** 2 / np.mean(e ** 2))

    p_plain, p_warm, p_spec = psnr(out_p.cpu().numpy()), psnr(out_w.cpu().numpy()), psnr(out_s.cpu().numpy())
    # plain FSE given about the warm start's time
    b45 = wl.blocks.copy()
    b45["iters"] = 45
    bb = fse.Batch(plan, b45, *wl.frames.shape)
    out_45 = img.to(torch.float32)
    bb.run(img, av, out_45, st_p)
    torch.cuda.synchronize()
    p_45 = psnr(out_45.cpu().numpy())
    _say(f"  plain-100 {p_plain:.3f} dB, warm {p_warm:.3f} dB, spectrum candidates {p_spec:.3f} dB, "
         f"plain-45 {p_45:.3f} dB")
    assert p_plain - p_warm <= 0.1
    assert p_warm - p_spec >= 0.5
    assert p_warm - p_45 >= 0.5


def test_initial_power_spectrum():
    """fse_initial_power: |DFT(s w)|^2 of every bin (eq. (11)) against the
    oracle's projection in FP64 (relative to the block's largest value), and
    bit for bit the value plain FSE compares at its first selection."""
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    wl = workloads.subset(workloads.isolated_256(iters=1), np.arange(0, 64, 5))
    n = len(wl.blocks)
    _say(f"case initial power spectrum: {n} blocks")
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, 4096)
    blocks = wl.blocks.copy()
    blocks["iters"] = 0
    batch = fse.Batch(plan, blocks, *wl.frames.shape)
    pw = torch.full((n, 4096), -1.0, dtype=torch.float32, device=dev)
    warm.initial_power(batch, img, av, pw)
    torch.cuda.synchronize()
    got = pw.cpu().numpy()
    _, _, tr = fse.extrapolate_batch(img, av, wl.blocks, wl.rho, wl.gamma, trace=True)
    for i, blk in enumerate(wl.blocks):
        s, A, B = cfse.area_of_block(wl.frames, wl.avail, blk)
        w = cfse.weighting(*s.shape, wl.rho, A)
        R = cfse.project(s * w, cfse.analysis_matrix(64, s.shape[0]), cfse.analysis_matrix(64, s.shape[1]))
        ref = (np.abs(R) ** 2).ravel()
        assert np.abs(got[i] - ref).max() <= 2e-6 * ref.max(), i
        sel = int(tr[i, 0]["u"]) * 64 + int(tr[i, 0]["v"])
        assert got[i, sel] == tr[i, 0]["r2"] and got[i].max() == tr[i, 0]["r2"], i
    batch.close()
    plan.close()


def test_warm_leg_as_benchmarked_replays_against_oracle():
    """The benchmark's warm leg exactly as timed: the eight 1080p frames
    (6432 blocks), network candidates from the packaged weights at the
    package's operating point (top-KC bins, RESTRICTED_ITERS restricted
    iterations, in-loop model on B), one call of WarmStart.run with a trace.
    A seeded sample of 32 blocks is replayed against the oracle restricted
    to the same candidates: selections (near ties aside), coefficients,
    pixels, and the sample's PSNR against the free-running oracle."""
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    kc, ir, gr = warm.KC, warm.RESTRICTED_ITERS, warm.RESTRICTED_GAMMA
    wl = workloads.random_1080p_16x16(seeds=tuple(range(99, 107)), iters=100)
    n = len(wl.blocks)
    _say(f"case warm leg as benchmarked: {n} blocks, kc={kc}, ir={ir}, restricted gamma={gr}")
    gr = wl.gamma if gr is None else gr
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    wb = wl.blocks.copy()
    wb["iters"] = 0
    plan = fse.Plan(wl.rho, wl.gamma, ir + 100)
    bw = fse.Batch(plan, wb, *wl.frames.shape)
    net = warm.Net(n)
    net.load()
    ws = warm.WarmStart(net, bw, kc, ir, 100)
    out = img.to(torch.float32)
    st = torch.full((n,), -1, dtype=torch.int32, device=dev)
    stride = warm.trace_stride(bw, ir, 100)
    tr = torch.zeros((n, stride * 16), dtype=torch.uint8, device=dev)
    ws.run(img, av, out, st, trace=tr)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == fse.BLOCK_OK).all() and int(ws.flags.sum().item()) == 0
    trace = tr.cpu().numpy().view(fse.TRACE_DTYPE).reshape(n, stride)
    cand = ws.cand.cpu().numpy()
    o = out.cpu().numpy()
    idx = np.sort(np.random.default_rng(21).choice(n, 32, replace=False))
    worst = 0.0
    for i in idx:
        blk = wl.blocks[i]
        r = parity.replay_warm_block(wl.frames, wl.avail, blk, wl.rho, wl.gamma, trace[i], cand[i], ir, 0, gr)
        rr = r["restricted"]
        assert rr["gap_violations"] == 0, (i, rr)
        assert rr["coef_max"] <= parity.COEF_TOL and rr["coef_l2"] <= parity.COEF_TOL, (i, rr)
        f, y0, x0 = int(blk["frame"]), int(blk["y0"]), int(blk["x0"])
        pix = float(np.abs(o[f, y0:y0 + 16, x0:x0 + 16] - r["values"]).max())
        assert pix < parity.PIX_TOL, (i, pix)
        worst = max(worst, pix)
    d, pg, po = parity.warm_psnr_delta(wl.frames, wl.avail, wl.blocks[idx], cand[idx], wl.rho, gr, ir, o,
                                       processes=8)
    _say(f"  pix={worst:.2e} sample psnr gpu={pg:.4f} oracle={po:.4f}")
    assert d <= parity.PSNR_TOL
    net.close()


def test_split_warm_large_blocks_use_the_list_synthesis():
    """Blocks with more pixels than the restricted kernel keeps in registers
    (32x32 losses, border 8: 48x48 areas) take the coefficient-list
    synthesis; replayed against the oracle and bit-identical to the single
    kernel form."""
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    from synth import images, losses
    _say("case split warm, 32x32 blocks")
    ir, fb = 30, 20
    frame = images.synthetic_image(256, 256, 4)[None]
    blk = losses.blocks_to_array(losses.isolated_grid_losses(256, 256, 32, 8, 64, 0))
    avail = losses.availability_mask(frame.shape, losses.array_to_blocks(blk))
    rng = np.random.default_rng(5)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(frame * avail).to(dev)
    av = torch.from_numpy(avail).to(dev)
    n = len(blk)
    outs = []
    for extra in (False, True):
        b = blk.copy()
        if extra:  # one more block with full iterations: single-kernel form
            b = np.concatenate([b, losses.blocks_to_array([losses.Block(0, 0, 0, 8, 8, 8, 64, 3)])])
        plan = fse.Plan(0.8, 0.5, 4096)
        batch = fse.Batch(plan, b, 1, 256, 256)
        rng = np.random.default_rng(5)
        cands = np.stack([np.sort(rng.choice(4096, 256, replace=False)) for _ in range(len(b))]).astype(np.int16)
        flags = np.zeros(len(b), np.int32)
        out = (img * (av != 0)).to(torch.float32)
        st = torch.full((len(b),), -1, dtype=torch.int32, device=dev)
        stride = warm.trace_stride(batch, ir, fb)
        tr = torch.zeros((len(b), stride * 16), dtype=torch.uint8, device=dev)
        warm.warm_extrapolate(batch, img, av, out, st, torch.from_numpy(cands).to(dev),
                              torch.from_numpy(flags).to(dev), 256, ir, fb, trace=tr)
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == 0).all()
        outs.append((out.cpu().numpy(), tr.cpu().numpy().view(fse.TRACE_DTYPE).reshape(len(b), stride), cands))
    (o1, t1, c1), (o2, t2, c2) = outs
    for i in range(n):
        y0, x0 = int(blk["y0"][i]), int(blk["x0"][i])
        sl = (0, slice(y0, y0 + 32), slice(x0, x0 + 32))
        assert np.array_equal(o1[sl], o2[sl]), i
        assert np.array_equal(t1[i, :ir], t2[i, :ir]), i
    for i in range(0, n, 4):
        r = parity.replay_warm_block(frame, avail, blk[i], 0.8, 0.5, t1[i], c1[i], ir, 0)
        rr = r["restricted"]
        assert rr["gap_violations"] == 0 and rr["coef_max"] <= parity.COEF_TOL, (i, rr)
        y0, x0 = int(blk["y0"][i]), int(blk["x0"][i])
        assert np.abs(o1[0, y0:y0 + 32, x0:x0 + 32] - r["values"]).max() < 0.05, i
