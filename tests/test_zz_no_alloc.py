"""The allocation-free warm start (fse_warm_extrapolate_batch_noalloc)
against the allocating entry point (fse_warm_extrapolate_batch): same
kernels, so the same bits; two calls in a row, the second on a smaller
batch, the first spanning two ranges of the static staging."""
import numpy as np
import pytest

from synth import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _case(wl, kc, ir, fb, noalloc, net):
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    blocks = wl.blocks.copy()
    blocks["iters"] = 0
    n = len(blocks)
    plan = fse.Plan(wl.rho, wl.gamma, ir + fb)
    batch = fse.Batch(plan, blocks, *wl.frames.shape)
    logits = torch.empty((n, warm.N_BINS), dtype=torch.float32, device=dev)
    cand = torch.empty((n, kc), dtype=torch.int16, device=dev)
    flags = torch.empty((n,), dtype=torch.int32, device=dev)
    net.forward_blocks(batch, img, av, logits)
    warm.topk(logits, kc, cand, flags)
    flags[::97] = 1                                   # some blocks take the plain fallback
    out = (img * (av != 0)).to(torch.float32)
    status = torch.full((n,), -1, dtype=torch.int32, device=dev)
    stride = warm.trace_stride(batch, ir, fb)
    tr = torch.zeros((n, stride * 16), dtype=torch.uint8, device=dev)
    go = warm.warm_extrapolate_noalloc if noalloc else warm.warm_extrapolate
    go(batch, img, av, out, status, cand, flags, kc, ir, fb, trace=tr)
    torch.cuda.synchronize()
    res = out.cpu().numpy(), status.cpu().numpy(), tr.cpu().numpy(), cand.cpu().numpy()
    batch.close()
    plan.close()
    return res


def test_noalloc_warm_start_matches_the_allocating_entry_point():
    from paper_2204_14193_amd import warm
    kc, ir, fb = warm.KC, 40, 30
    big = workloads.random_1080p_16x16(seeds=(99, 100, 101, 102), iters=0)
    small = workloads.random_1080p_16x16(seeds=(103,), iters=0)
    small = workloads.subset(small, np.arange(0, len(small.blocks), 3))
    per = warm.noalloc_max_blocks(kc)
    _say(f"case noalloc warm start: {len(big.blocks)} then {len(small.blocks)} blocks, "
         f"{per} blocks per staging range, kc={kc}, ir={ir}")
    assert len(big.blocks) > per and len(small.blocks) < per     # the first call spans two ranges
    net = warm.Net(len(big.blocks), seed=0)
    net.load()
    for wl in (big, small):
        o1, s1, t1, c1 = _case(wl, kc, ir, fb, False, net)
        o2, s2, t2, c2 = _case(wl, kc, ir, fb, True, net)
        assert (s1 == 0).all() and np.array_equal(s1, s2)
        assert np.array_equal(c1, c2)
        assert np.array_equal(o1, o2)
        assert np.array_equal(t1, t2)
    assert warm.noalloc_max_blocks(1024) == 0
    net.close()
