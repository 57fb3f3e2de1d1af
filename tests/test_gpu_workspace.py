"""Batches in a caller's workspace (fse_batch_create_in, fse_batch3d_create_in):
the same results, bit for bit, as batches whose device memory the library
allocates, for the three transform sizes, the fixed-point plan, the warm
start and 3-D volumes; the device-side rejections of a workspace.

Each test prints the case it runs before touching the GPU.
"""
import numpy as np
import pytest

from synth import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _workspace(plan, n, warm=False, extra=0):
    import torch
    nbytes = plan.workspace_size(n, warm) + extra
    return torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda:0")   # not zeroed on purpose


def _run(batch, img, av, trace_rows):
    import torch
    out = (img * (av != 0)).to(torch.float32)
    status = torch.full((batch.n,), -1, dtype=torch.int32, device=img.device)
    tr = torch.zeros((batch.n, max(trace_rows, 1) * 16), dtype=torch.uint8, device=img.device)
    batch.run(img, av, out, status, trace=tr)
    torch.cuda.synchronize()
    return out.cpu().numpy(), status.cpu().numpy(), tr.cpu().numpy()


@pytest.mark.parametrize("kind", ["mixed", "fixed"])
def test_workspace_batch_matches_the_allocating_batch(kind):
    import torch
    import paper_2204_14193_amd as fse
    if kind == "mixed":
        wl = workloads.mixed_4k(seeds=(2,))
        wl = workloads.subset(wl, np.arange(0, len(wl.blocks), 7))
        plan = fse.Plan(wl.rho, wl.gamma, int(wl.blocks["iters"].max()))
    else:
        wl = workloads.isolated_256(iters=60)
        plan = fse.Plan(wl.rho, wl.gamma, 60, fixed=True)
    sizes = sorted(set(int(f) for f in wl.blocks["fft"]))
    _say(f"case workspace batch {kind}: {len(wl.blocks)} blocks, transforms {sizes}")
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    ref = fse.Batch(plan, wl.blocks, *wl.frames.shape)
    o1, s1, t1 = _run(ref, img, av, ref.max_iters)
    ref.close()
    ws = _workspace(plan, len(wl.blocks), extra=4096)
    for rep in range(2):                             # the second batch reuses the first one's workspace
        b = fse.Batch(plan, wl.blocks, *wl.frames.shape, workspace=ws)
        o2, s2, t2 = _run(b, img, av, b.max_iters)
        b.close()
        assert (s1 == 0).all() and np.array_equal(s1, s2), rep
        assert np.array_equal(o1, o2), rep
        assert np.array_equal(t1, t2), rep
    plan.close()


def test_workspace_batch_warm_start_and_capture_on_first_use():
    """The warm start on a batch whose staging lies in its workspace: the
    same bits as on a library-allocated batch; its first call captured into
    a graph replays bit-identical; without FSE_WS_WARM the set-up fails with
    FSE_ERR_WORKSPACE."""
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import warm
    wl = workloads.random_1080p_16x16(seeds=(100,), iters=0)
    blocks = wl.blocks
    n = len(blocks)
    _say(f"case workspace batch warm start: {n} blocks")
    dev = torch.device("cuda:0")
    img = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, warm.RESTRICTED_ITERS + 100)
    net = warm.Net(n, seed=0)
    net.load()
    base = (img * (av != 0)).to(torch.float32)
    status = torch.full((n,), -1, dtype=torch.int32, device=dev)

    ref = fse.Batch(plan, blocks, *wl.frames.shape)
    w_ref = warm.WarmStart(net, ref)
    out_ref = base.clone()
    w_ref.run(img, av, out_ref, status)
    torch.cuda.synchronize()
    assert (status == 0).all()
    cand_ref = w_ref.cand.clone()
    ref.close()

    bare = fse.Batch(plan, blocks, *wl.frames.shape, workspace=_workspace(plan, n))
    with pytest.raises(fse.FseError) as e:
        warm.WarmStart(net, bare)
    assert e.value.code == -6
    bare.close()

    b = fse.Batch(plan, blocks, *wl.frames.shape, workspace=_workspace(plan, n, warm=True), warm=True)
    w = warm.WarmStart(net, b)
    out = base.clone()
    status.fill_(-1)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        w.run(img, av, out, status, stream=s)
    out.copy_(base)
    w.run(img, av, out, status)
    torch.cuda.synchronize()
    assert (status == 0).all()
    assert torch.equal(w.cand, cand_ref) and torch.equal(out, out_ref)
    for rep in range(3):
        out.copy_(base)
        status.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert (status == 0).all(), rep
        assert torch.equal(out, out_ref), rep
        _ = (base * 2).sum().item()                 # unrelated eager work between replays
    del g
    b.close()
    net.close()
    plan.close()


def test_workspace_device_rejections():
    """A workspace in pinned host memory, one that is not 256-byte aligned
    and one smaller than fse_batch_workspace_size are refused, and no batch
    is made."""
    import ctypes as C
    import torch
    import paper_2204_14193_amd as fse
    from paper_2204_14193_amd import _lib
    wl = workloads.isolated_256(iters=20)
    _say(f"case workspace rejections: {len(wl.blocks)} blocks")
    plan = fse.Plan(wl.rho, wl.gamma, 20)
    arr = np.ascontiguousarray(wl.blocks)
    need = plan.workspace_size(len(arr))
    dev_ws = torch.empty((need + 256,), dtype=torch.uint8, device="cuda:0")
    host_ws = torch.empty((need,), dtype=torch.uint8).pin_memory()
    L = _lib.lib()
    for ptr, size, code in ((host_ws.data_ptr(), need, -1), (dev_ws.data_ptr() + 8, need, -1),
                            (dev_ws.data_ptr(), need - 256, -6)):
        h = C.c_void_p()
        st = L.fse_batch_create_in(plan.handle, arr.ctypes.data_as(C.c_void_p), len(arr), *wl.frames.shape,
                                   C.c_void_p(ptr), size, 0, C.byref(h))
        assert st == code and not h.value, (st, L.fse_last_error())
    b = fse.Batch(plan, wl.blocks, *wl.frames.shape, workspace=dev_ws[256:])   # offset by 256: aligned
    b.close()
    plan.close()


def test_workspace_batch3d_matches_the_allocating_batch():
    """A 3-D batch in a caller's workspace gives the allocating batch's
    output and status, bit for bit, twice in a row on the same workspace."""
    import torch
    import paper_2204_14193_amd as fse
    wl = workloads.clip_small()
    n = len(wl.blocks)
    _say(f"case workspace batch3d: {n} volumes")
    dev = torch.device("cuda:0")
    fr = torch.from_numpy(wl.distorted).to(dev)
    av = torch.from_numpy(wl.avail).to(dev)
    plan = fse.Plan(wl.rho, wl.gamma, int(wl.blocks["iters"].max()))

    def run(b):
        out = (fr * (av != 0)).to(torch.float32)
        st = torch.full((n,), -1, dtype=torch.int32, device=dev)
        b.run(fr, av, out, st)
        torch.cuda.synchronize()
        return out.cpu().numpy(), st.cpu().numpy()

    ref = fse.Batch3d(plan, wl.blocks, *wl.frames.shape)
    o1, s1 = run(ref)
    ref.close()
    ws = torch.full((plan.workspace3d_size(n) + 512,), 0x5A, dtype=torch.uint8, device=dev)
    for rep in range(2):
        b = fse.Batch3d(plan, wl.blocks, *wl.frames.shape, workspace=ws)
        o2, s2 = run(b)
        b.close()
        assert (s1 == 0).all() and np.array_equal(s1, s2), rep
        assert np.array_equal(o1, o2), rep
    plan.close()
