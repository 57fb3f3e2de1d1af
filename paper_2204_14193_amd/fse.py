"""Python binding of libfse (argument marshalling only).

Device memory and streams come from PyTorch; every step of the
extrapolation runs in the library's HIP kernels.
"""
import ctypes as C
import os

import numpy as np

from . import _lib

BLOCK_OK, BLOCK_EMPTY_SUPPORT, BLOCK_NONFINITE = 0, 1, 2
# FSE_KERNEL_* of include/fse.h, by value
KERNEL_KINDS = ("plain", "warm_fused", "warm_prep", "restricted", "real", "fixed")

BLOCK_DTYPE = np.dtype([("frame", "<i4"), ("y0", "<i4"), ("x0", "<i4"),
                        ("bh", "<i2"), ("bw", "<i2"), ("border", "<i2"),
                        ("fft", "<i2"), ("iters", "<i4")])
TRACE_DTYPE = np.dtype([("u", "<u2"), ("v", "<u2"), ("c_re", "<f4"),
                        ("c_im", "<f4"), ("r2", "<f4")])
VOLUME_DTYPE = np.dtype([("frame", "<i4"), ("y0", "<i4"), ("x0", "<i4"),
                         ("bt", "<i2"), ("bh", "<i2"), ("bw", "<i2"), ("border", "<i2"),
                         ("tborder", "<i2"), ("fft", "<i2"), ("fft_t", "<i2"), ("pad", "<i2"),
                         ("iters", "<i4")])
assert BLOCK_DTYPE.itemsize == C.sizeof(_lib.fse_block_t) == 24
assert VOLUME_DTYPE.itemsize == C.sizeof(_lib.fse_volume_t) == 32
assert TRACE_DTYPE.itemsize == C.sizeof(_lib.fse_trace_t) == 16

_STATUS = {0: "FSE_OK", -1: "FSE_ERR_INVALID_ARG", -2: "FSE_ERR_UNSUPPORTED",
           -3: "FSE_ERR_OOM", -4: "FSE_ERR_HIP", -5: "FSE_ERR_OVERLAP",
           -6: "FSE_ERR_WORKSPACE"}


class FseError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib.lib().fse_last_error().decode()
        super().__init__(f"{where}: {_STATUS.get(code, code)}: {msg}")


def _check(code, where):
    if code != 0:
        raise FseError(code, where)


def _blocks_array(blocks):
    arr = np.ascontiguousarray(blocks)
    if arr.dtype != BLOCK_DTYPE:
        arr = arr.astype(BLOCK_DTYPE)
    return arr


WS_WARM = 1  # FSE_WS_WARM: the workspace also holds the warm-start staging
PLAN_MASKED_B = 1  # FSE_PLAN_MASKED_B of include/fse.h
PLAN_REAL = 2      # FSE_PLAN_REAL: real-valued FSE (rFSE)
PLAN_FIXED = 4     # FSE_PLAN_FIXED: fixed-point cFSE
PLAN_REAL_INLOOP = 8  # FSE_PLAN_REAL_INLOOP: rFSE with the pair constants recomputed per iteration
PLAN_REAL_POWER = 16  # FSE_PLAN_REAL_POWER: rFSE selecting the pair of largest |R_w|^2


class Plan:
    """fse_plan_t: window decay rho, compensation gamma, iteration limit;
    masked=True makes every block's loss area the lost pixels of its
    rectangle (arbitrary loss shapes, FSE_PLAN_MASKED_B); real=True runs
    real-valued FSE instead of cFSE (FSE_PLAN_REAL, F = 64 blocks only);
    fixed=True runs the fixed-point cFSE encoding (FSE_PLAN_FIXED, F = 64);
    real="inloop" runs rFSE with its constants recomputed in every iteration;
    real="power" runs rFSE selecting the pair of largest |R_w|^2."""

    def __init__(self, rho=0.8, gamma=0.5, max_iters=4096, masked=False, real=False, fixed=False):
        L = _lib.lib()
        flags = (PLAN_MASKED_B if masked else 0) | (PLAN_REAL if real else 0) | (PLAN_FIXED if fixed else 0)
        if real == "inloop":
            flags |= PLAN_REAL_INLOOP
        elif real == "power":
            flags |= PLAN_REAL_POWER
        desc = _lib.fse_plan_desc_t(float(rho), float(gamma), int(max_iters), flags)
        h = C.c_void_p()
        _check(L.fse_plan_create(C.byref(desc), C.byref(h)), "fse_plan_create")
        self._h = h
        self.rho, self.gamma, self.max_iters = float(rho), float(gamma), int(max_iters)
        self.masked = bool(masked)
        self.real = bool(real)
        self.fixed = bool(fixed)

    @property
    def handle(self):
        return self._h

    def validate(self, blocks, n_frames, H, W):
        """Host-only check of a block list; returns (status, bad_index)."""
        arr = _blocks_array(blocks)
        bad = C.c_int32(-1)
        st = _lib.lib().fse_validate_blocks(self._h, arr.ctypes.data_as(C.c_void_p), len(arr),
                                            int(n_frames), int(H), int(W), C.byref(bad))
        return st, bad.value

    def workspace_size(self, n_blocks, warm=False):
        """Device bytes a Batch of n_blocks needs in a caller's workspace
        (fse_batch_workspace_size; warm=True adds the warm-start staging)."""
        n = C.c_size_t()
        _check(_lib.lib().fse_batch_workspace_size(self._h, int(n_blocks), WS_WARM if warm else 0, C.byref(n)),
               "fse_batch_workspace_size")
        return n.value

    def workspace3d_size(self, n_volumes):
        """Device bytes a Batch3d of n_volumes needs in a caller's workspace
        (fse_batch3d_workspace_size)."""
        n = C.c_size_t()
        _check(_lib.lib().fse_batch3d_workspace_size(self._h, int(n_volumes), C.byref(n)),
               "fse_batch3d_workspace_size")
        return n.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().fse_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """fse_batch_t: a validated, scheduled block list resident on the GPU."""

    def __init__(self, plan, blocks, n_frames, H, W, workspace=None, warm=False):
        """workspace: None (the library allocates the batch's device memory)
        or a CUDA uint8 tensor of at least plan.workspace_size(len(blocks),
        warm) bytes that holds it instead (fse_batch_create_in; the batch
        keeps a reference)."""
        arr = _blocks_array(blocks)
        h = C.c_void_p()
        if workspace is None:
            _check(_lib.lib().fse_batch_create(plan.handle, arr.ctypes.data_as(C.c_void_p), len(arr),
                                               int(n_frames), int(H), int(W), C.byref(h)),
                   "fse_batch_create")
        else:
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous CUDA tensor")
            _check(_lib.lib().fse_batch_create_in(
                plan.handle, arr.ctypes.data_as(C.c_void_p), len(arr), int(n_frames), int(H), int(W),
                C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                WS_WARM if warm else 0, C.byref(h)), "fse_batch_create_in")
        self._workspace = workspace
        self._h = h
        self.plan = plan
        self.n = len(arr)
        self.shape = (int(n_frames), int(H), int(W))
        self.max_iters = _lib.lib().fse_batch_max_iters(h)

    def launch_info(self, F):
        t, w, g, l = (C.c_int32() for _ in range(4))
        _check(_lib.lib().fse_batch_launch_info(self._h, int(F), C.byref(t), C.byref(w),
                                                C.byref(g), C.byref(l)), "fse_batch_launch_info")
        return dict(threads=t.value, wg_per_cu=w.value, grid=g.value, lds_bytes=l.value)

    def set_timing(self, max_records):
        """Record HIP events around each of the next max_records kernels this
        batch launches (0 = off); read them with kernel_times()."""
        _check(_lib.lib().fse_batch_set_timing(self._h, int(max_records)), "fse_batch_set_timing")

    def kernel_times(self):
        """[(kind, F, ms), ...] of the recorded kernels in launch order; kind
        is one of KERNEL_KINDS. Waits for them."""
        n = int(_lib.lib().fse_batch_kernel_times(self._h, None, None, None, 0))
        if n < 0:
            _check(n, "fse_batch_kernel_times")
        ms = np.zeros(max(n, 1), np.float32)
        kind = np.zeros(max(n, 1), np.int32)
        fft = np.zeros(max(n, 1), np.int32)
        got = int(_lib.lib().fse_batch_kernel_times(self._h, ms.ctypes.data_as(C.c_void_p),
                                                    kind.ctypes.data_as(C.c_void_p),
                                                    fft.ctypes.data_as(C.c_void_p), n))
        if got < 0:
            _check(got, "fse_batch_kernel_times")
        return [(KERNEL_KINDS[int(kind[i])], int(fft[i]), float(ms[i])) for i in range(min(n, got))]

    def set_variant(self, F, threads):
        _check(_lib.lib().fse_batch_set_variant(self._h, int(F), int(threads)), "fse_batch_set_variant")

    def autotune(self, image, avail, out, status, reps=3, stream=None, cache=None):
        """Time every compiled workgroup shape on these inputs and keep the
        fastest per transform size; returns [(F, threads, us), ...] (us None
        for a decision taken from the cache file `cache`, if given)."""
        import torch
        self._check_tensors(image, avail, out, status)
        s = stream if stream is not None else torch.cuda.current_stream()
        buf = C.create_string_buffer(4096)
        _check(_lib.lib().fse_batch_autotune_cached(
            self._h, C.c_void_p(image.data_ptr()), C.c_void_p(avail.data_ptr()), image.stride(1),
            C.c_void_p(out.data_ptr()), out.stride(1), C.c_void_p(status.data_ptr()), int(reps),
            C.c_void_p(s.cuda_stream), buf, len(buf), None if cache is None else os.fsencode(cache)),
            "fse_batch_autotune_cached")
        rows = []
        for line in buf.value.decode().splitlines():
            f, t, us = line.split()
            rows.append((int(f), int(t), None if us == "cached" else float(us)))
        return rows

    def _check_tensors(self, image, avail, out, status):
        import torch
        nf, H, W = self.shape
        for name, t, dt in (("image", image, torch.uint8), ("avail", avail, torch.uint8),
                            ("out", out, torch.float32)):
            if not t.is_cuda or t.dtype != dt or tuple(t.shape) != (nf, H, W) or t.stride(2) != 1 \
                    or t.stride(0) != t.stride(1) * H:
                raise ValueError(f"{name} must be a CUDA {dt} tensor of shape {(nf, H, W)} with dense frames")
        if image.stride(1) != avail.stride(1):
            raise ValueError("image and avail must share a pitch")
        if not status.is_cuda or status.dtype != torch.int32 or status.numel() < self.n:
            raise ValueError("status must be a CUDA int32 tensor with one entry per block")

    def run(self, image, avail, out, status, trace=None, stream=None):
        """Launch on torch CUDA tensors: image/avail uint8 [F,H,W] (rows may
        be padded: pitch = stride(1)), out float32 [F,H,W], status int32
        [n], trace None or uint8 [n, max_iters*16]. Asynchronous."""
        import torch
        self._check_tensors(image, avail, out, status)
        tptr = None
        if trace is not None:
            if not trace.is_cuda or trace.numel() * trace.element_size() < self.n * self.max_iters * 16:
                raise ValueError("trace buffer too small")
            tptr = C.c_void_p(trace.data_ptr())
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(_lib.lib().fse_extrapolate_batch(
            self._h, C.c_void_p(image.data_ptr()), C.c_void_p(avail.data_ptr()), image.stride(1),
            C.c_void_p(out.data_ptr()), out.stride(1), C.c_void_p(status.data_ptr()), tptr,
            C.c_void_p(s.cuda_stream)), "fse_extrapolate_batch")

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().fse_batch_destroy(self._h)
            self._h = None
            self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch3d:
    """fse_batch3d_t: validated lost volumes of a clip, resident on the GPU
    (3-D cFSE, 64 x 64 x 8 transform)."""

    def __init__(self, plan, volumes, n_frames, H, W, workspace=None):
        """workspace: None, or a CUDA uint8 tensor of at least
        Plan.workspace3d_size(len(volumes)) bytes that holds the batch's
        device memory (fse_batch3d_create_in; the batch keeps a reference)."""
        arr = np.ascontiguousarray(volumes)
        if arr.dtype != VOLUME_DTYPE:
            arr = arr.astype(VOLUME_DTYPE)
        h = C.c_void_p()
        bad = C.c_int32(-1)
        if workspace is None:
            st = _lib.lib().fse_batch3d_create(plan.handle, arr.ctypes.data_as(C.c_void_p), len(arr), int(n_frames),
                                               int(H), int(W), C.byref(h), C.byref(bad))
            _check(st, f"fse_batch3d_create (volume {bad.value})")
        else:
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous CUDA tensor")
            st = _lib.lib().fse_batch3d_create_in(
                plan.handle, arr.ctypes.data_as(C.c_void_p), len(arr), int(n_frames), int(H), int(W),
                C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(), C.byref(h),
                C.byref(bad))
            _check(st, f"fse_batch3d_create_in (volume {bad.value})")
        self._workspace = workspace
        self._h = h
        self.plan = plan
        self.n = len(arr)
        self.shape = (int(n_frames), int(H), int(W))
        self.max_iters = int(arr["iters"].max()) if len(arr) else 0

    def run(self, frames, avail, out, status, trace=None, stream=None):
        """frames/avail uint8 [F,H,W], out float32 [F,H,W] (CUDA, dense
        frames), status int32 [n], trace None or uint8 [n, max_iters*16]."""
        import torch
        Batch._check_tensors(self, frames, avail, out, status)
        tptr = None
        if trace is not None:
            if not trace.is_cuda or trace.numel() * trace.element_size() < self.n * self.max_iters * 16:
                raise ValueError("trace buffer too small")
            tptr = C.c_void_p(trace.data_ptr())
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(_lib.lib().fse_extrapolate3d_batch(
            self._h, C.c_void_p(frames.data_ptr()), C.c_void_p(avail.data_ptr()), frames.stride(1),
            C.c_void_p(out.data_ptr()), out.stride(1), C.c_void_p(status.data_ptr()), tptr,
            C.c_void_p(s.cuda_stream)), "fse_extrapolate3d_batch")

    def run_warm(self, frames, avail, out, status, cand2, flags, trace=None, stream=None):
        """Warm-started form (fse_warm3d_extrapolate_batch): cand2 int16
        [n, 128] candidate columns k*64+l per volume (ascending), flags
        int32 [n] (nonzero: volume skipped with status BLOCK_NONFINITE)."""
        import torch
        Batch._check_tensors(self, frames, avail, out, status)
        if not cand2.is_cuda or cand2.dtype != torch.int16 or tuple(cand2.shape) != (self.n, 128) \
                or not cand2.is_contiguous():
            raise ValueError("cand2 must be a contiguous CUDA int16 tensor [n, 128]")
        if not flags.is_cuda or flags.dtype != torch.int32 or flags.numel() < self.n:
            raise ValueError("flags must be a CUDA int32 tensor with one entry per volume")
        tptr = None
        if trace is not None:
            if not trace.is_cuda or trace.numel() * trace.element_size() < self.n * self.max_iters * 16:
                raise ValueError("trace buffer too small")
            tptr = C.c_void_p(trace.data_ptr())
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(_lib.lib().fse_warm3d_extrapolate_batch(
            self._h, C.c_void_p(frames.data_ptr()), C.c_void_p(avail.data_ptr()), frames.stride(1),
            C.c_void_p(out.data_ptr()), out.stride(1), C.c_void_p(status.data_ptr()), tptr,
            C.c_void_p(cand2.data_ptr()), C.c_void_p(flags.data_ptr()), 128, C.c_void_p(s.cuda_stream)),
            "fse_warm3d_extrapolate_batch")

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().fse_batch3d_destroy(self._h)
            self._h = None
            self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def extrapolate3d(frames, avail, volumes, rho=0.8, gamma=0.5, trace=False, out=None):
    """3-D cFSE of lost ``volumes`` (VOLUME_DTYPE) in a clip ``frames`` (uint8
    CUDA [F,H,W]) with availability ``avail``. Returns (out float32, status
    numpy, trace numpy [n, max_iters] of TRACE_DTYPE or None)."""
    import torch
    arr = np.ascontiguousarray(volumes).astype(VOLUME_DTYPE)
    nf, H, W = frames.shape
    plan = Plan(rho, gamma, max(4096, int(arr["iters"].max()) if len(arr) else 0))
    batch = Batch3d(plan, arr, nf, H, W)
    if out is None:
        out = (frames * (avail != 0)).to(torch.float32)
    status = torch.full((max(len(arr), 1),), -1, dtype=torch.int32, device=frames.device)
    tbuf = None
    if trace and batch.max_iters > 0:
        tbuf = torch.zeros((len(arr), batch.max_iters * 16), dtype=torch.uint8, device=frames.device)
    batch.run(frames, avail, out, status, tbuf)
    torch.cuda.synchronize()
    st = status.cpu().numpy()[:len(arr)]
    tr = None if tbuf is None else tbuf.cpu().numpy().view(TRACE_DTYPE).reshape(len(arr), batch.max_iters)
    batch.close()
    plan.close()
    return out, st, tr


def blocks_from_mask(avail, cell=16, border=16, fft=64, iters=100):
    """Blocks covering the lost pixels of ``avail`` (uint8 numpy [F,H,W] or
    [H,W], 0 = lost) with cell x cell tiles (fse_blocks_from_mask), for a
    plan with masked=True. Host-only."""
    av = np.ascontiguousarray(avail, dtype=np.uint8)
    if av.ndim == 2:
        av = av[None]
    nf, H, W = av.shape
    L = _lib.lib()
    n = C.c_int32(0)
    args = (av.ctypes.data_as(C.c_void_p), nf, H, W, W, int(cell), int(border), int(fft), int(iters))
    _check(L.fse_blocks_from_mask(*args, None, 0, C.byref(n)), "fse_blocks_from_mask")
    arr = np.zeros(n.value, dtype=BLOCK_DTYPE)
    got = C.c_int32(0)
    _check(L.fse_blocks_from_mask(*args, arr.ctypes.data_as(C.c_void_p), len(arr), C.byref(got)),
           "fse_blocks_from_mask")
    return arr


def extrapolate_batch(image, avail, blocks, rho=0.8, gamma=0.5, trace=False, out=None, masked=False, real=False,
                      fixed=False):
    """Conceal ``blocks`` in frames ``image`` (uint8 CUDA tensor [F,H,W] or
    [H,W]) with availability ``avail``. Returns (out float32, status int32
    numpy, trace numpy of TRACE_DTYPE [n, max_iters] or None). ``out``
    defaults to the distorted frames as float32. ``masked``: mask-driven
    loss areas; ``real``: rFSE; ``fixed``: fixed-point cFSE (see Plan)."""
    import torch
    if image.dim() == 2:
        image, avail = image[None], avail[None]
    arr = _blocks_array(blocks)
    nf, H, W = image.shape
    plan = Plan(rho, gamma, max(4096, int(arr["iters"].max()) if len(arr) else 0), masked=masked, real=real,
                fixed=fixed)
    batch = Batch(plan, arr, nf, H, W)
    if out is None:
        out = (image * (avail != 0)).to(torch.float32)
    status = torch.full((max(len(arr), 1),), -1, dtype=torch.int32, device=image.device)
    tbuf = None
    if trace and batch.max_iters > 0:
        tbuf = torch.zeros((len(arr), batch.max_iters * 16), dtype=torch.uint8, device=image.device)
    batch.run(image, avail, out, status, tbuf)
    torch.cuda.synchronize()
    st = status.cpu().numpy()[:len(arr)]
    tr = None
    if tbuf is not None:
        tr = tbuf.cpu().numpy().view(TRACE_DTYPE).reshape(len(arr), batch.max_iters)
    batch.close()
    plan.close()
    return out, st, tr


def measure_lds_bandwidth(iters=2000):
    """Aggregate LDS read bandwidth of the current device in bytes/s
    (fse_measure_lds_bandwidth), for roofline accounting."""
    import torch
    out = C.c_double(0.0)
    _check(_lib.lib().fse_measure_lds_bandwidth(int(iters), C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                                C.byref(out)), "fse_measure_lds_bandwidth")
    return out.value
