"""Python binding of the learned warm start (argument marshalling only).

The network, its training and the warm-started FSE all run in libfse's HIP
kernels; torch tensors provide device memory and streams.
"""
import ctypes as C
import os

import numpy as np

from . import _lib
from .fse import _check

N_BINS = 4096
# Operating point of the packaged network: candidate bins per block,
# restricted iterations and their step, the fastest setting within 0.05 dB
# of plain FSE-100 on validation frames (seeds 5000-5007; the sweep is in
# weights/operating_point.json, written by paper_2204_14193_amd.operating_point)
KC = 256
RESTRICTED_ITERS = 60
RESTRICTED_GAMMA = 1.0       # None: the plan's gamma
PATCH = (48, 48, 2)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warm_cnn.npz")


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def num_params():
    return int(_lib.lib().fse_cnn_num_params())


class Net:
    """fse_cnn_t: FP32 master parameters, BF16 working copy, Adam state."""

    def __init__(self, max_batch, seed=0):
        h = C.c_void_p()
        _check(_lib.lib().fse_cnn_create(int(max_batch), C.c_uint64(seed), C.byref(h)), "fse_cnn_create")
        self._h = h
        self.max_batch = int(max_batch)

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == num_params()
        _check(_lib.lib().fse_cnn_set_params(self._h, p.ctypes.data_as(C.c_void_p)), "fse_cnn_set_params")

    def get_params(self, grads=False):
        p = np.empty(num_params(), np.float32)
        g = np.empty(num_params(), np.float32) if grads else None
        _check(_lib.lib().fse_cnn_get_params(self._h, p.ctypes.data_as(C.c_void_p),
                                             g.ctypes.data_as(C.c_void_p) if grads else None),
               "fse_cnn_get_params")
        return (p, g) if grads else p

    def forward(self, x, logits, keep=False, stream=None):
        """x: CUDA bfloat16 [B,48,48,2]; logits: CUDA float32 [B,4096]."""
        B = x.shape[0]
        _check(_lib.lib().fse_cnn_forward(self._h, _ptr(x), int(B), _ptr(logits), int(bool(keep)),
                                          _stream(stream)), "fse_cnn_forward")

    def forward_blocks(self, batch, image, avail, logits, stream=None):
        """Logits for every block of `batch`, inputs built from the frames."""
        _check(_lib.lib().fse_cnn_forward_blocks(self._h, batch._h, _ptr(image), _ptr(avail), image.stride(1),
                                                 _ptr(logits), _stream(stream)), "fse_cnn_forward_blocks")

    def backward(self, x, logits, target_bits, pos_weight, loss, stream=None):
        """target_bits: CUDA int32 [B,128]; loss: CUDA float32 [1] (added to)."""
        _check(_lib.lib().fse_cnn_backward(self._h, _ptr(x), _ptr(logits), _ptr(target_bits), int(x.shape[0]),
                                           float(pos_weight), _ptr(loss), _stream(stream)), "fse_cnn_backward")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_lib.lib().fse_cnn_adam(self._h, float(lr), float(beta1), float(beta2), float(eps),
                                       _stream(stream)), "fse_cnn_adam")

    def save(self, path):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        np.savez_compressed(path, params=self.get_params())

    def load(self, path=WEIGHTS):
        with np.load(path, allow_pickle=False) as z:
            self.set_params(z["params"])

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().fse_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def patches(batch, image, avail, x, stream=None):
    """Network inputs for every block of `batch` (48x48 areas) into x."""
    _check(_lib.lib().fse_cnn_patches(batch._h, _ptr(image), _ptr(avail), image.stride(1), _ptr(x),
                                      _stream(stream)), "fse_cnn_patches")


def initial_power(batch, image, avail, power, stream=None):
    """|DFT(s w)|^2 of every bin of every block of `batch` into power
    (CUDA float32 [n, 4096]): candidate sets from the initial spectrum."""
    _check(_lib.lib().fse_initial_power(batch._h, _ptr(image), _ptr(avail), image.stride(1), _ptr(power),
                                        _stream(stream)), "fse_initial_power")


def topk(logits, K, cand, flags, stream=None):
    _check(_lib.lib().fse_cnn_topk(_ptr(logits), int(logits.shape[0]), int(K), _ptr(cand), _ptr(flags),
                                   _stream(stream)), "fse_cnn_topk")


def trace_stride(batch, restricted_iters, fallback_iters):
    return int(_lib.lib().fse_warm_trace_stride(batch._h, int(restricted_iters), int(fallback_iters)))


def warm_prepare(batch, kc, restricted_iters, fallback_iters):
    """Kernel choice and staging of the warm start for these counts (the one
    allocating step; later warm launches with the same counts allocate nothing)."""
    _check(_lib.lib().fse_warm_prepare(batch._h, int(kc), int(restricted_iters), int(fallback_iters)),
           "fse_warm_prepare")


def set_restricted_gamma(batch, gamma_r):
    """Step of the restricted iterations (None: the plan's gamma)."""
    _check(_lib.lib().fse_warm_set_restricted_gamma(batch._h, -1.0 if gamma_r is None else float(gamma_r)),
           "fse_warm_set_restricted_gamma")


def warm_extrapolate(batch, image, avail, out, status, cand, flags, kc, restricted_iters, fallback_iters,
                     trace=None, stream=None):
    batch._check_tensors(image, avail, out, status)
    _check(_lib.lib().fse_warm_extrapolate_batch(
        batch._h, _ptr(image), _ptr(avail), image.stride(1), _ptr(out), out.stride(1), _ptr(status),
        None if trace is None else _ptr(trace), _ptr(cand), _ptr(flags), int(kc), int(restricted_iters),
        int(fallback_iters), _stream(stream)), "fse_warm_extrapolate_batch")


def warm_extrapolate_noalloc(batch, image, avail, out, status, cand, flags, kc, restricted_iters, fallback_iters,
                             trace=None, stream=None):
    """warm_extrapolate without any device allocation: the staging lives in
    the library's static per-device array (calls on one device must not
    overlap)."""
    batch._check_tensors(image, avail, out, status)
    _check(_lib.lib().fse_warm_extrapolate_batch_noalloc(
        batch._h, _ptr(image), _ptr(avail), image.stride(1), _ptr(out), out.stride(1), _ptr(status),
        None if trace is None else _ptr(trace), _ptr(cand), _ptr(flags), int(kc), int(restricted_iters),
        int(fallback_iters), _stream(stream)), "fse_warm_extrapolate_batch_noalloc")


def noalloc_max_blocks(kc):
    """Blocks per launch range of the allocation-free warm start."""
    return int(_lib.lib().fse_warm_noalloc_max_blocks(int(kc)))


class WarmStart:
    """The whole warm-started concealment of one batch: forward pass (inputs
    built from the frames), candidate sets, warm-started FSE. Buffers and the
    warm start's staging are allocated here; run() only launches kernels (it
    may be captured into a HIP graph from its first call on)."""

    def __init__(self, net, batch, kc=KC, restricted_iters=RESTRICTED_ITERS, fallback_iters=100,
                 restricted_gamma=RESTRICTED_GAMMA):
        import torch
        self.net, self.batch = net, batch
        self.gamma_r = restricted_gamma
        self.kc, self.ir, self.fb = int(kc), int(restricted_iters), int(fallback_iters)
        n = batch.n
        dev = torch.device("cuda")
        self.logits = torch.empty((n, N_BINS), dtype=torch.float32, device=dev)
        self.cand = torch.empty((n, self.kc), dtype=torch.int16, device=dev)
        self.flags = torch.empty((n,), dtype=torch.int32, device=dev)
        warm_prepare(batch, self.kc, self.ir, self.fb)
        set_restricted_gamma(batch, restricted_gamma)

    def run(self, image, avail, out, status, trace=None, stream=None):
        self.net.forward_blocks(self.batch, image, avail, self.logits, stream)
        topk(self.logits, self.kc, self.cand, self.flags, stream)
        warm_extrapolate(self.batch, image, avail, out, status, self.cand, self.flags, self.kc, self.ir, self.fb,
                         trace, stream)


class WarmStart3d:
    """Warm-started 3-D concealment. The 2-D network runs on each volume's
    first lost frame (its 48x48 area around the 16x16 hole, the input it was
    trained on) and its top-128 bins (k, l) become the volume's candidate
    columns; the 3-D iterations then run over those columns with every s
    (fse_warm3d_extrapolate_batch). Volumes must be 16x16 with a 16-pixel
    border. Buffers are allocated once; run() only launches kernels."""

    def __init__(self, net, batch3d, volumes, plan):
        import torch
        from .fse import Batch, BLOCK_DTYPE
        vols = np.ascontiguousarray(volumes)
        blocks = np.zeros(len(vols), dtype=BLOCK_DTYPE)
        for f in ("frame", "y0", "x0", "bh", "bw", "border"):
            blocks[f] = vols[f]
        blocks["fft"] = 64
        blocks["iters"] = 0
        self.net, self.batch3d = net, batch3d
        self.batch2d = Batch(plan, blocks, *batch3d.shape)
        n = len(vols)
        dev = torch.device("cuda")
        self.logits = torch.empty((n, N_BINS), dtype=torch.float32, device=dev)
        self.cand = torch.empty((n, 128), dtype=torch.int16, device=dev)
        self.flags = torch.empty((n,), dtype=torch.int32, device=dev)

    def run(self, frames, avail, out, status, trace=None, stream=None):
        self.net.forward_blocks(self.batch2d, frames, avail, self.logits, stream)
        topk(self.logits, 128, self.cand, self.flags, stream)
        self.batch3d.run_warm(frames, avail, out, status, self.cand, self.flags, trace, stream)

    def close(self):
        self.batch2d.close()
