"""FP64 forward and backward of the warm-start network.

TEST INFRASTRUCTURE ONLY: used by tests/ to check the GPU training and
inference kernels; never by the product path. Not from the paper (which has
no network): the architecture is the library's own.

Network (NHWC activations, weights [Cout][ky][kx][Cin]):
  x: [B, 48, 48, 2]       channel 0 = masked, centred patch, channel 1 = mask
  conv1..conv4: 3x3, stride 2, zero padding 1, bias, ReLU; 2->32->32->32->32
                channels, 48 -> 24 -> 12 -> 6 -> 3 pixels
  head: the 3x3x32 = 288 features (flattened y, x, c) -> 4096 logits (one per
        bin k*64 + l of the 64x64 transform), bias, no activation
Loss: binary cross-entropy with logits against the indicator of the bins
that plain FSE selected, positives weighted by pos_weight, averaged over
all B*4096 terms.

Everything here is plain numpy loops over taps and matrix products, written
for checking, not speed.
"""
import numpy as np

CH = 32
SIZES = (48, 24, 12, 6, 3)
CIN = (2, CH, CH, CH)
N_BINS = 4096
N_FEAT = 3 * 3 * CH


def param_shapes():
    """Ordered (name, shape) of every parameter tensor."""
    shapes = []
    for i, cin in enumerate(CIN):
        shapes.append((f"conv{i + 1}.w", (CH, 3, 3, cin)))
        shapes.append((f"conv{i + 1}.b", (CH,)))
    shapes.append(("head.w", (N_BINS, N_FEAT)))
    shapes.append(("head.b", (N_BINS,)))
    return shapes


def unflatten(flat):
    """Flat parameter vector -> dict of arrays (views)."""
    out, o = {}, 0
    for name, shp in param_shapes():
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp)
        o += n
    assert o == flat.size
    return out


def n_params():
    return sum(int(np.prod(s)) for _, s in param_shapes())


def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))


def conv_forward(x, w, b):
    """3x3 stride-2 convolution with zero padding 1: y[n,oy,ox,o] =
    b[o] + sum_{ky,kx,c} x[n, 2oy-1+ky, 2ox-1+kx, c] * w[o,ky,kx,c]."""
    B, H, W, C = x.shape
    Ho, Wo = H // 2, W // 2
    xp = _pad(x)
    y = np.zeros((B, Ho, Wo, w.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]          # [B,Ho,Wo,C]
            y += patch @ w[:, ky, kx, :].T
    return y


def conv_backward(x, w, dy):
    """Gradients of conv_forward: (dx, dw, db)."""
    B, H, W, C = x.shape
    Ho, Wo = H // 2, W // 2
    xp = _pad(x)
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]
            dw[:, ky, kx, :] = np.einsum("nhwo,nhwc->oc", dy, patch)
            dxp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :] += dy @ w[:, ky, kx, :]
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1, :], dw, db


def forward(params, x):
    """Returns (logits [B,4096], cache for backward)."""
    p = params
    acts = [x]
    pre = []
    h = x
    for i in range(4):
        z = conv_forward(h, p[f"conv{i + 1}.w"], p[f"conv{i + 1}.b"])
        pre.append(z)
        h = np.maximum(z, 0.0)
        acts.append(h)
    feat = h.reshape(h.shape[0], -1)                                     # (y, x, c) order
    logits = feat @ p["head.w"].T + p["head.b"]
    return logits, (acts, pre, feat)


def bce_loss(logits, target, pos_weight):
    """Mean over all terms of -(pw*t*log s(z) + (1-t)*log(1-s(z))), and its
    gradient with respect to the logits."""
    z = logits
    log_sig = -np.logaddexp(0.0, -z)          # log s(z)
    log_1m = -np.logaddexp(0.0, z)            # log (1 - s(z))
    terms = -(pos_weight * target * log_sig + (1.0 - target) * log_1m)
    sig = 1.0 / (1.0 + np.exp(-z))
    grad = (pos_weight * target * (sig - 1.0) + (1.0 - target) * sig) / z.size
    return float(terms.mean()), grad


def backward(params, cache, dlogits):
    """Gradient of the loss with respect to every parameter (dict)."""
    p = params
    acts, pre, feat = cache
    g = {"head.w": dlogits.T @ feat, "head.b": dlogits.sum(axis=0)}
    dh = (dlogits @ p["head.w"]).reshape(acts[4].shape)
    for i in reversed(range(4)):
        dz = dh * (pre[i] > 0)
        dx, dw, db = conv_backward(acts[i], p[f"conv{i + 1}.w"], dz)
        g[f"conv{i + 1}.w"], g[f"conv{i + 1}.b"] = dw, db
        dh = dx
    return g


def flatten_grads(g):
    return np.concatenate([g[name].ravel() for name, _ in param_shapes()])


def loss_and_grad(flat, x, target, pos_weight):
    params = unflatten(flat)
    logits, cache = forward(params, x)
    loss, dl = bce_loss(logits, target, pos_weight)
    return loss, flatten_grads(backward(params, cache, dl))


def init_params(seed):
    """He-uniform weights, zero biases (the scheme the training driver uses)."""
    rng = np.random.default_rng(seed)
    flat = np.zeros(n_params())
    p = unflatten(flat)
    for name, shp in param_shapes():
        if name.endswith(".w"):
            fan_in = int(np.prod(shp[1:]))
            lim = np.sqrt(6.0 / fan_in)
            p[name][...] = rng.uniform(-lim, lim, size=shp)
    return flat
