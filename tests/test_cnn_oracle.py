"""Pins of the FP64 warm-start network oracle: the convolution against a
brute-force loop over its definition, the loss against a scalar formula, and
every gradient against central finite differences."""
import math

import numpy as np
import pytest

from oracle import cnn


def test_conv_matches_bruteforce_definition():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 6, 8, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = cnn.conv_forward(x, w, b)
    assert y.shape == (2, 3, 4, 4)
    for n in range(2):
        for oy in range(3):
            for ox in range(4):
                for o in range(4):
                    acc = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            iy, ix = 2 * oy - 1 + ky, 2 * ox - 1 + kx
                            if 0 <= iy < 6 and 0 <= ix < 8:
                                for c in range(3):
                                    acc += x[n, iy, ix, c] * w[o, ky, kx, c]
                    assert abs(y[n, oy, ox, o] - acc) < 1e-12


def test_bce_matches_scalar_formula():
    z = np.array([[-3.0, 0.0, 2.5, 40.0, -40.0]])
    t = np.array([[1.0, 0.0, 1.0, 0.0, 1.0]])
    pw = 3.0
    loss, _ = cnn.bce_loss(z, t, pw)
    ref = 0.0
    for zi, ti in zip(z[0], t[0]):
        s = 1.0 / (1.0 + math.exp(-zi))
        ref += -(pw * ti * math.log(s) + (1 - ti) * math.log1p(-s)) if 0 < s < 1 else \
            (-(pw * ti * (-math.log1p(math.exp(-zi)))) - (1 - ti) * (-math.log1p(math.exp(zi))))
    assert loss == pytest.approx(ref / z.size, rel=1e-12)


def test_shapes_and_param_count():
    assert cnn.n_params() == 32 * 9 * 2 + 32 + 3 * (32 * 9 * 32 + 32) + 4096 * 288 + 4096
    p = cnn.unflatten(cnn.init_params(1))
    x = np.random.default_rng(2).normal(size=(3, 48, 48, 2))
    logits, (acts, pre, feat) = cnn.forward(p, x)
    assert logits.shape == (3, 4096) and feat.shape == (3, 288)
    assert [a.shape[1] for a in acts] == [48, 24, 12, 6, 3]


def test_gradients_match_finite_differences():
    """Central differences (h = 1e-6) on a sample of parameters from every
    tensor: relative error 1e-6 above the differences' own rounding floor
    (about eps * loss / h = 2e-10 absolute)."""
    rng = np.random.default_rng(3)
    flat = cnn.init_params(4) * 0.5
    x = rng.normal(size=(2, 48, 48, 2))
    x[..., 1] = (rng.random((2, 48, 48)) > 0.3)
    target = (rng.random((2, 4096)) < 0.02).astype(float)
    pw = 4.0
    _, g = cnn.loss_and_grad(flat, x, target, pw)
    offsets, o = {}, 0
    for name, shp in cnn.param_shapes():
        offsets[name] = (o, int(np.prod(shp)))
        o += int(np.prod(shp))
    h = 1e-6
    for name, (start, size) in offsets.items():
        for idx in rng.choice(size, min(4, size), replace=False):
            i = start + int(idx)
            fp, fm = flat.copy(), flat.copy()
            fp[i] += h
            fm[i] -= h
            lp, _ = cnn.loss_and_grad(fp, x, target, pw)
            lm, _ = cnn.loss_and_grad(fm, x, target, pw)
            fd = (lp - lm) / (2 * h)
            scale = max(abs(fd), abs(g[i]), 1e-9)
            assert abs(fd - g[i]) <= 1e-6 * scale + 2e-10, (name, i, fd, g[i])
