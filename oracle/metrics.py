"""Quality measures. TEST INFRASTRUCTURE ONLY (tests/ and the benchmark's
CPU-baseline and quality legs).

The paper reports extrapolation quality as PSNR (Section IV). Here PSNR is
taken over the lost pixels of a frame (the union of all B), with the
reconstruction clipped to the 8-bit range first.
"""
import numpy as np


def psnr_lost(reference, reconstruction, avail):
    """10*log10(255^2 / MSE) over pixels with avail == 0."""
    lost = avail == 0
    rec = np.clip(np.asarray(reconstruction, dtype=np.float64), 0.0, 255.0)
    err = rec[lost] - np.asarray(reference, dtype=np.float64)[lost]
    mse = float(np.mean(err ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


def psnr_between(a, b, avail):
    """PSNR of one reconstruction against another over the lost pixels."""
    lost = avail == 0
    err = np.asarray(a, dtype=np.float64)[lost] - np.asarray(b, dtype=np.float64)[lost]
    mse = float(np.mean(err ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)
