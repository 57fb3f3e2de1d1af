"""Fixed-point cFSE: Algorithm 1 in integer arithmetic with one division
per block.

TEST INFRASTRUCTURE ONLY: used by tests/ and the benchmark's CPU-baseline
leg; never by the product path. Shares no code with the GPU side.

The paper's conclusion argues that cFSE suits fixed-point implementations
because its loop has no division: the only division is by W[0,0], once per
block, so rounding errors of repeated divisions cannot propagate. This
module fixes one such encoding (reading R20) exactly, so that any
implementation of it must agree bit for bit. Every quantity is an integer;
round(x / 2^s) is (x + 2^(s-1)) >> s with an arithmetic shift (ties
upward); all sums are exact in int64.

* window (eq. (3)):   wq = round(2^15 rho^d) (FP64, once per plan)
* twiddles:           T[j] = round(2^14 exp(-j 2 pi j / 64)), real and
                      imaginary parts rounded separately, j < 64
* input:              z[m,n] = s[m,n] wq[m,n] + j 2^7 wq[m,n] on the support
* transform (eq. (11)), separable and direct, exact sums:
      Y[m,l] = round(sum_n z[m,n] T[l n mod 64] / 2^14)
      Z[k,l] = round(sum_m Y[m,l] T[k m mod 64] / 2^23)
* split (a2):         R2 = Z[k,l] + conj(Z[-k,-l])           (= 2^7 R_w)
                      W2 = -j (Z[k,l] - conj(Z[-k,-l]))      (= 2^14 W)
* per block:          G = floor(round(2^16 gamma) 2^33 / W2[0,0])
* iteration (Algorithm 1):
      (u,v) = argmax R2x^2 + R2y^2, lowest linear index on ties   (eq. (12))
      c = round(R2[u,v] G / 2^26), per component   (eq. (13), c in 2^-16 px)
      R2[k,l] -= round(c W2[k-u, l-v] / 2^23), per component      (eq. (18))
* model on B:         out = round(sum_nu Re{c_nu conj(T[u m + v n])} / 2^22)
                      / 2^8 (pixel units)

The scales keep every stored value in int32 and every product in int64 for
48 x 48 areas of 8-bit pixels (bounds in the tests). The encoding is pinned
against the FP64 oracle (``oracle.cfse``) within error bounds that follow
from the roundings.
"""
import numpy as np

F = 64
Q_W = 15          # window scale
Q_T = 14          # twiddle scale
IMAG_SHIFT = 7    # z = s w + j 2^7 w
S_ROW, S_COL = 14, 23
S_G, S_UPD, S_OUT, Q_OUT, Q_C = 26, 23, 22, 8, 16


def rshift(x, s):
    """round(x / 2^s), ties upward, for int64 arrays or ints."""
    return (x + (1 << (s - 1))) >> s


def window_q(M, N, rho):
    """round(2^15 rho^d), d = distance to the area's centre (eq. (3))."""
    m = np.arange(M, dtype=np.float64)[:, None]
    n = np.arange(N, dtype=np.float64)[None, :]
    d = np.sqrt((m - (M - 1) / 2.0) ** 2 + (n - (N - 1) / 2.0) ** 2)
    return np.floor(np.power(float(rho), d) * (1 << Q_W) + 0.5).astype(np.int64)


def twiddles_q():
    """(re, im) int64 arrays: round(2^14 cos(2 pi j / 64)), round(-2^14 sin(..))."""
    j = np.arange(F, dtype=np.float64)
    re = np.floor(np.cos(2 * np.pi * j / F) * (1 << Q_T) + 0.5).astype(np.int64)
    im = np.floor(-np.sin(2 * np.pi * j / F) * (1 << Q_T) + 0.5).astype(np.int64)
    return re, im


def gamma_q(gamma):
    return int(np.floor(float(gamma) * (1 << 16) + 0.5))


def transform(zr, zi):
    """The two direct passes of the encoding: Z over the F x F grid from
    z on the M x N area (int64 arrays)."""
    M, N = zr.shape
    Tr, Ti = twiddles_q()
    n = np.arange(N)
    l = np.arange(F)
    Er, Ei = Tr[(l[:, None] * n[None, :]) % F], Ti[(l[:, None] * n[None, :]) % F]   # [l, n]
    Yr = rshift(zr @ Er.T - zi @ Ei.T, S_ROW)                                    # [m, l]
    Yi = rshift(zr @ Ei.T + zi @ Er.T, S_ROW)
    m = np.arange(M)
    k = np.arange(F)
    Cr, Ci = Tr[(k[:, None] * m[None, :]) % F], Ti[(k[:, None] * m[None, :]) % F]   # [k, m]
    Zr = rshift(Cr @ Yr - Ci @ Yi, S_COL)
    Zi = rshift(Cr @ Yi + Ci @ Yr, S_COL)
    return Zr, Zi


def split(Zr, Zi):
    """R2 = Z + conj(Z[-k,-l]) and W2 = -j (Z - conj(Z[-k,-l]))."""
    neg = (-np.arange(F)) % F
    Nr, Ni = Zr[np.ix_(neg, neg)], Zi[np.ix_(neg, neg)]
    return Zr + Nr, Zi - Ni, Zi + Ni, Nr - Zr


def cfse_fixed(s, wq, gamma, iters, forced=None):
    """Fixed-point cFSE of one area: s uint8-valued signal, wq int64 window
    (0 off the support). Returns dict(seq, c (int pairs), score, out (the
    model on the whole area in pixel units, float64), r2/w2 spectra) or
    None when W2[0,0] <= 0."""
    s = np.asarray(s, dtype=np.int64)
    wq = np.asarray(wq, dtype=np.int64)
    zr, zi = s * wq, wq << IMAG_SHIFT
    Zr, Zi = transform(zr, zi)
    Rx, Ry, Wx, Wy = split(Zr, Zi)
    W0 = int(Wx[0, 0])
    if W0 <= 0:
        return None
    G = (gamma_q(gamma) << 33) // W0
    Rx, Ry = Rx.copy(), Ry.copy()
    seq, cs, scores = [], [], []
    for nu in range(iters):
        sc = Rx * Rx + Ry * Ry                                     # eq. (12), exact
        idx = int(np.argmax(sc.ravel())) if forced is None else int(forced[nu])
        u, v = divmod(idx, F)
        cr, ci = int(rshift(int(Rx[u, v]) * G, S_G)), int(rshift(int(Ry[u, v]) * G, S_G))   # eq. (13)
        Sx = np.roll(np.roll(Wx, u, axis=0), v, axis=1)            # W2[k-u, l-v]
        Sy = np.roll(np.roll(Wy, u, axis=0), v, axis=1)
        Rx = Rx - rshift(cr * Sx - ci * Sy, S_UPD)                 # eq. (18)
        Ry = Ry - rshift(cr * Sy + ci * Sx, S_UPD)
        seq.append(idx)
        cs.append((cr, ci))
        scores.append(int(sc.ravel()[idx]))
    M, N = s.shape
    Tr, Ti = twiddles_q()
    m = np.arange(M)[:, None]
    n = np.arange(N)[None, :]
    acc = np.zeros((M, N), dtype=np.int64)
    for idx, (cr, ci) in zip(seq, cs):
        u, v = divmod(idx, F)
        ph = (u * m + v * n) % F
        acc += cr * Tr[ph] + ci * Ti[ph]                          # Re{c conj(T)} = Re{c e^{j theta}}
    out = rshift(acc, S_OUT).astype(np.float64) / (1 << Q_OUT)
    return dict(seq=seq, c=cs, score=scores, out=out, W0=W0, G=G)


def extrapolate_block(frames, avail, blk, rho, gamma, forced=None, iters=None):
    """Fixed-point cFSE for one block descriptor (F = 64): the run dict
    plus 'values' = the model on B, or None without support."""
    from . import cfse as c2
    if int(blk["fft"]) != F:
        raise ValueError("the fixed-point encoding is defined for F = 64")
    s, A, B = c2.area_of_block(frames, avail, blk)
    M, N = s.shape
    wq = np.where(A, window_q(M, N, rho), 0)
    I = int(blk["iters"]) if iters is None else iters
    res = cfse_fixed(np.where(A, s, 0).astype(np.int64), wq, gamma, I, forced=forced)
    if res is None:
        return None
    bd, bh, bw = int(blk["border"]), int(blk["bh"]), int(blk["bw"])
    res["values"] = res["out"][bd:bd + bh, bd:bd + bw].copy()
    return res
