"""Plain FP64 complex-valued FSE in three dimensions (video), by direct
spatio-temporal projection.

TEST INFRASTRUCTURE ONLY: used by tests/ and the benchmark's CPU-baseline
leg; never by the product path. Shares no code with the GPU side.

The paper derives cFSE for images and states that it extends to more
dimensions, where its advantage over the real-valued form grows (Section II
and the Conclusion, both referring to its reference on higher-dimensional
extrapolation [Meisinger2007]). This module is the same
algorithm as ``oracle.cfse`` (eqs. (3), (7)-(10), (13), (14), (17)) with one
more axis:

* the area L is M x N pixels x T frames around a lost volume B of
  bh x bw pixels x bt frames (border b in space, bt_border in time);
* the basis is phi_(k,l,s)[m,n,t] = exp(j2pi(k m / F + l n / F + s t / Ft))
  on an F x F x Ft grid; the linear bin index is (k F + l) Ft + s, so that
  with Ft = T = 1 everything reduces to the 2-D oracle;
* the window is rho ** (Euclidean distance of (m, n, t) to the area centre
  ((M-1)/2, (N-1)/2, (T-1)/2)), in pixel and frame units alike (reading:
  the paper gives no separate temporal decay);
* every other reading of ``oracle.cfse`` holds unchanged (lowest index on
  ties, repeated selections add up, I iterations, w = 0 on B, on other lost
  pixels and outside the clip).
"""
import numpy as np

from . import cfse as c2

TIE_RTOL = c2.TIE_RTOL


def window(M, N, T, rho):
    """rho ** distance to the volume's centre, eq. (3) in three dimensions."""
    m = np.arange(M, dtype=np.float64)[:, None, None]
    n = np.arange(N, dtype=np.float64)[None, :, None]
    t = np.arange(T, dtype=np.float64)[None, None, :]
    d = np.sqrt((m - (M - 1) / 2.0) ** 2 + (n - (N - 1) / 2.0) ** 2 + (t - (T - 1) / 2.0) ** 2)
    return np.power(float(rho), d)


def area_of_volume(frames, avail, vol):
    """Cut the area of volume ``vol`` (fields frame, y0, x0, bt, bh, bw,
    border, tborder) from a clip frames[t][y][x]. Returns (s, A, B) as
    M x N x T arrays: signal (0 where unknown), support mask (received,
    inside the clip, not in B), loss mask."""
    f0, y0, x0 = int(vol["frame"]), int(vol["y0"]), int(vol["x0"])
    bt, bh, bw = int(vol["bt"]), int(vol["bh"]), int(vol["bw"])
    bd, td = int(vol["border"]), int(vol["tborder"])
    M, N, T = bh + 2 * bd, bw + 2 * bd, bt + 2 * td
    nf, H, W = frames.shape
    s = np.zeros((M, N, T))
    A = np.zeros((M, N, T), dtype=bool)
    ya, xa, ta = y0 - bd, x0 - bd, f0 - td
    for ti in range(T):
        f = ta + ti
        if not 0 <= f < nf:
            continue
        r0, r1 = max(ya, 0), min(ya + M, H)
        q0, q1 = max(xa, 0), min(xa + N, W)
        if r0 < r1 and q0 < q1:
            s[r0 - ya:r1 - ya, q0 - xa:q1 - xa, ti] = frames[f, r0:r1, q0:q1]
            A[r0 - ya:r1 - ya, q0 - xa:q1 - xa, ti] = avail[f, r0:r1, q0:q1] != 0
    B = np.zeros((M, N, T), dtype=bool)
    B[bd:bd + bh, bd:bd + bw, td:td + bt] = True
    A &= ~B
    return np.where(A, s, 0.0), A, B


def project(x, EM, EN, ET):
    """sum over L of x * phi*_(k,l,s) for every bin: eq. (7) in 3-D,
    separable over the three axes. Returns an F x F x Ft array [k, l, s]."""
    return np.einsum("km,ln,st,mnt->kls", EM, EN, ET, x, optimize=True)


def basis(F, Ft, M, N, T, k, l, s):
    """phi_(k,l,s) on the M x N x T area."""
    tF, tT = c2.twiddle_table(F), c2.twiddle_table(Ft)
    m = np.arange(M)[:, None, None]
    n = np.arange(N)[None, :, None]
    t = np.arange(T)[None, None, :]
    return np.conj(tF[(k * m) % F]) * np.conj(tF[(l * n) % F]) * np.conj(tT[(s * t) % Ft])


def cfse3(s, w, F, Ft, gamma, iters, forced=None, cand=None):
    """cFSE on one M x N x T area by direct projection (the 3-D counterpart
    of ``oracle.cfse.cfse``; same return dict, bins as linear indices
    (k F + l) Ft + s and coefficients keyed (k, l, s)). ``cand`` optionally
    restricts the argmax to a boolean F x F x Ft mask of candidate bins (a
    restriction of the dictionary; every equation unchanged)."""
    M, N, T = s.shape
    if F < M or F < N or Ft < T:
        raise ValueError("transform smaller than the area")
    EM, EN, ET = c2.analysis_matrix(F, M), c2.analysis_matrix(F, N), c2.analysis_matrix(Ft, T)
    den = project(w.astype(np.complex128), np.abs(EM) ** 2, np.abs(EN) ** 2, np.abs(ET) ** 2).real
    if not np.all(den > 0):
        raise ValueError("empty support area (sum of weights is zero)")
    g = np.zeros((M, N, T), dtype=np.complex128)
    coefs = {}
    r = s.astype(np.complex128)
    out = dict(seq=[], chat=[], free=[], short=[], gap=[], energy=[], coefs=coefs)
    out["energy"].append(float(np.sum(w * np.abs(r) ** 2)))
    for nu in range(iters):
        p = project(r * w, EM, EN, ET) / den                    # eq. (9)
        crit = np.abs(p) ** 2 * den                              # eq. (10)
        free = c2.select(crit, cand)
        idx = free if forced is None else int(forced[nu])
        mag = np.sqrt(crit)
        ref = mag.ravel()[free]
        out["free"].append(free)
        out["short"].append(float((ref - mag.ravel()[idx]) / ref) if ref > 0 else 0.0)
        live = mag if cand is None else mag[cand]
        out["gap"].append(c2.top2_gap(live) if live.size >= 2 else 1.0)
        kl, sv = divmod(idx, Ft)
        u, v = divmod(kl, F)
        c = gamma * p[u, v, sv]                                  # eq. (13)
        phi = basis(F, Ft, M, N, T, u, v, sv)
        g = g + c * phi                                          # eq. (14)
        r = r - c * phi                                          # eq. (17)
        coefs[(u, v, sv)] = coefs.get((u, v, sv), 0) + c
        out["seq"].append(idx)
        out["chat"].append(complex(c))
        out["energy"].append(float(np.sum(w * np.abs(r) ** 2)))
    out["g"] = g
    return out


def extrapolate_volume(frames, avail, vol, rho, gamma, forced=None, iters=None, cand=None):
    """cFSE for one volume descriptor; the run dict plus 'values' = Re{g} on
    B as a bh x bw x bt array, or None when the volume has no support."""
    s, A, B = area_of_volume(frames, avail, vol)
    M, N, T = s.shape
    w = np.where(A, window(M, N, T, rho), 0.0)
    if w.sum() == 0:
        return None
    I = int(vol["iters"]) if iters is None else iters
    res = cfse3(s, w, int(vol["fft"]), int(vol["fft_t"]), gamma, I, forced=forced, cand=cand)
    bd, td = int(vol["border"]), int(vol["tborder"])
    res["values"] = res["g"][bd:bd + int(vol["bh"]), bd:bd + int(vol["bw"]), td:td + int(vol["bt"])].real.copy()
    return res
