"""Plain FP64 complex-valued FSE by direct spatial projection.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product path. Shares no code with the GPU side.

What it follows (Seiler & Kaup, "Complex-Valued Frequency Selective
Extrapolation for Fast Image and Video Signal Extrapolation"):

* extrapolation area L = A u B of size M x N around a lost block
  (Section II, Fig. 1);
* weighting function w, eq. (3): rho^distance-from-area-centre on A, 0 on B;
* Fourier basis phi_(k,l), eq. (1), taken on the F x F transform grid (the
  experiments pad a 48x48 area to a 64x64 transform, Section IV);
* per iteration: residual r = s - g, eq. (8); weighted projection p, eq. (9);
  selection maximising |p|^2 * sum(phi* w phi), eq. (10); coefficient
  c = gamma * p, eq. (13); model update g += c*phi, eq. (14); residual update
  r -= c*phi, eq. (17);
* output Re{g} on B (Algorithm 1, last loop; Section III, real-valued input).

Unlike Algorithm 1 it never updates a spectrum: every iteration re-projects
the spatial residual onto all F*F basis functions with a matrix product.

Readings of the paper taken here:
* the basis lives on the F x F grid: phi_(k,l)[m,n] = exp(j2pi(k(m+a)+l(n+b))/F)
  for the area placed at offset (a, b) of the grid, default (0, 0);
* m is the row index, n the column index; the linear bin index is k*F + l;
* the argmax runs over all F*F bins; bins whose criterion is within a
  relative 1e-12 of the maximum count as tied, and ties go to the lowest
  linear index (real input makes conjugate bins tie exactly);
* a basis function may be selected again; its coefficients add up;
* I iterations are always run (no early stop);
* the window centre is ((M-1)/2, (N-1)/2) of the area; pixels outside the
  frame, lost pixels of other blocks and B itself get w = 0.
* arbitrary loss shapes (the concealment and inpainting setting the paper
  names in Section I, "masked" below): the block's rectangle only bounds
  the loss; B is the set of its pixels that were not received, received
  pixels inside the rectangle belong to the support A, and only B is
  written.
"""
import numpy as np

TIE_RTOL = 1e-12


# ---------------------------------------------------------------- geometry

def window(M, N, rho):
    """eq. (3) before masking: rho ** distance to the area centre."""
    m = np.arange(M, dtype=np.float64)[:, None]
    n = np.arange(N, dtype=np.float64)[None, :]
    dist = np.sqrt((m - (M - 1) / 2.0) ** 2 + (n - (N - 1) / 2.0) ** 2)
    return np.power(float(rho), dist)


def area_of_block(frames, avail, blk, masked=False):
    """Cut the area L of block ``blk`` (fields frame, y0, x0, bh, bw, border).

    Returns (s, A, B): the signal as float64 (0 where unknown), the support
    mask A (received, inside the frame, not in B) and the loss mask B (the
    block's rectangle, or with ``masked`` its pixels that were not
    received)."""
    f, y0, x0 = int(blk["frame"]), int(blk["y0"]), int(blk["x0"])
    bh, bw, bd = int(blk["bh"]), int(blk["bw"]), int(blk["border"])
    M, N = bh + 2 * bd, bw + 2 * bd
    H, W = frames.shape[1:]
    s = np.zeros((M, N))
    A = np.zeros((M, N), dtype=bool)
    ya, xa = y0 - bd, x0 - bd
    r0, r1 = max(ya, 0), min(ya + M, H)
    c0, c1 = max(xa, 0), min(xa + N, W)
    if r0 < r1 and c0 < c1:
        s[r0 - ya:r1 - ya, c0 - xa:c1 - xa] = frames[f, r0:r1, c0:c1]
        A[r0 - ya:r1 - ya, c0 - xa:c1 - xa] = avail[f, r0:r1, c0:c1] != 0
    B = np.zeros((M, N), dtype=bool)
    B[bd:bd + bh, bd:bd + bw] = True
    if masked:
        B &= ~A  # the rectangle lies inside the frame (a validated block)
    A &= ~B
    s = np.where(A, s, 0.0)
    return s, A, B


def weighting(M, N, rho, A):
    """eq. (3): window on the support area A, zero elsewhere."""
    return np.where(A, window(M, N, rho), 0.0)


# ---------------------------------------------------------------- basis

def twiddle_table(F):
    """t[j] = exp(-j*2*pi*j/F) with t[F-j] = conj(t[j]) and the points
    1, -j, -1, +j exact, so that real data gets exactly conjugate-symmetric
    projections."""
    j = np.arange(F)
    t = np.exp(-2j * np.pi * j / F)
    t[0] = 1.0
    if F % 2 == 0:
        t[F // 2] = -1.0
    if F % 4 == 0:
        t[F // 4] = -1j
        t[3 * F // 4] = 1j
    lo = np.arange(1, (F + 1) // 2)
    t[F - lo] = np.conj(t[lo])
    return t


def analysis_matrix(F, size, offset=0):
    """E[k, m] = phi*_k[m + offset] = exp(-j2pi k (m+offset) / F), k < F, m < size."""
    k = np.arange(F)[:, None]
    m = np.arange(size)[None, :] + offset
    return twiddle_table(F)[(k * m) % F]


def basis(F, M, N, k, l, offset=(0, 0)):
    """phi_(k,l)[m, n] on the M x N area, eq. (1) on the F x F grid."""
    t = twiddle_table(F)
    m = np.arange(M)[:, None] + offset[0]
    n = np.arange(N)[None, :] + offset[1]
    # exp(+j..) is the conjugate of the analysis table entry
    return np.conj(t[(k * m) % F]) * np.conj(t[(l * n) % F])


def project(x, EM, EN):
    """sum over L of x[m,n] * phi*_(k,l)[m,n] for every (k,l): eq. (7),
    the numerator of eq. (9) when x = r*w. Separable: EM @ x @ EN^T."""
    return EM @ x @ EN.T


# ---------------------------------------------------------------- selection

def select(crit, cand=None):
    """Lowest linear index among bins within TIE_RTOL of the largest
    criterion (eq. (10)); ``cand`` optionally restricts the bins."""
    c = crit.ravel()
    if cand is not None:
        c = np.where(cand.ravel(), c, -np.inf)
    cmax = c.max()
    idx = int(np.flatnonzero(c >= cmax * (1.0 - TIE_RTOL))[0])
    return idx


def top2_gap(mag):
    """(largest - second largest) / largest over a flat array of |R| values."""
    v = np.sort(mag.ravel())
    if v[-1] == 0:
        return 0.0
    return float((v[-1] - v[-2]) / v[-1])


# ---------------------------------------------------------------- cFSE

def cfse(s, w, F, gamma, iters, offset=(0, 0), forced=None, init=None, cand=None):
    """Run cFSE on one area by direct projection.

    s      : M x N signal (real or complex), values on B are ignored
    w      : M x N weighting, eq. (3), zero outside the support area
    F      : transform size (F >= M, N)
    forced : optional sequence of linear bin indices to follow instead of the
             free argmax (replay of another implementation's choices)
    init   : optional dict {(k, l): c} of initial coefficients (warm start)
    cand   : optional boolean F x F mask restricting the argmax

    Returns a dict with the per-iteration selections ``seq`` (linear index),
    coefficients ``chat``, free choices ``free``, the shortfall ``short`` of
    the followed bin against the largest |R| (relative), the top-two gap
    ``gap``, the weighted residual energies ``energy`` (energy[0] before the
    first iteration), the accumulated coefficients ``coefs`` {(k, l): c} and
    the complex model ``g`` on the area.
    """
    M, N = s.shape
    if F < M or F < N:
        raise ValueError("transform smaller than the area")
    EM = analysis_matrix(F, M, offset[0])
    EN = analysis_matrix(F, N, offset[1])
    # denominator of eq. (9), literally sum_L phi* w phi for every bin
    den = (np.abs(EM) ** 2) @ w @ (np.abs(EN) ** 2).T
    if not np.all(den > 0):
        raise ValueError("empty support area (sum of weights is zero)")
    g = np.zeros((M, N), dtype=np.complex128)
    coefs = {}
    if init:
        for (k, l), c in init.items():
            g += c * basis(F, M, N, k, l, offset)
            coefs[(k, l)] = coefs.get((k, l), 0) + c
    r = s.astype(np.complex128) - g                               # eq. (8)
    out = dict(seq=[], chat=[], free=[], short=[], gap=[], energy=[], coefs=coefs)
    out["energy"].append(float(np.sum(w * np.abs(r) ** 2)))
    for nu in range(iters):
        num = project(r * w, EM, EN)                             # eq. (9) numerator
        p = num / den                                            # eq. (9)
        crit = np.abs(p) ** 2 * den                              # eq. (10)
        free = select(crit, cand)
        idx = free if forced is None else int(forced[nu])
        mag = np.sqrt(crit)
        ref = mag.ravel()[free]
        out["free"].append(free)
        out["short"].append(float((ref - mag.ravel()[idx]) / ref) if ref > 0 else 0.0)
        out["gap"].append(top2_gap(mag if cand is None else np.where(cand, mag, 0.0)))
        u, v = divmod(idx, F)
        c = gamma * p[u, v]                                      # eq. (13)
        phi = basis(F, M, N, u, v, offset)
        g = g + c * phi                                          # eq. (14)
        r = r - c * phi                                          # eq. (17)
        coefs[(u, v)] = coefs.get((u, v), 0) + c
        out["seq"].append(idx)
        out["chat"].append(complex(c))
        out["energy"].append(float(np.sum(w * np.abs(r) ** 2)))
    out["g"] = g
    return out


def extrapolate_block(frames, avail, blk, rho, gamma, forced=None, init=None, cand=None,
                      iters=None, masked=False):
    """cFSE for one block descriptor; returns the run dict plus 'values' =
    Re{g} on the block's rectangle as a bh x bw float64 array (Algorithm 1,
    last loop) and 'lost' = B on the rectangle, or None for the run when the
    block has no support."""
    s, A, B = area_of_block(frames, avail, blk, masked)
    M, N = s.shape
    w = weighting(M, N, rho, A)
    F = int(blk["fft"])
    I = int(blk["iters"]) if iters is None else iters
    if w.sum() == 0:
        return None
    res = cfse(s, w, F, gamma, I, forced=forced, init=init, cand=cand)
    bd, bh, bw = int(blk["border"]), int(blk["bh"]), int(blk["bw"])
    res["values"] = res["g"][bd:bd + bh, bd:bd + bw].real.copy()
    res["lost"] = B[bd:bd + bh, bd:bd + bw].copy()
    return res


_SHARED = {}


def _one_blas_thread():
    """Worker processes use one BLAS thread each (the matrices are small)."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _block_worker(i):
    frames, avail, blocks, rho, gamma, masked = _SHARED["job"]
    res = extrapolate_block(frames, avail, blocks[i], rho, gamma, masked=masked)
    return None if res is None else (res["values"], res["lost"])


def extrapolate_frames(frames, avail, blocks, rho, gamma, processes=1, masked=False):
    """Conceal every block of ``blocks`` (a BLOCK_DTYPE array): returns a
    float64 copy of the distorted frames with each B replaced by Re{g}
    (with ``masked``, B = the lost pixels of each block's rectangle).
    Blocks whose area has no support keep the distorted value (0)."""
    out = (frames * (avail != 0)).astype(np.float64)
    _SHARED["job"] = (frames, avail, blocks, rho, gamma, masked)
    try:
        if processes > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(processes, initializer=_one_blas_thread) as pool:
                vals = pool.map(_block_worker, range(len(blocks)),
                                chunksize=max(1, len(blocks) // (4 * processes)))
        else:
            vals = [_block_worker(i) for i in range(len(blocks))]
    finally:
        _SHARED.clear()
    for b, v in zip(blocks, vals):
        if v is not None:
            f, y0, x0 = int(b["frame"]), int(b["y0"]), int(b["x0"])
            sub = out[f, y0:y0 + int(b["bh"]), x0:x0 + int(b["bw"])]
            sub[v[1]] = v[0][v[1]]
    return out
