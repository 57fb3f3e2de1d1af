"""Plain FP64 real-valued FSE (rFSE), the algorithm cFSE is compared with.

TEST INFRASTRUCTURE ONLY: used by tests/ and the benchmark's CPU-baseline
leg; never by the product path. Shares no code with the GPU side.

The paper defines rFSE by its model, eq. (2): every iteration adds one
Fourier basis function together with its complex conjugate,
g += (c phi* + c* phi) / 2 = Re{c phi*}, so the model stays real; it names
the weighting of eq. (3), the I iterations and the special treatment of the
real-valued basis functions (constant and highest alternating frequency),
and leaves the selection and estimation rules to its reference [Kaup2005],
which is not available. This module derives them from eq. (2) alone
(reading R19):

* a pair (k, l) / (-k, -l) is fitted to the weighted residual by weighted
  least squares over the real span {Re phi*, Im phi*} (two real unknowns;
  one for the four self-conjugate bins with 2k = 2l = 0 mod F, whose basis
  function is real);
* the pair with the largest decrease of the weighted residual energy is
  selected (lowest linear index on ties, so the selected member is the
  pair's lower-index bin);
* its coefficient is scaled by gamma (the compensation of eq. (13)) and
  the real model is subtracted from the residual in the spatial domain.

Two selection rules are implemented (``selection``):
* "decrease" (the kept reading): the pair with the largest decrease of the
  weighted residual energy under its least-squares fit (per-bin divisions,
  the cost Section II attributes to rFSE's selection);
* "power" (the other reading): the pair holding the bin of largest
  |R_w[k,l]|^2, the criterion of eq. (12), with the same least-squares
  estimate. Neither reproduces Section IV's "rFSE slightly above cFSE" on
  the synthetic frames at the paper's gamma = 0.2 (both are 0.1-0.7 dB
  below cFSE at equal numbers of basis functions); "decrease" is closer
  there.

Closed forms (P = R_w[k,l] = sum w r phi*, W0 = sum w, Q = W[2k, 2l] =
sum w phi*^2, D = W0^2 - |Q|^2):
  c = 2 (W0 P* - Q* P) / D,  decrease = Re{c P} = 2 (W0 |P|^2 - Re{Q* P^2}) / D;
  self-conjugate bins: c = P / W0 (real), decrease = P^2 / W0.
They are pinned against a brute-force weighted least-squares fit. Whether
they are [Kaup2005]'s rules cannot be checked here: parity unpinned
against the paper's rFSE (no numbers of it are available).
"""
import numpy as np

from . import cfse as c2

TIE_RTOL = c2.TIE_RTOL


def self_conjugate(F):
    """F x F mask of the bins with (2k, 2l) = (0, 0) mod F."""
    k = np.arange(F)
    s = (2 * k) % F == 0
    return s[:, None] & s[None, :]


def pair_index(F, idx):
    """Linear index of the conjugate partner (-k, -l) of bin idx = k F + l."""
    k, l = divmod(int(idx), F)
    return ((-k) % F) * F + ((-l) % F)


def double_freq(Wf):
    """Q[k, l] = W[2k mod F, 2l mod F] for an F x F spectrum W."""
    F = Wf.shape[0]
    d = (2 * np.arange(F)) % F
    return Wf[np.ix_(d, d)]


def pair_fit(P, W0, Q, sc):
    """Closed-form weighted least-squares fit of every pair: coefficient c
    and energy decrease, arrays over the F x F bins (sc: self-conjugate
    mask)."""
    D = W0 * W0 - np.abs(Q) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.where(sc, P.real / W0, 2.0 * (W0 * np.conj(P) - np.conj(Q) * P) / D)
        dec = np.where(sc, P.real ** 2 / W0, 2.0 * (W0 * np.abs(P) ** 2 - (np.conj(Q) * P * P).real) / D)
    return c, dec


def rfse(s, w, F, gamma, iters, offset=(0, 0), forced=None, selection="decrease"):
    """rFSE on one M x N area (s: signal, 0 where unknown; w: eq. (3)
    weights). Returns dict(seq, chat, free, short, gap, energy, coefs, g):
    seq the selected lower-index bins, chat their coefficients c (model
    increment Re{c phi*}), g the real model on the area. ``selection``:
    "power" (largest |R_w|^2) or "decrease" (largest least-squares energy
    decrease, the default); short and gap are in |R_w| or in decrease
    accordingly."""
    if selection not in ("power", "decrease"):
        raise ValueError("selection must be 'power' or 'decrease'")
    M, N = s.shape
    if F < M or F < N:
        raise ValueError("transform smaller than the area")
    EM, EN = c2.analysis_matrix(F, M, offset[0]), c2.analysis_matrix(F, N, offset[1])
    W0 = float(w.sum())
    if not W0 > 0:
        raise ValueError("empty support area (sum of weights is zero)")
    Q = double_freq(c2.project(w.astype(np.complex128), EM, EN))
    sc = self_conjugate(F)
    r = s.astype(np.float64).copy()
    g = np.zeros((M, N))
    coefs = {}
    out = dict(seq=[], chat=[], free=[], short=[], gap=[], energy=[], coefs=coefs)
    out["energy"].append(float(np.sum(w * r * r)))
    for nu in range(iters):
        P = c2.project((w * r).astype(np.complex128), EM, EN)     # R_w, eq. (7)
        c, dec = pair_fit(P, W0, Q, sc)
        dec = np.maximum(dec.real, 0.0)
        if selection == "power":
            free = c2.select(np.abs(P) ** 2)
            crit = np.abs(P)
        else:
            free = c2.select(dec)
            crit = dec
        idx = free if forced is None else int(forced[nu])
        ref = crit.ravel()[free]
        out["free"].append(free)
        out["short"].append(float((ref - crit.ravel()[idx]) / ref) if ref > 0 else 0.0)
        # the partner of the best bin has the same criterion: the gap is to
        # the best bin of another pair
        others = crit.ravel().copy()
        others[[free, pair_index(F, free)]] = -1.0
        out["gap"].append(float((ref - others.max()) / ref) if ref > 0 else 0.0)
        u, vv = divmod(idx, F)
        ch = gamma * c[u, vv]                                      # compensation, eq. (13)
        inc = (ch * np.conj(c2.basis(F, M, N, u, vv, offset))).real  # Re{c phi*}, eq. (2)
        g = g + inc
        r = r - inc
        coefs[(u, vv)] = coefs.get((u, vv), 0) + ch
        out["seq"].append(idx)
        out["chat"].append(complex(ch))
        out["energy"].append(float(np.sum(w * r * r)))
    out["g"] = g
    return out


def extrapolate_block(frames, avail, blk, rho, gamma, forced=None, iters=None, selection="decrease"):
    """rFSE for one block descriptor; the run dict plus 'values' = g on
    the block's rectangle, or None when the block has no support."""
    s, A, B = c2.area_of_block(frames, avail, blk)
    M, N = s.shape
    w = c2.weighting(M, N, rho, A)
    if w.sum() == 0:
        return None
    I = int(blk["iters"]) if iters is None else iters
    res = rfse(s, w, int(blk["fft"]), gamma, I, forced=forced, selection=selection)
    bd, bh, bw = int(blk["border"]), int(blk["bh"]), int(blk["bw"])
    res["values"] = res["g"][bd:bd + bh, bd:bd + bw].copy()
    return res
