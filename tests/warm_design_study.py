"""FP64 study behind the warm start's design (not a test: run it by name).

    python tests/warm_design_study.py [--blocks 240] [--processes 8]

Uses the oracle's frequency-domain form and the oracle network (FP64) with
the packaged weights, on a seeded sample of the isolated 16x16 losses of
one 1080p frame (seed 99), and prints frame PSNR over the sampled blocks'
lost pixels for:

  plain-100           plain FSE, 100 iterations (the reference);
  plain-25            plain FSE, 25 iterations;
  ideal32+{0,25}      the design the workload description names (a network
                      proposing 32 first coefficients, then 25 iterations),
                      with the best possible proposal: plain-100's own 32
                      largest accumulated coefficients;
  ls{N}+{ir}          first coefficients from a weighted least-squares fit
                      over the network's top-N bins (normal equations with
                      the window spectrum as Gram matrix), then ir restricted
                      iterations over its top-256; with the condition number
                      of the Gram matrix;
  ls{N}r{lam}+{ir}    the same with a ridge term lam * W0 on the diagonal;
  step{g}+{ir}        no fitted start: ir restricted iterations over the
                      network's top-256 with step g (the library's warm start).
"""
import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import cfse, cnn, metrics, spectral  # noqa: E402
from synth import workloads  # noqa: E402

F = 64
WEIGHTS = os.path.join(ROOT, "paper_2204_14193_amd", "weights", "warm_cnn.npz")
_JOB = {}


def _patch(s, A):
    mu = s[A].mean()
    x = np.zeros((48, 48, 2))
    x[:, :, 0] = np.where(A, (s - mu) / 64.0, 0.0)
    x[:, :, 1] = A
    return x


def _shift_update(st, b, c):
    u, v = divmod(int(b), F)
    st.residual -= c * st.window[np.ix_((np.arange(F) - u) % F, (np.arange(F) - v) % F)]
    st.terms.append((int(b), complex(c)))


def _restricted(st, cand, iters):
    flat = cand.ravel()
    for _ in range(iters):
        p = np.where(flat, (st.residual.real ** 2 + st.residual.imag ** 2).ravel(), -1.0)
        st.advance(int(np.flatnonzero(p >= p.max() * (1 - 1e-12))[0]))


def _block(i):
    wl, P = _JOB["wl"], _JOB["P"]
    blk = wl.blocks[i]
    s, A, B = cfse.area_of_block(wl.frames, wl.avail, blk)
    w = cfse.weighting(*s.shape, wl.rho, A)
    lg, _ = cnn.forward(P, _patch(s, A)[None])
    order = np.lexsort((np.arange(F * F), -lg[0]))
    cand = np.zeros(F * F, bool)
    cand[order[:256]] = True
    cand = cand.reshape(F, F)
    out, cond = {}, {}
    bo = slice(16, 32)

    st = spectral.SpectralState(s, w, F, wl.gamma)
    for _ in range(100):
        st.advance()
    out["plain-100"] = st.model().real[bo, bo]
    acc = {}
    for b, c in st.terms:
        acc[b] = acc.get(b, 0) + c
    st = spectral.SpectralState(s, w, F, wl.gamma)
    for _ in range(25):
        st.advance()
    out["plain-25"] = st.model().real[bo, bo]
    top = sorted(acc.items(), key=lambda kv: -abs(kv[1]))[:32]
    for it in (0, 25):
        st = spectral.SpectralState(s, w, F, wl.gamma)
        for b, c in top:
            _shift_update(st, b, c)
        for _ in range(it):
            st.advance()
        out[f"ideal32+{it}"] = st.model().real[bo, bo]

    for N in (32, 48):
        bins = order[:N]
        u, v = bins // F, bins % F
        for lam in (0.0, 0.003, 0.01):
            st0 = spectral.SpectralState(s, w, F, wl.gamma)
            G = st0.window[(u[:, None] - u[None, :]) % F, (v[:, None] - v[None, :]) % F]
            G = G + lam * st0.window[0, 0].real * np.eye(N)
            c = np.linalg.solve(G, st0.residual[u, v])
            name = f"ls{N}" if lam == 0 else f"ls{N}r{lam}"
            cond[name] = float(np.linalg.cond(G))
            for ir in (0, 25):
                st = spectral.SpectralState(s, w, F, wl.gamma)
                for b, cc in zip(bins, c):
                    _shift_update(st, b, cc)
                _restricted(st, cand, ir)
                out[f"{name}+{ir}"] = st.model().real[bo, bo]

    for g in (0.5, 1.0):
        st = spectral.SpectralState(s, w, F, g)
        done = 0
        for ir in (40, 60, 110):
            _restricted(st, cand, ir - done)
            done = ir
            out[f"step{g}+{ir}"] = st.model().real[bo, bo]
    return i, out, cond


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--blocks", type=int, default=240)
    ap.add_argument("--processes", type=int, default=8)
    args = ap.parse_args()
    wl = workloads.random_1080p_16x16(seeds=(99,), iters=100)
    with np.load(WEIGHTS, allow_pickle=False) as z:
        P = cnn.unflatten(z["params"].astype(np.float64))
    _JOB.update(wl=wl, P=P)
    idx = np.sort(np.random.default_rng(3).choice(len(wl.blocks), args.blocks, replace=False))
    t0 = time.time()
    with mp.get_context("fork").Pool(args.processes) as pool:
        res = pool.map(_block, idx, chunksize=4)
    ref = np.concatenate([wl.frames[0, wl.blocks[i]["y0"]:wl.blocks[i]["y0"] + 16,
                                    wl.blocks[i]["x0"]:wl.blocks[i]["x0"] + 16].ravel() for i, _, _ in res])
    zero = np.zeros_like(ref)
    base = None
    print(f"{len(res)} blocks of frame 99 (isolated 16x16 losses, border 16, F = 64, rho 0.8, gamma 0.5)")
    for k in res[0][1]:
        rec = np.concatenate([o[k].ravel() for _, o, _ in res])
        p = metrics.psnr_lost(ref, rec, zero)
        base = p if base is None else base
        worst = max(10 * np.log10(np.mean((np.clip(o[k], 0, 255) - ref_b) ** 2) /
                                  np.mean((np.clip(o["plain-100"], 0, 255) - ref_b) ** 2))
                    for (i, o, _), ref_b in zip(res, [wl.frames[0, wl.blocks[i]["y0"]:wl.blocks[i]["y0"] + 16,
                                                                wl.blocks[i]["x0"]:wl.blocks[i]["x0"] + 16]
                                                      .astype(float) for i, _, _ in res]))
        print(f"  {k:16s} {p:7.3f} dB  ({p - base:+.3f} vs plain-100, worst block {worst:+.2f} dB MSE)")
    for k in res[0][2]:
        c = np.array([r[2][k] for r in res])
        print(f"  cond {k:10s} median {np.median(c):.3g}  max {c.max():.3g}")
    print(f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
