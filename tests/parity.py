"""GPU-versus-oracle comparison (test helper; imports the oracle, never the
other way round).

Replay protocol for one block, given the GPU's trace of selections and
coefficients:
1. the FP64 oracle is run forced along the GPU's selections; at every
   iteration the GPU's bin must be the oracle's own free choice, or lie within
   a relative 1e-6 of the largest |R_w| (a near tie that FP32 may break
   either way);
2. the accumulated coefficients per distinct bin must agree: for every bin
   |c_gpu - c_orc| <= 1e-4 * max|c_orc|, and ||dc||_2 <= 1e-4 * ||c_orc||_2;
3. the GPU's pixels on B must lie within 0.05 of the forced oracle's model
   (Re{g} along the same selections: FP32 rounding only);
4. frame PSNR over the lost pixels, GPU output vs the free-running oracle's
   output, each against the undistorted frame, must differ by <= 0.01 dB.
"""
import numpy as np

from oracle import cfse, metrics

GAP_TOL = 1e-6
COEF_TOL = 1e-4
PSNR_TOL = 0.01
PIX_TOL = 0.05


def gpu_sequence(trace_row, F, I):
    rec = trace_row[:I]
    seq = rec["u"].astype(np.int64) * F + rec["v"].astype(np.int64)
    c = rec["c_re"].astype(np.float64) + 1j * rec["c_im"].astype(np.float64)
    return seq, c


def accumulate(seq, c):
    acc = {}
    for s, v in zip(seq, c):
        acc[int(s)] = acc.get(int(s), 0) + v
    return acc


def replay_block(frames, avail, blk, rho, gamma, trace_row, masked=False):
    """Returns a dict of per-block parity figures (raises nothing)."""
    F, I = int(blk["fft"]), int(blk["iters"])
    seq, c = gpu_sequence(trace_row, F, I)
    res = cfse.extrapolate_block(frames, avail, blk, rho, gamma, forced=seq, masked=masked)
    short = np.array(res["short"]) if I else np.zeros(0)
    free = np.array(res["free"]) if I else np.zeros(0, dtype=int)
    diverged = free != seq
    bad_gap = diverged & (short >= GAP_TOL)
    ag = accumulate(seq, c)
    ao = accumulate(seq, np.array(res["chat"]))
    keys = sorted(ao)
    vo = np.array([ao[k] for k in keys])
    vg = np.array([ag.get(k, 0) for k in keys])
    scale = np.abs(vo).max() if len(vo) else 0.0
    d = np.abs(vg - vo)
    return dict(
        ties=int(diverged.sum()), gap_violations=int(bad_gap.sum()),
        max_short=float(short[diverged].max()) if diverged.any() else 0.0,
        coef_max=float(d.max() / scale) if scale > 0 else 0.0,
        coef_l2=float(np.linalg.norm(vg - vo) / np.linalg.norm(vo)) if scale > 0 else 0.0,
        values=res["values"], lost=res["lost"])


def check_blocks(frames, avail, blocks, rho, gamma, trace, out_gpu, idx=None, masked=False):
    """Replay every block in ``idx`` (default all); assert the per-block bars
    and return the per-block figures (pixel differences over the block's
    loss area)."""
    idx = range(len(blocks)) if idx is None else idx
    rows = []
    for i in idx:
        blk = blocks[i]
        r = replay_block(frames, avail, blk, rho, gamma, trace[i], masked)
        f, y0, x0 = int(blk["frame"]), int(blk["y0"]), int(blk["x0"])
        g = out_gpu[f, y0:y0 + int(blk["bh"]), x0:x0 + int(blk["bw"])].astype(np.float64)
        r["pix_maxabs"] = float(np.abs(g - r["values"])[r["lost"]].max())
        r["index"] = int(i)
        rows.append(r)
        assert r["gap_violations"] == 0, (i, r)
        assert r["coef_max"] <= COEF_TOL and r["coef_l2"] <= COEF_TOL, (i, r)
        assert r["pix_maxabs"] < PIX_TOL, (i, r["pix_maxabs"])
    return rows


def psnr_delta(frames, avail, blocks, rho, gamma, out_gpu, processes=1, masked=False):
    """|PSNR(GPU) - PSNR(free-running oracle)| over the lost pixels of the
    given blocks (other lost pixels are ignored), plus both PSNRs."""
    ref = cfse.extrapolate_frames(frames, avail, blocks, rho, gamma, processes=processes, masked=masked)
    mask = np.ones_like(avail)
    for b in blocks:
        sl = (int(b["frame"]), slice(int(b["y0"]), int(b["y0"]) + int(b["bh"])),
              slice(int(b["x0"]), int(b["x0"]) + int(b["bw"])))
        mask[sl] = avail[sl] if masked else 0
    p_gpu = metrics.psnr_lost(frames, out_gpu, mask)
    p_orc = metrics.psnr_lost(frames, ref, mask)
    return abs(p_gpu - p_orc), p_gpu, p_orc, metrics.psnr_between(out_gpu, ref, mask)


def _restricted_worker(args):
    frames, avail, blk, rho, gamma, cand_bins, ir = args
    F = int(blk["fft"])
    cand = np.zeros(F * F, dtype=bool)
    cand[np.asarray(cand_bins, dtype=np.int64)] = True
    res = cfse.extrapolate_block(frames, avail, blk, rho, gamma, cand=cand.reshape(F, F), iters=ir)
    return res["values"]


def warm_psnr_delta(frames, avail, blocks, cands, rho, gamma, ir, out_gpu, processes=1):
    """Restricted-only warm start: |PSNR(GPU) - PSNR(oracle)| over the lost
    pixels of the given blocks, the oracle running free over each block's
    candidate bins for ``ir`` iterations; returns (delta, gpu, oracle)."""
    jobs = []
    for b, c in zip(blocks, cands):
        b = b.copy()
        f = int(b["frame"])
        b["frame"] = 0
        jobs.append((frames[f:f + 1], avail[f:f + 1], b, rho, gamma, c, ir))
    if processes > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(processes) as pool:
            vals = pool.map(_restricted_worker, jobs, chunksize=1)
    else:
        vals = [_restricted_worker(j) for j in jobs]
    ref, rec_gpu, rec_orc = [], [], []
    for b, v in zip(blocks, vals):
        f, y0, x0 = int(b["frame"]), int(b["y0"]), int(b["x0"])
        sl = (f, slice(y0, y0 + int(b["bh"])), slice(x0, x0 + int(b["bw"])))
        ref.append(frames[sl].astype(np.float64).ravel())
        rec_gpu.append(out_gpu[sl].astype(np.float64).ravel())
        rec_orc.append(v.ravel())
    ref, rec_gpu, rec_orc = np.concatenate(ref), np.concatenate(rec_gpu), np.concatenate(rec_orc)
    lost = np.zeros(ref.shape, dtype=np.uint8)
    p_gpu = metrics.psnr_lost(ref, rec_gpu, lost)
    p_orc = metrics.psnr_lost(ref, rec_orc, lost)
    return abs(p_gpu - p_orc), p_gpu, p_orc


def replay_warm_block(frames, avail, blk, rho, gamma, trace_row, cand_bins, ir, iters, gamma_r=None):
    """Warm-started block: the restricted phase (step gamma_r, default gamma)
    is replayed with the argmax limited to the candidate bins, then the full
    phase from the oracle's own restricted model. Returns the same figures as
    replay_block, per phase."""
    F = int(blk["fft"])
    s, A, B = cfse.area_of_block(frames, avail, blk)
    w = cfse.weighting(*s.shape, rho, A)
    cand = np.zeros(F * F, dtype=bool)
    cand[np.asarray(cand_bins, dtype=np.int64)] = True
    cand = cand.reshape(F, F)
    out = {}
    seq_r, c_r = gpu_sequence(trace_row, F, ir)
    r1 = cfse.cfse(s, w, F, gamma if gamma_r is None else gamma_r, ir, forced=seq_r, cand=cand)
    seq_f, c_f = gpu_sequence(trace_row[ir:], F, iters)
    r2 = cfse.cfse(s, w, F, gamma, iters, forced=seq_f, init=dict(r1["coefs"]))
    for name, seq, c, res in (("restricted", seq_r, c_r, r1), ("full", seq_f, c_f, r2)):
        n = len(seq)
        short = np.array(res["short"]) if n else np.zeros(0)
        free = np.array(res["free"]) if n else np.zeros(0, dtype=int)
        div = free != seq
        ag, ao = accumulate(seq, c), accumulate(seq, np.array(res["chat"]))
        keys = sorted(ao)
        vo = np.array([ao[k] for k in keys])
        vg = np.array([ag.get(k, 0) for k in keys])
        scale = np.abs(vo).max() if len(vo) else 0.0
        out[name] = dict(ties=int(div.sum()), gap_violations=int((div & (short >= GAP_TOL)).sum()),
                         coef_max=float(np.abs(vg - vo).max() / scale) if scale > 0 else 0.0,
                         coef_l2=float(np.linalg.norm(vg - vo) / np.linalg.norm(vo)) if scale > 0 else 0.0)
    bd, bh, bw = int(blk["border"]), int(blk["bh"]), int(blk["bw"])
    out["values"] = r2["g"][bd:bd + bh, bd:bd + bw].real.copy()
    return out


def volume_candidates(cand_row, F=64, Ft=8):
    """The warm-started 3-D candidate mask: the given columns k F + l with
    every s."""
    cols = np.zeros(F * F, dtype=bool)
    cols[np.asarray(cand_row, dtype=np.int64)] = True
    return np.repeat(cols.reshape(F, F)[:, :, None], Ft, axis=2)


def replay_volume(frames, avail, vol, rho, gamma, trace_row, cand=None):
    """3-D counterpart of replay_block: the trace's (u, v) are (k, l Ft + s),
    so the linear bin (k F + l) Ft + s is u F Ft + v. ``cand``: the
    candidate mask of a warm-started volume."""
    from oracle import cfse3
    F, Ft, I = int(vol["fft"]), int(vol["fft_t"]), int(vol["iters"])
    rec = trace_row[:I]
    seq = rec["u"].astype(np.int64) * (F * Ft) + rec["v"].astype(np.int64)
    c = rec["c_re"].astype(np.float64) + 1j * rec["c_im"].astype(np.float64)
    res = cfse3.extrapolate_volume(frames, avail, vol, rho, gamma, forced=seq, cand=cand)
    short = np.array(res["short"]) if I else np.zeros(0)
    free = np.array(res["free"]) if I else np.zeros(0, dtype=int)
    div = free != seq
    ag, ao = accumulate(seq, c), accumulate(seq, np.array(res["chat"]))
    keys = sorted(ao)
    vo = np.array([ao[k] for k in keys])
    vg = np.array([ag.get(k, 0) for k in keys])
    scale = np.abs(vo).max() if len(vo) else 0.0
    return dict(ties=int(div.sum()), gap_violations=int((div & (short >= GAP_TOL)).sum()),
                max_short=float(short[div].max()) if div.any() else 0.0,
                coef_max=float(np.abs(vg - vo).max() / scale) if scale > 0 else 0.0,
                coef_l2=float(np.linalg.norm(vg - vo) / np.linalg.norm(vo)) if scale > 0 else 0.0,
                values=res["values"])


def volume_slices(vol):
    """(frames, rows, cols) slices of a volume's lost voxels."""
    f, y, x = int(vol["frame"]), int(vol["y0"]), int(vol["x0"])
    return (slice(f, f + int(vol["bt"])), slice(y, y + int(vol["bh"])), slice(x, x + int(vol["bw"])))


def replay_real_block(frames, avail, blk, rho, gamma, trace_row, selection="decrease"):
    """rFSE counterpart of replay_block: the trace names each selected
    pair by its lower-index bin and that bin's coefficient, as the oracle
    does; ``selection`` is the oracle's selection reading."""
    from oracle import rfse
    F, I = int(blk["fft"]), int(blk["iters"])
    seq, c = gpu_sequence(trace_row, F, I)
    res = rfse.extrapolate_block(frames, avail, blk, rho, gamma, forced=seq, selection=selection)
    short = np.array(res["short"]) if I else np.zeros(0)
    free = np.array(res["free"]) if I else np.zeros(0, dtype=int)
    div = free != seq
    ag, ao = accumulate(seq, c), accumulate(seq, np.array(res["chat"]))
    keys = sorted(ao)
    vo = np.array([ao[k] for k in keys])
    vg = np.array([ag.get(k, 0) for k in keys])
    scale = np.abs(vo).max() if len(vo) else 0.0
    return dict(ties=int(div.sum()), gap_violations=int((div & (short >= GAP_TOL)).sum()),
                max_short=float(short[div].max()) if div.any() else 0.0,
                coef_max=float(np.abs(vg - vo).max() / scale) if scale > 0 else 0.0,
                coef_l2=float(np.linalg.norm(vg - vo) / np.linalg.norm(vo)) if scale > 0 else 0.0,
                values=res["values"])
