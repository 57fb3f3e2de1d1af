"""Seeded block-loss patterns and the per-block descriptors handed to FSE.

A lost block ``B`` is a ``bh x bw`` rectangle at ``(y0, x0)`` of frame
``frame``; its extrapolation area is ``B`` grown by ``border`` pixels on every
side (Section II, Fig. 1 of the paper: loss area B, support area A, together
the area L of size M x N). Each descriptor also carries the transform size
``fft`` and the iteration count ``iters`` used for that block.

The availability mask is ``uint8`` with 1 = received and 0 = lost.
Loss-pattern random numbers come from ``default_rng(seed + 10**6)`` so that
the image and its loss pattern can share one seed without sharing a stream.
"""
from dataclasses import dataclass
import math

import numpy as np

#: Memory layout of one block descriptor, identical to ``fse_block_t`` in
#: ``include/fse.h`` (24 bytes, naturally aligned).
BLOCK_DTYPE = np.dtype([("frame", "<i4"), ("y0", "<i4"), ("x0", "<i4"),
                        ("bh", "<i2"), ("bw", "<i2"), ("border", "<i2"),
                        ("fft", "<i2"), ("iters", "<i4")])
assert BLOCK_DTYPE.itemsize == 24

#: Layout of one lost volume of a clip (three dimensions), identical to
#: ``fse_volume_t`` in ``include/fse.h`` (32 bytes): B is bh x bw pixels of
#: frames frame .. frame + bt - 1; its area grows it by ``border`` pixels and
#: ``tborder`` frames on every side; fft x fft x fft_t transform.
VOLUME_DTYPE = np.dtype([("frame", "<i4"), ("y0", "<i4"), ("x0", "<i4"),
                         ("bt", "<i2"), ("bh", "<i2"), ("bw", "<i2"), ("border", "<i2"),
                         ("tborder", "<i2"), ("fft", "<i2"), ("fft_t", "<i2"), ("pad", "<i2"),
                         ("iters", "<i4")])
assert VOLUME_DTYPE.itemsize == 32

FFT_SIZES = (32, 64, 128)
LOSS_SEED_OFFSET = 10 ** 6


@dataclass(frozen=True)
class Block:
    frame: int
    y0: int
    x0: int
    bh: int
    bw: int
    border: int
    fft: int
    iters: int

    @property
    def M(self):
        return self.bh + 2 * self.border

    @property
    def N(self):
        return self.bw + 2 * self.border


def blocks_to_array(blocks):
    """List of :class:`Block` -> structured array of ``BLOCK_DTYPE``."""
    arr = np.zeros(len(blocks), dtype=BLOCK_DTYPE)
    for i, b in enumerate(blocks):
        arr[i] = (b.frame, b.y0, b.x0, b.bh, b.bw, b.border, b.fft, b.iters)
    return arr


def array_to_blocks(arr):
    return [Block(*(int(v) for v in rec)) for rec in arr]


def fft_size_for_area(M, N):
    """Smallest F in {32, 64, 128} with F >= ceil(4*max(M,N)/3).

    The paper pads a 48x48 area to a 64x64 transform (Section IV); this rule
    keeps that ratio for other area sizes."""
    need = math.ceil(4 * max(M, N) / 3)
    for F in FFT_SIZES:
        if F >= need:
            return F
    raise ValueError(f"area {M}x{N} needs a transform larger than {FFT_SIZES[-1]}")


def isolated_grid_losses(height, width, bs, border, fft, iters, frame=0):
    """Every other ``bs x bs`` block in both directions, starting at block
    index (1, 1): each lost block has all 8 neighbours intact."""
    blocks = []
    for by in range(1, height // bs, 2):
        for bx in range(1, width // bs, 2):
            blocks.append(Block(frame, by * bs, bx * bs, bs, bs, border, fft, iters))
    return blocks


def random_grid_losses(height, width, bs, frac, seed, border, fft, iters, frame=0):
    """Exactly ``round(frac * cells)`` cells of the ``bs`` grid, no two of
    them 8-neighbours, drawn by seeded rejection sampling."""
    rng = np.random.default_rng(seed + LOSS_SEED_OFFSET)
    gh, gw = height // bs, width // bs
    want = int(round(frac * gh * gw))
    taken = np.zeros((gh + 2, gw + 2), dtype=bool)  # one-cell guard ring
    chosen = []
    for cell in rng.permutation(gh * gw):
        cy, cx = divmod(int(cell), gw)
        if taken[cy:cy + 3, cx:cx + 3].any():
            continue
        taken[cy + 1, cx + 1] = True
        chosen.append((cy, cx))
        if len(chosen) == want:
            break
    if len(chosen) != want:
        raise RuntimeError(f"could only place {len(chosen)} of {want} non-adjacent blocks")
    chosen.sort()
    return [Block(frame, cy * bs, cx * bs, bs, bs, border, fft, iters) for cy, cx in chosen]


def mixed_size_losses(height, width, seed, frame=0, sizes=(4, 8, 16, 32), per_size=305,
                      border_range=(8, 16), iter_choices=(50, 100, 200, 500)):
    """``per_size`` square blocks of each size at uniform positions, no two
    blocks overlapping or closer than 1 pixel; border ~ U{border_range},
    transform size by :func:`fft_size_for_area`, iterations drawn from
    ``iter_choices``. Larger blocks are placed first."""
    rng = np.random.default_rng(seed + LOSS_SEED_OFFSET)
    occ = np.zeros((height, width), dtype=bool)
    blocks = []
    for bs in sorted(sizes, reverse=True):
        placed = 0
        tries = 0
        while placed < per_size:
            tries += 1
            if tries > 10000 * per_size:
                raise RuntimeError("could not place blocks")
            y0 = int(rng.integers(0, height - bs + 1))
            x0 = int(rng.integers(0, width - bs + 1))
            ya, yb = max(y0 - 1, 0), min(y0 + bs + 1, height)
            xa, xb = max(x0 - 1, 0), min(x0 + bs + 1, width)
            if occ[ya:yb, xa:xb].any():
                continue
            occ[y0:y0 + bs, x0:x0 + bs] = True
            border = int(rng.integers(border_range[0], border_range[1] + 1))
            iters = int(iter_choices[int(rng.integers(0, len(iter_choices)))])
            M = bs + 2 * border
            blocks.append(Block(frame, y0, x0, bs, bs, border, fft_size_for_area(M, M), iters))
            placed += 1
    return blocks


def availability_mask(shape, blocks):
    """``uint8`` mask of shape ``(frames, H, W)``: 0 inside every block, else 1."""
    avail = np.ones(shape, dtype=np.uint8)
    for b in blocks:
        avail[b.frame, b.y0:b.y0 + b.bh, b.x0:b.x0 + b.bw] = 0
    return avail


def stroke_mask(height, width, seed, density=0.06, width_range=(2, 7), frame_count=1):
    """Irregular losses (inpainting-like scribbles): random polyline strokes
    of random width until ``density`` of the pixels are lost. Returns a
    ``uint8`` availability mask ``(frame_count, H, W)`` (1 = received)."""
    rng = np.random.default_rng(seed + LOSS_SEED_OFFSET)
    avail = np.ones((frame_count, height, width), dtype=np.uint8)
    yy, xx = np.mgrid[0:height, 0:width]
    for f in range(frame_count):
        lost = np.zeros((height, width), dtype=bool)
        while lost.mean() < density:
            y, x = rng.uniform(0, height), rng.uniform(0, width)
            r = rng.uniform(width_range[0], width_range[1]) / 2
            for _ in range(int(rng.integers(3, 9))):
                ang = rng.uniform(0, 2 * np.pi)
                ln = rng.uniform(10, 60)
                y1 = min(max(y + ln * np.sin(ang), 0), height - 1)
                x1 = min(max(x + ln * np.cos(ang), 0), width - 1)
                # pixels within r of the segment (y, x) -> (y1, x1), in its bounding box
                ya, yb = int(max(min(y, y1) - r - 1, 0)), int(min(max(y, y1) + r + 2, height))
                xa, xb = int(max(min(x, x1) - r - 1, 0)), int(min(max(x, x1) + r + 2, width))
                py, px = yy[ya:yb, xa:xb], xx[ya:yb, xa:xb]
                dy, dx = y1 - y, x1 - x
                t = np.clip(((py - y) * dy + (px - x) * dx) / max(dy * dy + dx * dx, 1e-9), 0, 1)
                d2 = (py - (y + t * dy)) ** 2 + (px - (x + t * dx)) ** 2
                lost[ya:yb, xa:xb] |= d2 <= r * r
                y, x = y1, x1
        avail[f][lost] = 0
    return avail


def blocks_from_mask(avail, cell, border, fft, iters):
    """Cover the lost pixels of an availability mask with blocks: the frame
    is cut into ``cell x cell`` tiles from (0, 0) (clipped at the right and
    bottom edges) and every tile holding a lost pixel becomes one block,
    frame-major, then row-major. With a mask-driven loss area, each block
    conceals only its tile's lost pixels."""
    nf, H, W = avail.shape
    out = []
    for f in range(nf):
        for y0 in range(0, H, cell):
            for x0 in range(0, W, cell):
                bh, bw = min(cell, H - y0), min(cell, W - x0)
                if (avail[f, y0:y0 + bh, x0:x0 + bw] == 0).any():
                    out.append(Block(f, y0, x0, bh, bw, border, fft, iters))
    return out


def random_volume_losses(n_frames, height, width, bs, bt, fraction, seed, border, tborder, fft, fft_t, iters):
    """Lost volumes of bs x bs pixels x bt frames on the (bt, bs, bs) grid of
    the clip, drawn until ``fraction`` of the voxels are lost, no two
    sharing a face, edge or corner of the grid (so every volume sees its
    neighbourhood). Returns a VOLUME_DTYPE array, in grid order."""
    rng = np.random.default_rng(seed + LOSS_SEED_OFFSET)
    gt, gy, gx = n_frames // bt, height // bs, width // bs
    taken = np.zeros((gt, gy, gx), dtype=bool)
    want = int(round(fraction * gt * gy * gx))
    order = rng.permutation(gt * gy * gx)
    cells = []
    for c in order:
        if len(cells) >= want:
            break
        t, y, x = np.unravel_index(c, (gt, gy, gx))
        if taken[max(t - 1, 0):t + 2, max(y - 1, 0):y + 2, max(x - 1, 0):x + 2].any():
            continue
        taken[t, y, x] = True
        cells.append((t, y, x))
    cells.sort()
    out = np.zeros(len(cells), dtype=VOLUME_DTYPE)
    for i, (t, y, x) in enumerate(cells):
        out[i] = (t * bt, y * bs, x * bs, bt, bs, bs, border, tborder, fft, fft_t, 0, iters)
    return out


def volume_availability(shape, vols):
    """``uint8`` mask (frames, H, W): 0 inside every lost volume, else 1."""
    avail = np.ones(shape, dtype=np.uint8)
    for v in vols:
        f, y0, x0 = int(v["frame"]), int(v["y0"]), int(v["x0"])
        avail[f:f + int(v["bt"]), y0:y0 + int(v["bh"]), x0:x0 + int(v["bw"])] = 0
    return avail
