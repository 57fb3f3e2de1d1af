"""Named synthetic workloads (frames + availability + block descriptors).

Each workload mirrors one experiment shape: the paper's isolated 16x16
losses with a 16-pixel support band and a 64x64 transform (Section IV), at
frame sizes and loss densities that fill a GPU.
"""
from dataclasses import dataclass

import numpy as np

from .images import synthetic_clip, synthetic_image
from .losses import (array_to_blocks, availability_mask, blocks_from_mask, blocks_to_array,
                     isolated_grid_losses, mixed_size_losses, random_grid_losses, random_volume_losses,
                     stroke_mask, volume_availability)


@dataclass
class Workload:
    name: str
    frames: np.ndarray        # uint8 [n_frames][H][W], the undistorted frames
    avail: np.ndarray         # uint8 [n_frames][H][W], 1 = received
    blocks: np.ndarray        # BLOCK_DTYPE [n_blocks]
    rho: float
    gamma: float

    @property
    def block_list(self):
        return array_to_blocks(self.blocks)

    @property
    def distorted(self):
        """Frames with every lost pixel set to 0 (what a receiver holds)."""
        return (self.frames * self.avail).astype(np.uint8)

    @property
    def lost_pixels(self):
        return int((self.avail == 0).sum())


def _finish(name, frames, blocks, rho=0.8, gamma=0.5):
    avail = availability_mask(frames.shape, blocks)
    return Workload(name, frames, avail, blocks_to_array(blocks), rho, gamma)


def isolated_256(iters=100):
    """256x256 frame (seed 0), every other 16x16 block lost (64 blocks, 25%),
    border 16 (48x48 area), F=64."""
    frames = synthetic_image(256, 256, 0)[None]
    return _finish("isolated-256", frames, isolated_grid_losses(256, 256, 16, 16, 64, iters))


def random_1080p_8x8(iters=200, seed=1):
    """1920x1080 frame, 10% of the 8x8 grid lost, non-adjacent (3240 blocks),
    border 16 (40x40 area), F=64."""
    frames = synthetic_image(1080, 1920, seed)[None]
    return _finish("random-1080p-8x8", frames,
                   random_grid_losses(1080, 1920, 8, 0.10, seed, 16, 64, iters))


def random_1080p_16x16(seeds=(99,), iters=100):
    """1920x1080 frames, 10% of the 16x16 grid lost per frame, non-adjacent
    (804 blocks per frame), border 16 (48x48 area), F=64."""
    frames, blocks = [], []
    for f, s in enumerate(seeds):
        frames.append(synthetic_image(1080, 1920, s))
        blocks += random_grid_losses(1080, 1920, 16, 0.10, s, 16, 64, iters, frame=f)
    return _finish("random-1080p-16x16", np.stack(frames), blocks)


def mixed_4k(seeds=tuple(range(2, 10))):
    """3840x2160 frames with 305 blocks each of 4, 8, 16 and 32 pixels per
    frame (5% loss), border 8..16, F in {32, 64, 128}, I in {50,...,500}."""
    frames, blocks = [], []
    for f, s in enumerate(seeds):
        frames.append(synthetic_image(2160, 3840, s))
        blocks += mixed_size_losses(2160, 3840, s, frame=f)
    return _finish("mixed-4k", np.stack(frames), blocks)


def strokes_1080p(seeds=(31,), iters=100, density=0.06):
    """1920x1080 frames with irregular scribble losses (6% of the pixels,
    strokes 2-7 px wide), covered by 16x16 tiles with border 16 (48x48
    areas) and F=64; each block conceals only its tile's lost pixels (a
    mask-driven loss area)."""
    frames, avails = [], []
    for s in seeds:
        frames.append(synthetic_image(1080, 1920, s))
        avails.append(stroke_mask(1080, 1920, s, density)[0])
    avail = np.stack(avails)
    blocks = blocks_from_mask(avail, 16, 16, 64, iters)
    return Workload("strokes-1080p", np.stack(frames), avail, blocks_to_array(blocks), 0.8, 0.5)


def strokes_256(seed=5, iters=60, density=0.08):
    """256x256 frame with scribble losses, 16x16 tiles, border 16, F=64."""
    frames = synthetic_image(256, 256, seed)[None]
    avail = stroke_mask(256, 256, seed, density)
    blocks = blocks_from_mask(avail, 16, 16, 64, iters)
    return Workload("strokes-256", frames, avail, blocks_to_array(blocks), 0.8, 0.5)


def subset(w, idx):
    """Workload restricted to the blocks ``idx`` (frames shared); pixels of
    dropped blocks stay marked lost, so every kept block sees exactly the
    availability it had in the full workload."""
    return Workload(w.name + "-subset", w.frames, w.avail, w.blocks[np.asarray(idx)], w.rho, w.gamma)


def clip_1080p_16x16x2(n_frames=16, seed=41, iters=200, fraction=0.05):
    """A 1920x1080x16-frame clip (one synthetic image moving by up to +-3 px
    per frame), 16x16x2 lost volumes at 5% of the volume grid, border 16 in
    space and 2 in time (48x48x6 area), 64x64x8 transform."""
    frames = synthetic_clip(1080, 1920, n_frames, seed)
    vols = random_volume_losses(n_frames, 1080, 1920, 16, 2, fraction, seed, 16, 2, 64, 8, iters)
    return Workload("clip-1080p-16x16x2", frames, volume_availability(frames.shape, vols), vols, 0.8, 0.5)


def clip_small(n_frames=8, seed=43, iters=40, fraction=0.05):
    """A 256x256x8-frame clip, 16x16x2 lost volumes (border 16, 2), 64x64x8."""
    frames = synthetic_clip(256, 256, n_frames, seed)
    vols = random_volume_losses(n_frames, 256, 256, 16, 2, fraction, seed, 16, 2, 64, 8, iters)
    return Workload("clip-256", frames, volume_availability(frames.shape, vols), vols, 0.8, 0.5)
