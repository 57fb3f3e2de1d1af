"""Seeded synthetic inputs for block-loss concealment experiments.

This package only draws random numbers and paints pixels: it holds none of
the extrapolation arithmetic. Both the FP64 CPU oracle (``oracle/``) and the
GPU path (``paper_2204_14193_amd``) take their inputs from here, so that the
two sides see identical frames, masks and block lists.

The paper evaluates on natural photographs (the Kodak set, Section IV); those
are not available, so these generators stand in for them with images of the
same bit depth that mix smooth oscillations, sharp edges and sensor-like
noise.
"""
from .images import synthetic_image, synthetic_frames
from .losses import (Block, BLOCK_DTYPE, blocks_to_array, isolated_grid_losses,
                     random_grid_losses, mixed_size_losses, fft_size_for_area, stroke_mask,
                     blocks_from_mask)

__all__ = ["synthetic_image", "synthetic_frames", "Block", "BLOCK_DTYPE",
           "blocks_to_array", "isolated_grid_losses", "random_grid_losses",
           "mixed_size_losses", "fft_size_for_area", "stroke_mask", "blocks_from_mask"]
