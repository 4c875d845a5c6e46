"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Holds no RPCA arithmetic: it only builds input windows and their ground truth.
"""
from .ultrasound import (Window, casorati, frames_of, density_counts, make_window,
                         window_128x128x20, window_512x512x20, window_1024x1024x40,
                         batch_shapes, batch_window, serve_trace, planted_low_rank_sparse,
                         BATCH_SIZES, BATCH_FRAMES, SERVE_SIDES, SERVE_FRAMES)

__all__ = ["Window", "casorati", "frames_of", "density_counts", "make_window",
           "window_128x128x20", "window_512x512x20", "window_1024x1024x40",
           "batch_shapes", "batch_window", "serve_trace", "planted_low_rank_sparse",
           "BATCH_SIZES", "BATCH_FRAMES", "SERVE_SIDES", "SERVE_FRAMES"]
