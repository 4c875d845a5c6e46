"""The seeded generator produces the stated structure (no RPCA arithmetic here)."""
import numpy as np

from synth import (make_window, casorati, frames_of, density_counts, batch_shapes,
                   serve_trace, BATCH_SIZES, BATCH_FRAMES, SERVE_SIDES, SERVE_FRAMES)
from synth.ultrasound import BUBBLE_AMPLITUDE


def test_shapes_layout_and_determinism():
    w1 = make_window(64, 48, 10, 5, 10, 3, 20.0, seed=123)
    w2 = make_window(64, 48, 10, 5, 10, 3, 20.0, seed=123)
    w3 = make_window(64, 48, 10, 5, 10, 3, 20.0, seed=124)
    assert w1.frames.shape == (10, 64, 48)
    assert np.array_equal(w1.frames, w2.frames)
    assert not np.array_equal(w1.frames, w3.frames)
    X = w1.X()
    assert X.shape == (64 * 48, 10) and X.flags.f_contiguous
    # frame t is column t, contiguous at offset t*m
    assert np.array_equal(X[:, 3], w1.frames[3].ravel())
    assert np.array_equal(frames_of(X, 64, 48), w1.frames)
    assert casorati(w1.frames).base is not None or casorati(w1.frames).flags.f_contiguous


def test_tissue_is_rank_two_and_bound_is_static():
    w = make_window(64, 64, 12, 6, 0, 3, 200.0, seed=5)
    T = (w.L_gt - w.bound[None]).reshape(12, -1).T
    s = np.linalg.svd(T, compute_uv=False)
    assert s[2] < 1e-10 * s[0] and s[1] > 1e-4 * s[0]
    # ground truth low-rank part = tissue + the same bound image in every frame
    assert np.allclose(w.L_gt - (w.L_gt - w.bound[None]), w.bound[None])
    assert w.bound_mask.sum() > 0
    assert w.bound.max() <= BUBBLE_AMPLITUDE * 6 + 1e-9


def test_noise_level_matches_snr():
    w = make_window(128, 128, 8, 10, 20, 3, 20.0, seed=9)
    clean = w.L_gt + w.S_gt
    noise = w.frames - clean
    snr = 20 * np.log10(np.sqrt(np.mean(clean ** 2)) / np.sqrt(np.mean(noise ** 2)))
    assert abs(snr - 20.0) < 0.1


def test_free_bubbles_move_and_stay_sparse():
    w = make_window(128, 128, 10, 0, 20, 3, 20.0, seed=3)
    assert np.abs(w.S_gt).max() > 1.0
    # frames differ (the bubbles move)
    assert np.abs(w.S_gt[0] - w.S_gt[5]).max() > 1.0
    # sparse: most pixels carry almost no free-bubble signal
    assert np.mean(np.abs(w.S_gt) > 0.1) < 0.1


def test_density_rule_and_batch_set():
    assert density_counts(512, 512) == (202, 403, 6)
    assert density_counts(128, 128)[2] == 3
    shapes = batch_shapes()
    assert len(shapes) == 64
    assert all((H, W) in BATCH_SIZES and n in BATCH_FRAMES for H, W, n, _ in shapes)
    assert [s[3] for s in shapes] == list(range(3000, 3064))


def test_serve_trace_poisson():
    tr = serve_trace()
    assert 2700 < len(tr) < 3300            # 50/s for 60 s
    t = np.array([a for a, *_ in tr])
    assert np.all(np.diff(t) > 0) and t[-1] < 60.0
    assert all(s in SERVE_SIDES and n in SERVE_FRAMES for _, s, n, _ in tr)


def test_device_window_geometry_in_worker_processes():
    """The serve workload draws a window's host-side geometry in worker
    processes and renders it in the main process: the result is the window
    built in one piece, bit for bit (CPU device here)."""
    import pickle
    from concurrent.futures import ProcessPoolExecutor

    import torch
    from synth.device import device_window, render_window, window_geometry

    shapes = [(40, 52, 20, 5001), (64, 48, 10, 5002), (24, 24, 3, 5003)]
    with ProcessPoolExecutor(2) as ex:
        geoms = list(ex.map(window_geometry, *zip(*shapes)))
    for (H, W, n, seed), g in zip(shapes, geoms):
        pickle.dumps(g)
        a = render_window(g, torch.device("cpu"))
        b = device_window(H, W, n, seed, torch.device("cpu"))
        assert a.shape == (n, H, W)
        assert torch.equal(a, b)
