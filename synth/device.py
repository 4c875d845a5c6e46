"""Seeded ultrasound-shaped windows built directly in device memory.

The same model as ``synth.ultrasound.make_window`` (rank-2 drifting speckle,
fixed bound bubbles, free bubbles moving 2-6 px/frame along random-
acceleration vessel paths, white noise at a given SNR), for the serving
workload, whose windows (up to 1024 x 1024 px x 100 frames) are too large to
build with the host generator at the arrival rate.  Bubble positions, vessel
paths and drift phases are drawn on the host from ``numpy`` with the window's
seed; the speckle and noise fields come from a device ``torch.Generator``
seeded with the same seed, so a window is reproducible but its values differ
from the host generator's window of the same seed.  The speckle blur is a
periodic Gaussian applied in the Fourier domain.

Holds no RPCA arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

from .ultrasound import (BUBBLE_AMPLITUDE, DRIFT, PSF_SIGMA, _vessel_path, density_counts)


def _gauss_hat(H: int, W: int, device):
    import torch
    fy = torch.fft.fftfreq(H, device=device, dtype=torch.float64)
    fx = torch.fft.fftfreq(W, device=device, dtype=torch.float64)
    g = torch.exp(-2.0 * (math.pi * PSF_SIGMA) ** 2 * (fy[:, None] ** 2 + fx[None, :] ** 2))
    return g


def _speckle(gen, H: int, W: int, ghat, device):
    import torch
    re = torch.randn((H, W), generator=gen, device=device, dtype=torch.float64)
    im = torch.randn((H, W), generator=gen, device=device, dtype=torch.float64)
    re = torch.fft.ifft2(torch.fft.fft2(re) * ghat).real
    im = torch.fft.ifft2(torch.fft.fft2(im) * ghat).real
    env = torch.hypot(re, im)
    return env / env.mean()


def _splat_many(img_flat, H: int, W: int, frame_idx: np.ndarray, cy: np.ndarray, cx: np.ndarray,
                amp: float, device):
    """Add Gaussian blobs (centres cy, cx in frame frame_idx) into the
    flattened (frames*H*W) image, clipped at the borders."""
    import torch
    if len(cy) == 0:
        return
    rad = int(math.ceil(4.0 * PSF_SIGMA))
    off = torch.arange(-rad, rad + 2, device=device, dtype=torch.int64)
    cy_t = torch.as_tensor(cy, device=device, dtype=torch.float64)
    cx_t = torch.as_tensor(cx, device=device, dtype=torch.float64)
    fr = torch.as_tensor(frame_idx, device=device, dtype=torch.int64)
    yy = torch.floor(cy_t).to(torch.int64)[:, None] + off[None, :]        # (N, K)
    xx = torch.floor(cx_t).to(torch.int64)[:, None] + off[None, :]
    dy = yy.to(torch.float64) - cy_t[:, None]
    dx = xx.to(torch.float64) - cx_t[:, None]
    val = amp * torch.exp(-(dy[:, :, None] ** 2 + dx[:, None, :] ** 2) / (2.0 * PSF_SIGMA ** 2))
    ok = ((yy >= 0) & (yy < H))[:, :, None] & ((xx >= 0) & (xx < W))[:, None, :]
    idx = fr[:, None, None] * (H * W) + yy.clamp(0, H - 1)[:, :, None] * W + xx.clamp(0, W - 1)[:, None, :]
    img_flat.index_put_((idx[ok],), val[ok], accumulate=True)


def window_geometry(H: int, W: int, n: int, seed: int) -> dict:
    """The host-side draws of a window (drift phases, bound bubble centres,
    free bubble tracks along the vessel paths), from numpy with the window's
    seed, in the order ``device_window`` has always drawn them.  Plain
    arrays, so it can run in a worker process."""
    n_bound, n_free, n_vessels = density_counts(H, W)
    rng = np.random.default_rng(seed)
    phi1, phi2 = rng.uniform(0, 2 * np.pi, size=2)
    lo = 4.0
    by = rng.uniform(lo, H - lo, size=n_bound)
    bx = rng.uniform(lo, W - lo, size=n_bound)
    paths = [_vessel_path(rng, H, W) for _ in range(max(n_vessels, 1))]
    fy, fx, ff = [], [], []
    k = np.arange(n, dtype=np.float64)
    for b in range(n_free):
        path = paths[b % len(paths)]
        length = max(0.5 * (len(path) - 1), 1e-9)
        s0 = rng.uniform(0.0, length)
        speed = rng.uniform(2.0, 6.0)
        s = (s0 + speed * k) % length
        idx = s / 0.5
        i0 = np.floor(idx).astype(np.int64)
        i1 = np.minimum(i0 + 1, len(path) - 1)
        f = (idx - i0)[:, None]
        pos = (1 - f) * path[i0] + f * path[i1]
        fy.append(pos[:, 0])
        fx.append(pos[:, 1])
        ff.append(np.arange(n, dtype=np.int64))
    cat = (lambda a, dt: np.concatenate(a) if a else np.zeros(0, dtype=dt))
    return {"H": H, "W": W, "n": n, "seed": seed, "phi": (float(phi1), float(phi2)),
            "by": by, "bx": bx, "fy": cat(fy, np.float64), "fx": cat(fx, np.float64),
            "ff": cat(ff, np.int64)}


def render_window(geom: dict, device, dtype=None, snr_db: float = 20.0):
    """(n, H, W) C-contiguous window on `device` from its host-side draws:
    speckle and noise from a device generator seeded with the window's seed,
    bubbles splatted at the drawn positions."""
    import torch
    dtype = dtype or torch.float32
    H, W, n, seed = geom["H"], geom["W"], geom["n"], geom["seed"]
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    ghat = _gauss_hat(H, W, device)
    s1 = _speckle(gen, H, W, ghat, device)
    s2 = _speckle(gen, H, W, ghat, device)
    phi1, phi2 = geom["phi"]
    t = torch.arange(n, device=device, dtype=torch.float64)
    c1 = 1.0 + DRIFT * torch.sin(2 * math.pi * t / (4 * n) + phi1)
    c2 = DRIFT * torch.cos(2 * math.pi * t / (4 * n) + phi2)
    clean = c1[:, None, None] * s1[None] + c2[:, None, None] * s2[None]

    by, bx = geom["by"], geom["bx"]
    bound = torch.zeros(H * W, device=device, dtype=torch.float64)
    _splat_many(bound, H, W, np.zeros(len(by), dtype=np.int64), by, bx, BUBBLE_AMPLITUDE, device)
    clean += bound.view(1, H, W)
    if len(geom["ff"]):
        flat = clean.view(-1)
        _splat_many(flat, H, W, geom["ff"], geom["fy"], geom["fx"], BUBBLE_AMPLITUDE, device)
    rms = float(torch.sqrt(torch.mean(clean * clean)))
    sigma_n = rms * 10.0 ** (-snr_db / 20.0)
    clean += sigma_n * torch.randn(clean.shape, generator=gen, device=device, dtype=torch.float64)
    return clean.to(dtype).contiguous()


def device_window(H: int, W: int, n: int, seed: int, device, dtype=None, snr_db: float = 20.0):
    """(n, H, W) C-contiguous window on `device` (the Casorati layout with
    m = H*W), densities as for the batched and served sets."""
    return render_window(window_geometry(H, W, n, seed), device, dtype, snr_db)
