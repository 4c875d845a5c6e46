"""Seeded synthetic ultrasound windows shaped like the paper's Casorati input.

This module only manufactures inputs; it contains none of the RPCA arithmetic,
so it can serve both the CPU oracle and the GPU path.

What is modelled (paper Sec. II-A data model X = L + S, Eq. 1; Sec. II-C):

* tissue: two independent speckle images mixed with slow +-5 % amplitude drift,
  i.e. a rank-2 background that drifts over the frames;
* bound bubbles: Gaussian point-spread blobs fixed over all frames
  (the low-rank "bound microbubble" signal of Sec. II-A);
* free bubbles: the same blobs moving 2-6 px/frame along curved vessel paths.
  The paths are traced with the random-acceleration kinematics of Sec. II-C.2
  (v(t) = v(t-1) + a dt, x(t) = x(t-1) + v(t) dt, random acceleration angle),
  expressed in pixel units;
* additive white Gaussian noise at a given SNR (Sec. II-C.1 adds thermal noise
  relative to the RMS of the signal).

Layout: every array of frames is (n_frames, H, W), C-contiguous.  That is the
Casorati matrix X (pixels x frames, paper Sec. II-A) stored column-major with
leading dimension m = H*W: frame t is contiguous at offset t*m.  ``casorati``
returns the (m, n) Fortran-ordered view without copying.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.ndimage import gaussian_filter

PSF_SIGMA = 1.5          # px, blob and speckle correlation length
BUBBLE_AMPLITUDE = 3.0   # times the tissue mean (tissue is normalised to mean 1)
BOUND_MASK_LEVEL = 1.5   # ground-truth bound mask: B(p) >= this
DRIFT = 0.05             # +-5 % slow amplitude drift of the tissue


@dataclass
class Window:
    """One synthetic frame window and its ground truth."""
    frames: np.ndarray      # (n, H, W) float64: observed data X
    L_gt: np.ndarray        # (n, H, W) float64: tissue + bound bubbles
    S_gt: np.ndarray        # (n, H, W) float64: free bubbles
    bound: np.ndarray       # (H, W) float64: bound-bubble image B
    bound_mask: np.ndarray  # (H, W) bool: B >= BOUND_MASK_LEVEL
    noise_sigma: float
    seed: int

    @property
    def m(self) -> int:
        return int(self.frames.shape[1] * self.frames.shape[2])

    @property
    def n(self) -> int:
        return int(self.frames.shape[0])

    def X(self, dtype=np.float64) -> np.ndarray:
        """Casorati matrix, shape (m, n), Fortran order (ld = m)."""
        return casorati(self.frames.astype(dtype, copy=False))


def casorati(frames: np.ndarray) -> np.ndarray:
    """(n, H, W) C-contiguous frames -> (m, n) Fortran-ordered view."""
    n = frames.shape[0]
    return np.ascontiguousarray(frames).reshape(n, -1).T


def frames_of(X: np.ndarray, H: int, W: int) -> np.ndarray:
    """(m, n) Casorati matrix -> (n, H, W) frames (copy if needed)."""
    return np.asfortranarray(X).T.reshape(X.shape[1], H, W)


def density_counts(H: int, W: int) -> tuple[int, int, int]:
    """Bubble/vessel counts for the batched and served windows.

    1 bound and 2 free bubbles per 1300 px^2; vessels grow with area
    (3 at 128x128 ... 6 at 512x512, at least 3).
    """
    m = H * W
    n_bound = int(round(m / 1300.0))
    n_free = int(round(2.0 * m / 1300.0))
    n_vessels = max(3, int(np.floor(6.0 * m / 262144.0 + 0.5)))
    return n_bound, n_free, n_vessels


def _speckle(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    """Envelope of blurred complex white noise, normalised to mean 1."""
    re = gaussian_filter(rng.standard_normal((H, W)), PSF_SIGMA, mode="wrap")
    im = gaussian_filter(rng.standard_normal((H, W)), PSF_SIGMA, mode="wrap")
    env = np.hypot(re, im)
    return env / env.mean()


def _splat(img: np.ndarray, cy: float, cx: float, amp: float) -> None:
    """Add amp * exp(-r^2 / (2 sigma^2)) centred at (cy, cx), in place."""
    H, W = img.shape
    rad = int(np.ceil(4.0 * PSF_SIGMA))
    y0, y1 = int(np.floor(cy)) - rad, int(np.floor(cy)) + rad + 2
    x0, x1 = int(np.floor(cx)) - rad, int(np.floor(cx)) + rad + 2
    ya, yb = max(y0, 0), min(y1, H)
    xa, xb = max(x0, 0), min(x1, W)
    if ya >= yb or xa >= xb:
        return
    yy = np.arange(ya, yb, dtype=np.float64)[:, None] - cy
    xx = np.arange(xa, xb, dtype=np.float64)[None, :] - cx
    img[ya:yb, xa:xb] += amp * np.exp(-(yy * yy + xx * xx) / (2.0 * PSF_SIGMA ** 2))


def _vessel_path(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    """Curved path (K, 2) in pixel coordinates, resampled at 0.5 px spacing.

    Random-acceleration kinematics in pixel units: the tracer starts at a
    random border point heading inwards, and at every step receives an
    acceleration of random magnitude and random angle in [-pi, pi].
    """
    side = rng.integers(4)
    if side == 0:
        p = np.array([0.0, rng.uniform(0, W)]); ang = np.pi / 2
    elif side == 1:
        p = np.array([H - 1.0, rng.uniform(0, W)]); ang = -np.pi / 2
    elif side == 2:
        p = np.array([rng.uniform(0, H), 0.0]); ang = 0.0
    else:
        p = np.array([rng.uniform(0, H), W - 1.0]); ang = np.pi
    # (dy, dx) with angle measured so that ang=0 points along +x
    ang += rng.uniform(-np.pi / 4, np.pi / 4)
    v = 1.0 * np.array([np.sin(ang), np.cos(ang)])
    pts = [p.copy()]
    max_steps = 8 * (H + W)
    for _ in range(max_steps):
        a_mag = rng.uniform(0.01, 0.1)
        a_ang = rng.uniform(-np.pi, np.pi)
        v = v + a_mag * np.array([np.sin(a_ang), np.cos(a_ang)])
        sp = np.linalg.norm(v)
        v = v / sp * np.clip(sp, 0.5, 1.5)
        p = p + v
        pts.append(p.copy())
        if not (-2 <= p[0] <= H + 1 and -2 <= p[1] <= W + 1):
            break
    pts = np.asarray(pts)
    seg = np.linalg.norm(np.diff(pts, axis=0), axis=1)
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    s = np.arange(0.0, arc[-1], 0.5)
    return np.stack([np.interp(s, arc, pts[:, 0]), np.interp(s, arc, pts[:, 1])], axis=1)


def make_window(H: int, W: int, n: int, n_bound: int, n_free: int, n_vessels: int,
                snr_db: float, seed: int) -> Window:
    """Build one seeded window; see the module docstring for the model."""
    rng = np.random.default_rng(seed)
    s1 = _speckle(rng, H, W)
    s2 = _speckle(rng, H, W)
    phi1, phi2 = rng.uniform(0, 2 * np.pi, size=2)
    t = np.arange(n, dtype=np.float64)
    c1 = 1.0 + DRIFT * np.sin(2 * np.pi * t / (4 * n) + phi1)
    c2 = DRIFT * np.cos(2 * np.pi * t / (4 * n) + phi2)
    tissue = c1[:, None, None] * s1[None] + c2[:, None, None] * s2[None]

    bound = np.zeros((H, W))
    lo = 4.0
    for _ in range(n_bound):
        _splat(bound, rng.uniform(lo, H - lo), rng.uniform(lo, W - lo), BUBBLE_AMPLITUDE)

    free = np.zeros((n, H, W))
    paths = [_vessel_path(rng, H, W) for _ in range(max(n_vessels, 1))]
    for b in range(n_free):
        path = paths[b % len(paths)]
        length = 0.5 * (len(path) - 1)
        s0 = rng.uniform(0.0, max(length, 1e-9))
        speed = rng.uniform(2.0, 6.0)
        for k in range(n):
            s = (s0 + speed * k) % max(length, 1e-9)
            idx = s / 0.5
            i0 = int(np.floor(idx))
            i1 = min(i0 + 1, len(path) - 1)
            f = idx - i0
            pos = (1 - f) * path[i0] + f * path[i1]
            _splat(free[k], pos[0], pos[1], BUBBLE_AMPLITUDE)

    L_gt = tissue + bound[None]
    clean = L_gt + free
    rms = float(np.sqrt(np.mean(clean * clean)))
    sigma_n = rms * 10.0 ** (-snr_db / 20.0)
    frames = clean + sigma_n * rng.standard_normal(clean.shape)
    return Window(frames=frames, L_gt=L_gt, S_gt=free, bound=bound,
                  bound_mask=bound >= BOUND_MASK_LEVEL, noise_sigma=sigma_n, seed=seed)


# ---------------------------------------------------------------------------
# The named workloads.  Each is the paper-shaped stand-in for data that cannot
# be regenerated here (Field II / BubbleSim simulations, phantom and in vivo
# acquisitions).
# ---------------------------------------------------------------------------

def window_128x128x20(seed: int = 1) -> Window:
    """128x128 px x 20 frames; 30 bound, 60 free bubbles, 3 vessels, 20 dB."""
    return make_window(128, 128, 20, 30, 60, 3, 20.0, seed)


def window_512x512x20(seed: int = 2) -> Window:
    """512x512 px x 20 frames; 200 bound, 400 free bubbles, 6 vessels, 20 dB."""
    return make_window(512, 512, 20, 200, 400, 6, 20.0, seed)


def window_1024x1024x40(seed: int = 4) -> Window:
    """1024x1024 px x 40 frames; 800 bound, 1600 free bubbles, 24 vessels, 15 dB."""
    return make_window(1024, 1024, 40, 800, 1600, 24, 15.0, seed)


BATCH_SIZES = ((256, 256), (384, 512), (512, 512), (512, 768))
BATCH_FRAMES = (10, 20, 40, 60)


def batch_shapes(count: int = 64, seed: int = 3) -> list[tuple[int, int, int, int]]:
    """Uneven window shapes (H, W, n, seed_i) of the batched sliding-window set.

    Image size uniform over BATCH_SIZES, frame count uniform over BATCH_FRAMES;
    window i is generated with seed 3000 + i.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        H, W = BATCH_SIZES[rng.integers(len(BATCH_SIZES))]
        n = BATCH_FRAMES[rng.integers(len(BATCH_FRAMES))]
        out.append((int(H), int(W), int(n), 3000 + i))
    return out


def batch_window(H: int, W: int, n: int, seed: int, snr_db: float = 20.0) -> Window:
    nb, nf, nv = density_counts(H, W)
    return make_window(H, W, n, nb, nf, nv, snr_db, seed)


SERVE_SIDES = tuple(range(256, 1025, 32))
SERVE_FRAMES = (10, 20, 40, 100)


def serve_trace(rate_hz: float = 50.0, duration_s: float = 60.0, seed: int = 5):
    """Poisson arrival trace of serving requests.

    Returns a list of (arrival_time_s, side, n, seed_i): square windows with
    side uniform over SERVE_SIDES (256..1024 step 32), frame count uniform over
    SERVE_FRAMES; request i is generated with seed 5000 + i.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    i = 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        side = int(SERVE_SIDES[rng.integers(len(SERVE_SIDES))])
        n = int(SERVE_FRAMES[rng.integers(len(SERVE_FRAMES))])
        out.append((t, side, n, 5000 + i))
        i += 1
    return out


def planted_low_rank_sparse(m: int, n: int, rank: int, rho: float, seed: int):
    """Planted (L0, S0) pair for exact-recovery checks of the PCP model (Eq. 2).

    L0 = c U V^T with U (m x r) ~ N(0, 1/m), V (n x r) ~ N(0, 1/n) and
    c = sqrt(mn/r) / sqrt(max(m, n)), so its entries have RMS about
    1/sqrt(max(m, n)).  S0 is nonzero on an i.i.d. Bernoulli(rho) support with
    random signs and magnitude 10 x mean|L0|: the classical construction for
    testing principal component pursuit.
    """
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((m, rank)) / np.sqrt(m)
    V = rng.standard_normal((n, rank)) / np.sqrt(n)
    L0 = U @ V.T * np.sqrt(m * n / rank) / np.sqrt(max(m, n))
    supp = rng.random((m, n)) < rho
    S0 = np.where(supp, rng.choice([-1.0, 1.0], size=(m, n)), 0.0)
    scale = np.abs(L0).mean() * 10.0
    S0 = S0 * scale
    return np.asfortranarray(L0), np.asfortranarray(S0)
