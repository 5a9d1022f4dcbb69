"""Synthetic atom-column lattice series with known deformations.

Stand-in for the paper's high-resolution TEM series (Section 5, aluminium
oxidation data, not available here).  Recipe, per frame k of a series:

* lattice  L(q) = sum over the 3x3 nearest lattice sites s of
  exp(-|q - o - s|^2 / (2 sigma^2)), square lattice of spacing a, random
  origin o ~ U[0, a)^2, amplitude 1 on a zero background;
* frame    f_k(x) = L(x - d_k - w_k(x)) + n_k(x), n_k iid N(0, noise^2),
  plus N(0, extra_noise^2) on a seeded subset of frames;
  (rigid series: f_k(y) = L(Phi_k^{-1}(y)) + n_k(y) with Phi_k a rotation
  about the image centre and a translation whose parameters walk by
  U[-RIGID_STEP_ALPHA, RIGID_STEP_ALPHA] and U[-delta, delta]^2 per frame)
* drift    d_0 = 0, d_k = d_{k-1} + U[-delta, delta]^2 reflected into
  [-D, D], delta = min(a/4, D/2), so consecutive frames stay within half a
  lattice period of each other (Section 2.3.2) while the series as a whole
  drifts further;
* distortion w_k(x) = A_d (sin(2 pi y / H + th_k1), sin(2 pi x / W + th_k2)),
  th_0 ~ U[0, 2 pi)^2 and th_k = th_{k-1} + U[-0.25, 0.25]^2.

Ground truth: the displacement u_ik with f_k(x + u_ik(x)) ~ f_i(x) is p - x
where p solves p - d_k - w_k(p) = x - d_i - w_i(x) (a contraction, solved by
fixed-point iteration).

Scalar per-frame parameters come from NumPy's PCG64 seeded with the series
seed; pixel fields are evaluated with torch in float64 on the requested device
(noise from a torch generator seeded the same way), then rounded to float32.
A series generated on the CPU and one generated on a GPU therefore share
drift, distortion and origin but not the noise; every consumer is given the
same generated frames.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .configs import RIGID_STEP_ALPHA, SeriesSpec


@dataclass
class Series:
    spec: SeriesSpec
    frames: torch.Tensor      # [N][H][W] float32
    drift: np.ndarray         # [N][2]  (x, y) in px
    theta: np.ndarray         # [N][2]
    origin: np.ndarray        # [2]
    noisy: np.ndarray         # indices of frames with extra noise


def _frame_params(spec: SeriesSpec):
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    n = spec.n_frames
    a, dmax = spec.spacing, spec.drift
    delta = min(a / 4.0, dmax / 2.0)
    origin = rng.uniform(0.0, a, size=2)
    drift = np.zeros((n, 2))
    for k in range(1, n):
        v = drift[k - 1] + rng.uniform(-delta, delta, size=2)
        v = np.where(v > dmax, 2 * dmax - v, v)
        v = np.where(v < -dmax, -2 * dmax - v, v)
        drift[k] = v
    theta = np.zeros((n, 2))
    theta[0] = rng.uniform(0.0, 2 * math.pi, size=2)
    for k in range(1, n):
        theta[k] = theta[k - 1] + rng.uniform(-0.25, 0.25, size=2)
    n_extra = int(math.floor(spec.extra_noise_frac * n))
    noisy = np.sort(rng.choice(n, size=n_extra, replace=False)) if n_extra else np.zeros(0, np.int64)
    return origin, drift, theta, noisy


def _distortion(spec: SeriesSpec, theta, qx, qy):
    wx = spec.distort * torch.sin(2 * math.pi * qy / spec.height + float(theta[0]))
    wy = spec.distort * torch.sin(2 * math.pi * qx / spec.width + float(theta[1]))
    return wx, wy


def lattice_image(spec: SeriesSpec, origin, qx: torch.Tensor, qy: torch.Tensor) -> torch.Tensor:
    """Evaluate the lattice L at sample positions (qx, qy) (float64 tensors)."""
    a, s2 = spec.spacing, 2.0 * spec.sigma ** 2
    rx = qx - float(origin[0])
    ry = qy - float(origin[1])
    mx = torch.round(rx / a)
    my = torch.round(ry / a)
    out = torch.zeros_like(qx)
    for di in (-1.0, 0.0, 1.0):
        ex = rx - (mx + di) * a
        for dj in (-1.0, 0.0, 1.0):
            ey = ry - (my + dj) * a
            out += torch.exp(-(ex * ex + ey * ey) / s2)
    return out


def _window_grid(spec: SeriesSpec, window, dev):
    """Pixel coordinates of the frame, or of the window (y0, x0, h, w) of it:
    a crop that keeps the full frame's distortion (its period is the full
    height and width) and drift."""
    y0, x0, h, w = (0, 0, spec.height, spec.width) if window is None else window
    return torch.meshgrid(torch.arange(y0, y0 + h, dtype=torch.float64, device=dev),
                          torch.arange(x0, x0 + w, dtype=torch.float64, device=dev), indexing="ij")


def make_series(spec: SeriesSpec, device="cpu", frames_dtype=torch.float32, window=None) -> Series:
    """Generate the frame series of ``spec`` on ``device`` (only the pixels of
    ``window`` = (y0, x0, h, w) if given)."""
    origin, drift, theta, noisy = _frame_params(spec)
    dev = torch.device(device)
    N = spec.n_frames
    yy, xx = _window_grid(spec, window, dev)
    H, W = yy.shape
    gen = torch.Generator(device=dev)
    gen.manual_seed(spec.seed)
    frames = torch.empty((N, H, W), dtype=frames_dtype, device=dev)
    noisy_set = set(int(i) for i in noisy)
    for k in range(N):
        wx, wy = _distortion(spec, theta[k], xx, yy)
        f = lattice_image(spec, origin, xx - drift[k, 0] - wx, yy - drift[k, 1] - wy)
        if spec.noise > 0:
            f += spec.noise * torch.randn((H, W), generator=gen, dtype=torch.float64, device=dev)
        if k in noisy_set and spec.extra_noise > 0:
            f += spec.extra_noise * torch.randn((H, W), generator=gen, dtype=torch.float64, device=dev)
        frames[k] = f.to(frames_dtype)
    return Series(spec, frames, drift, theta, origin, noisy)


def ground_truth(series: Series, i: int, k: int, iters: int = 60, window=None) -> np.ndarray:
    """Analytic displacement u_ik as a float64 array [2][H][W] (x, y planes),
    on the pixels of ``window`` if given."""
    spec = series.spec
    yy, xx = _window_grid(spec, window, torch.device("cpu"))
    wix, wiy = _distortion(spec, series.theta[i], xx, yy)
    cx = xx - series.drift[i, 0] - wix + series.drift[k, 0]
    cy = yy - series.drift[i, 1] - wiy + series.drift[k, 1]
    px, py = cx.clone(), cy.clone()
    for _ in range(iters):
        wkx, wky = _distortion(spec, series.theta[k], px, py)
        px, py = cx + wkx, cy + wky
    return torch.stack([px - xx, py - yy]).numpy()


def clean_frame(series: Series, k: int, window=None) -> np.ndarray:
    """Noise-free frame k of a generated series as float64 [H][W] (for masks)."""
    spec = series.spec
    yy, xx = _window_grid(spec, window, torch.device("cpu"))
    wx, wy = _distortion(spec, series.theta[k], xx, yy)
    return lattice_image(spec, series.origin, xx - series.drift[k, 0] - wx,
                         yy - series.drift[k, 1] - wy).numpy()


def rigid_pair(spec: SeriesSpec, theta, seed_offset: int = 0):
    """Reference R(x) = L(x) and template T(y) = L(phi^{-1}(y)) for the rigid
    motion phi(x) = Rot(alpha)(x - c) + c + G, theta = (alpha, G_x, G_y),
    c = ((w - 1) / 2, (h - 1) / 2), so that T(phi(x)) = R(x); iid noise of
    spec.noise on both.  Returns float32 tensors [H][W]."""
    origin, _, _, _ = _frame_params(spec)
    H, W = spec.height, spec.width
    yy, xx = torch.meshgrid(torch.arange(H, dtype=torch.float64), torch.arange(W, dtype=torch.float64), indexing="ij")
    a, gx, gy = (float(v) for v in theta)
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    ux, uy = xx - cx - gx, yy - cy - gy
    qx = math.cos(a) * ux + math.sin(a) * uy + cx
    qy = -math.sin(a) * ux + math.cos(a) * uy + cy
    R = lattice_image(spec, origin, xx, yy)
    T = lattice_image(spec, origin, qx, qy)
    if spec.noise > 0:
        gen = torch.Generator()
        gen.manual_seed(spec.seed + 7919 * (1 + seed_offset))
        R = R + spec.noise * torch.randn((H, W), generator=gen, dtype=torch.float64)
        T = T + spec.noise * torch.randn((H, W), generator=gen, dtype=torch.float64)
    return R.to(torch.float32), T.to(torch.float32)


@dataclass
class RigidSeries:
    spec: SeriesSpec
    frames: torch.Tensor      # [N][H][W] float32
    theta: np.ndarray         # [N][3] (alpha, G_x, G_y) of Phi_k; Phi_0 = identity


def _rigid_frame(spec: SeriesSpec, origin, theta, xx, yy):
    """L(Phi^{-1}(y)) for Phi(x) = Rot(alpha)(x - c) + c + G."""
    a, gx, gy = (float(v) for v in theta)
    cx, cy = (spec.width - 1) / 2.0, (spec.height - 1) / 2.0
    ux, uy = xx - cx - gx, yy - cy - gy
    qx = math.cos(a) * ux + math.sin(a) * uy + cx
    qy = -math.sin(a) * ux + math.cos(a) * uy + cy
    return lattice_image(spec, origin, qx, qy)


def rigid_series(spec: SeriesSpec, device="cpu") -> RigidSeries:
    """Lattice series under rigid motion: frame k is the lattice moved by
    Phi_k, so f_k(Phi_k(x)) = f_0(x) up to noise and Phi_k is the motion that
    registers frame k to frame 0.  Phi_0 = identity; the angle and the
    translation of Phi_k walk from frame to frame (bounded steps, translation
    reflected into [-D, D]^2)."""
    origin, drift, _, _ = _frame_params(spec)
    rng = np.random.Generator(np.random.PCG64(spec.seed + 104729))
    n = spec.n_frames
    theta = np.zeros((n, 3))
    theta[:, 1:] = drift
    for k in range(1, n):
        theta[k, 0] = theta[k - 1, 0] + rng.uniform(-RIGID_STEP_ALPHA, RIGID_STEP_ALPHA)
    dev = torch.device(device)
    H, W = spec.height, spec.width
    yy, xx = torch.meshgrid(torch.arange(H, dtype=torch.float64, device=dev),
                            torch.arange(W, dtype=torch.float64, device=dev), indexing="ij")
    gen = torch.Generator(device=dev)
    gen.manual_seed(spec.seed + 15485863)
    frames = torch.empty((n, H, W), dtype=torch.float32, device=dev)
    for k in range(n):
        f = _rigid_frame(spec, origin, theta[k], xx, yy)
        if spec.noise > 0:
            f += spec.noise * torch.randn((H, W), generator=gen, dtype=torch.float64, device=dev)
        frames[k] = f.to(torch.float32)
    return RigidSeries(spec, frames, theta)
