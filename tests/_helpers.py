"""Shared helpers of the GPU parity tests (inputs only; no method arithmetic)."""
import sys

import numpy as np
import torch


def announce(msg):
    """Name the case before a GPU step, so a crash log says what was running."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev():
    return torch.device("cuda:0")


def gpu(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).to(dev())


def host(t):
    return t.detach().cpu().numpy()


def f64(t):
    """float32 GPU/CPU tensor -> float64 numpy (the oracle's input)."""
    return t.detach().cpu().double().numpy()


def smooth_field(rng, B, H, W, amp, freq=2.0):
    """Smooth random displacement [B][2][H][W] float32 with values in about [-amp, amp]."""
    yy, xx = np.mgrid[0:H, 0:W]
    out = np.zeros((B, 2, H, W))
    for b in range(B):
        for c in range(2):
            for _ in range(3):
                kx, ky = rng.uniform(-freq, freq, size=2) * 2 * np.pi
                ph = rng.uniform(0, 2 * np.pi)
                out[b, c] += np.sin(kx * xx / W + ky * yy / H + ph)
            out[b, c] *= amp / 3.0
            out[b, c] += rng.uniform(-0.3, 0.3, size=(H, W)) * amp * 0.2
    return out.astype(np.float32)
