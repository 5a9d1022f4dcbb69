"""Differentiation of the warp + energy step, CPU oracle.  TEST INFRASTRUCTURE ONLY.

Energy of a batch item, over a pyramid of ``levels`` levels built by the
binomial frame restriction of both images and half the 2x2 block mean of the
displacement (the restrictions of the registration's multilevel scheme):

    E(I_a, u, I_b) = sum_l [ sum_x (I_a^l(x + u^l(x)) - I_b^l(x))^2
                             + lam |grad u^l|^2 ]

(levels = 1 is the plain energy of the registration operator, Section 2.3.1).
Gradients are written out analytically: the transpose of the bilinear gather
(a scatter of the residual into the four taps), the energy gradient in u, and
the adjoints of the restrictions.
"""
from __future__ import annotations

import numpy as np

from .registration import (BINOMIAL6, energy, energy_and_gradient, restrict_field,
                           restrict_frame, restrict_image, sample_displaced, split_offset)


def warp_adjoint(v, u, shape):
    """Transpose of T -> T(x + u(x)) applied to v: scatter into the 4 taps."""
    H, W = shape
    h, w = u.shape[1:]
    yy, xx = np.mgrid[0:h, 0:w]
    cx, fx = split_offset(u[0])
    cy, fy = split_offset(u[1])
    x0, y0 = xx + cx, yy + cy
    xa, xb = np.clip(x0, 0, W - 1), np.clip(x0 + 1, 0, W - 1)
    ya, yb = np.clip(y0, 0, H - 1), np.clip(y0 + 1, 0, H - 1)
    out = np.zeros(shape)
    np.add.at(out, (ya, xa), v * (1 - fx) * (1 - fy))
    np.add.at(out, (ya, xb), v * fx * (1 - fy))
    np.add.at(out, (yb, xa), v * (1 - fx) * fy)
    np.add.at(out, (yb, xb), v * fx * fy)
    return out


def restrict_image_adjoint(gc):
    """Transpose of the 2x2 block mean: each fine pixel gets 1/4 of its parent."""
    return 0.25 * np.repeat(np.repeat(gc, 2, axis=0), 2, axis=1)


def restrict_field_adjoint(gc):
    return np.stack([0.5 * restrict_image_adjoint(gc[0]), 0.5 * restrict_image_adjoint(gc[1])])


def restrict_frame_adjoint(gc, shape):
    """Transpose of the binomial frame restriction: every coarse value is
    scattered with weight w_a w_b into the (clamped) fine taps it was formed
    from."""
    H, W = shape
    h, w = gc.shape
    ys, xs = np.arange(h), np.arange(w)
    out = np.zeros(shape)
    for a in range(6):
        ya = np.clip(2 * ys + a - 2, 0, H - 1)
        for b in range(6):
            xb = np.clip(2 * xs + b - 2, 0, W - 1)
            Y, X = np.meshgrid(ya, xb, indexing="ij")
            np.add.at(out, (Y, X), BINOMIAL6[a] * BINOMIAL6[b] * gc)
    return out


def _levels(Ia, u, Ib, levels):
    A, U, B = [np.asarray(Ia, np.float64)], [np.asarray(u, np.float64)], [np.asarray(Ib, np.float64)]
    for _ in range(levels - 1):
        A.append(restrict_frame(A[-1]))
        U.append(restrict_field(U[-1]))
        B.append(restrict_frame(B[-1]))
    return A, U, B


def pyramid_energy(Ia, u, Ib, lam, levels=1):
    A, U, B = _levels(Ia, u, Ib, levels)
    return sum(energy(B[l], A[l], U[l], lam) for l in range(levels))


def pyramid_energy_grads(Ia, u, Ib, lam, levels=1):
    """(E, dE/dIa, dE/du, dE/dIb)."""
    A, U, B = _levels(Ia, u, Ib, levels)
    E = 0.0
    gA = gU = gB = None
    for l in range(levels - 1, -1, -1):
        El, gu = energy_and_gradient(B[l], A[l], U[l], lam)
        r = sample_displaced(A[l], U[l])[0] - B[l]
        ga = warp_adjoint(2 * r, U[l], A[l].shape)
        gb = -2 * r
        E += El
        if gA is None:
            gA, gU, gB = ga, gu, gb
        else:
            gA = ga + restrict_frame_adjoint(gA, A[l].shape)
            gU = gu + restrict_field_adjoint(gU)
            gB = gb + restrict_frame_adjoint(gB, B[l].shape)
    return E, gA, gU, gB
