"""Rigid registration with normalized cross-correlation, CPU float64 oracle.
TEST INFRASTRUCTURE ONLY.

The paper's own operator (Definition "Image registration problem",
Section 2.3.1): phi is a rigid motion, a rotation by an angle alpha and a
translation G, and the distance is the normalized cross-correlation of the
reference R and the deformed template T o phi, minimised by a multilevel
gradient flow.  Readings (the paper fixes none of these details):

* rotation about the image centre c = ((w - 1) / 2, (h - 1) / 2):
      phi(x) = Rot(alpha) (x - c) + c + G,  theta = (alpha, G_x, G_y);
* energy E(theta) = 1 - NCC(R, T o phi),
      NCC = S_ab / sqrt(S_aa S_bb),  S_ab = sum (a - mean a)(b - mean b), ...
  with a = R(x), b = T(phi(x)) bilinear with edge-clamped taps; E = 1 when
  either image is constant (S_aa S_bb = 0), with zero gradient;
* gradient flow in the metric diag(r^2, 1, 1), r^2 = the mean squared
  distance of the pixels from c: theta <- theta - tau (grad_alpha / r^2,
  grad_Gx, grad_Gy), the same stopping rule as the dense operator;
* multilevel: G halves per coarser level, alpha is unchanged (the centres of
  the levels correspond, x_fine = 2 x_coarse + 1/2);
* composition phi_jk o phi_ij: alpha = alpha_ij + alpha_jk,
  G = Rot(alpha_jk) G_ij + G_jk.

The gradient of NCC with respect to b(x) is
  (a - mean a) / sqrt(S_aa S_bb) - NCC (b - mean b) / S_bb,
so dE/dtheta_p = -sum_x that * dT/dp(phi(x)), with dphi/dalpha =
Rot'(alpha)(x - c) and dphi/dG = identity.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .registration import STATUS_MAXITER, STATUS_NONFINITE, STATUS_OK, bilinear, pyramid


def centre(h, w):
    return (w - 1) / 2.0, (h - 1) / 2.0


def radius2(h, w):
    """Mean squared distance of the pixel centres from the image centre."""
    return ((w * w - 1) + (h * h - 1)) / 12.0


def rigid_positions(theta, h, w):
    """phi(x) for every pixel x = (column, row) of an h x w grid."""
    a, gx, gy = theta
    cx, cy = centre(h, w)
    yy, xx = np.mgrid[0:h, 0:w]
    dx, dy = xx - cx, yy - cy
    ca, sa = np.cos(a), np.sin(a)
    return ca * dx - sa * dy + cx + gx, sa * dx + ca * dy + cy + gy, dx, dy


def sample_at(img, px, py):
    """Bilinear value and position derivatives of img at (px, py) (float64
    positions; the cell is their floor)."""
    x0 = np.floor(px)
    y0 = np.floor(py)
    return bilinear(img, x0.astype(np.int64), y0.astype(np.int64), px - x0, py - y0)


def ncc_energy_grad(R, T, theta):
    """E = 1 - NCC(R, T o phi) and dE/dtheta."""
    h, w = R.shape
    px, py, dx, dy = rigid_positions(theta, h, w)
    b, bx, by = sample_at(T, px, py)
    a = R
    da = a - a.mean()
    db = b - b.mean()
    saa, sbb, sab = float(np.sum(da * da)), float(np.sum(db * db)), float(np.sum(da * db))
    if not saa * sbb > 0:
        return 1.0, np.zeros(3)
    ncc = sab / np.sqrt(saa * sbb)
    dn_db = da / np.sqrt(saa * sbb) - ncc * db / sbb
    al = theta[0]
    dpx_da = -np.sin(al) * dx - np.cos(al) * dy
    dpy_da = np.cos(al) * dx - np.sin(al) * dy
    g = np.array([-np.sum(dn_db * (bx * dpx_da + by * dpy_da)), -np.sum(dn_db * bx), -np.sum(dn_db * by)])
    return 1.0 - ncc, g


@dataclass
class RigidLevel:
    theta: np.ndarray
    iters: int
    status: int


def solve_level(R, T, theta0, tau, max_iter, fixed_iter, rel_tol):
    """Gradient flow on one level in the metric diag(r^2, 1, 1); the stopping
    rule of the dense operator (iteration t evaluates E_t at theta_t; for t > 0
    the level returns theta_t once E_{t-1} - E_t <= rel_tol E_{t-1})."""
    h, w = R.shape
    metric = np.array([radius2(h, w), 1.0, 1.0])
    theta = np.array(theta0, dtype=np.float64)
    e_prev = None
    for t in range(max_iter):
        E, g = ncc_energy_grad(R, T, theta)
        if not np.isfinite(E):
            return RigidLevel(theta, t, STATUS_NONFINITE)
        if not fixed_iter and e_prev is not None and (e_prev - E) <= rel_tol * e_prev:
            return RigidLevel(theta, t, STATUS_OK)
        e_prev = E
        theta = theta - tau * g / metric
    return RigidLevel(theta, max_iter, STATUS_OK if fixed_iter else STATUS_MAXITER)


@dataclass
class RigidResult:
    theta: np.ndarray      # (alpha, G_x, G_y) at full resolution
    iters: list            # per level, level 0 = finest
    status: int


def register(R_pyr, T_pyr, theta0, params):
    """Multilevel rigid registration: theta0 (identity when None) moved to the
    coarsest level (G / 2 per level), solved there, carried to each finer
    level (G * 2) and solved again."""
    L = params.levels
    theta = np.zeros(3) if theta0 is None else np.array(theta0, dtype=np.float64)
    theta = np.array([theta[0], theta[1] / 2 ** (L - 1), theta[2] / 2 ** (L - 1)])
    iters = [0] * L
    status = STATUS_OK
    for lvl in range(L - 1, -1, -1):
        if lvl < L - 1:
            theta = np.array([theta[0], 2.0 * theta[1], 2.0 * theta[2]])
        res = solve_level(R_pyr[lvl], T_pyr[lvl], theta, params.tau, params.max_iter, params.fixed_iter,
                          params.rel_tol)
        theta, iters[lvl] = res.theta, res.iters
        status |= res.status
        if res.status & STATUS_NONFINITE:
            return RigidResult(np.full(3, np.nan), iters, status)
    return RigidResult(theta, iters, status)


def compose(th_ij, th_jk):
    """theta of phi_jk o phi_ij (same centre): angles add,
    G = Rot(alpha_jk) G_ij + G_jk."""
    a1, g1x, g1y = th_ij
    a2, g2x, g2y = th_jk
    c, s = np.cos(a2), np.sin(a2)
    return np.array([a1 + a2, c * g1x - s * g1y + g2x, s * g1x + c * g1y + g2y])


def run_scan(frames, params, ops, M):
    """Pairwise registrations from the identity, then the plan's operator
    applications B(theta_ij, theta_jk) = register(f_i, f_k, compose(...)).
    Returns (phi0 [M][3], pairs [M][3], iters [M + n_ops][L])."""
    from . import plans
    pyrs = [pyramid(np.asarray(f, dtype=np.float64), params.levels) for f in frames]
    pairs, iters = [], []
    for k in range(1, M + 1):
        r = register(pyrs[k - 1], pyrs[k], None, params)
        pairs.append(r.theta)
        iters.append(r.iters)
    node = {m: pairs[m] for m in range(M)}
    for row in ops:
        i, k = int(row[4]), int(row[6])
        r = register(pyrs[i], pyrs[k], compose(node[int(row[2])], node[int(row[3])]), params)
        node[int(row[1])] = r.theta
        iters.append(r.iters)
    fin = plans.final_nodes(ops, M)
    return np.stack([node[int(fin[k])] for k in range(M)]), np.stack(pairs), np.array(iters)
