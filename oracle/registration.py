"""Registration operator, CPU float64 oracle.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the library never imports it.  It shares no code with the HIP
path.

The paper's registration problem (Section 2.3.1, Definition "Image
registration problem"): find phi minimising D(R, T o phi), solved by gradient
flow on a multilevel (coarse-to-fine) scheme.  The operator computed here is
the dense-displacement form used throughout this project:

    phi(x) = x + u(x),  u = (u_x, u_y) on the pixel grid,
    E(u) = sum_x (T(x + u(x)) - R(x))^2
         + lam * sum_c sum_x [ (u_c(x+e1) - u_c(x))^2 + (u_c(x+e2) - u_c(x))^2 ]
    (forward differences, only pairs inside the grid: Neumann boundary),

minimised by Euclidean gradient descent u <- u - tau * grad E on a 2x2 box
pyramid.  T is sampled bilinearly with edge-clamped taps.

Array conventions: images [H][W] (row y, column x), displacements [2][H][W]
with plane 0 = x and plane 1 = y, pixel centres on integer coordinates.

Storage precision.  Stored data are 32-bit floats: the frames, their pyramid
levels, and every displacement field the solver keeps (the initial guess on
the coarsest level, each gradient-descent iterate, each prolongation) - the
paper moves a deformation as single-precision floats (Section 5: 20 bytes of
deformation data and indices per message).  All arithmetic is float64; a
stored value is the float64 result rounded to float32 (``f32``).  The integer
part of a displacement (which bilinear cell a sample falls in) is therefore
decided on a float32 value.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

STATUS_OK = 0
STATUS_MAXITER = 1     # a level reached its iteration cap without meeting the rule
STATUS_NONFINITE = 2   # the energy became NaN or infinite; the task stopped


# ----------------------------------------------------------------------------
# Bilinear sampling
# ----------------------------------------------------------------------------

def f32(a):
    """Round to the float32 storage format (returned as float64)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def split_offset(off):
    """Integer cell offset (decided in float32) and the float64 remainder."""
    cell = np.floor(np.asarray(off, dtype=np.float64).astype(np.float32)).astype(np.float64)
    return cell.astype(np.int64), np.asarray(off, dtype=np.float64) - cell


def bilinear(img, xi, yi, wx, wy):
    """Bilinear value and its derivatives w.r.t. the sample position.

    The sample sits at (xi + wx, yi + wy) with integer cell (xi, yi).  The four
    taps are clamped to the image (replicate boundary), so a sample outside the
    image takes the edge value and has zero derivative across the edge.
    Returns (S, dS/dpx, dS/dpy).
    """
    H, W = img.shape
    xa = np.clip(xi, 0, W - 1)
    xb = np.clip(xi + 1, 0, W - 1)
    ya = np.clip(yi, 0, H - 1)
    yb = np.clip(yi + 1, 0, H - 1)
    i00 = img[ya, xa]
    i01 = img[ya, xb]
    i10 = img[yb, xa]
    i11 = img[yb, xb]
    s = (1 - wy) * ((1 - wx) * i00 + wx * i01) + wy * ((1 - wx) * i10 + wx * i11)
    dsx = (1 - wy) * (i01 - i00) + wy * (i11 - i10)
    dsy = (1 - wx) * (i10 - i00) + wx * (i11 - i01)
    return s, dsx, dsy


def sample_displaced(img, u):
    """img(x + u(x)) for every pixel x of u's grid, with derivatives."""
    h, w = u.shape[1:]
    yy, xx = np.mgrid[0:h, 0:w]
    cx, fx = split_offset(u[0])
    cy, fy = split_offset(u[1])
    return bilinear(img, xx + cx, yy + cy, fx, fy)


def warp(T, u):
    """(T o phi)(x) = T(x + u(x)) (the deformed template)."""
    return sample_displaced(T, u)[0]


# ----------------------------------------------------------------------------
# Energy and gradient
# ----------------------------------------------------------------------------

def energy(R, T, u, lam):
    """E(u): SSD of the warped template against R plus lam * |grad u|^2."""
    r = warp(T, u) - R
    reg = 0.0
    for c in range(2):
        dx = u[c][:, 1:] - u[c][:, :-1]   # pairs (x, x+e1) inside the grid
        dy = u[c][1:, :] - u[c][:-1, :]   # pairs (x, x+e2) inside the grid
        reg += np.sum(dx * dx) + np.sum(dy * dy)
    return float(np.sum(r * r) + lam * reg)


def neighbour_differences(v):
    """sum over the in-grid 4-neighbours n of x of (v(x) - v(n))."""
    out = np.zeros_like(v)
    out[:, 1:] += v[:, 1:] - v[:, :-1]    # left neighbour exists
    out[:, :-1] += v[:, :-1] - v[:, 1:]   # right neighbour exists
    out[1:, :] += v[1:, :] - v[:-1, :]    # upper neighbour exists
    out[:-1, :] += v[:-1, :] - v[1:, :]   # lower neighbour exists
    return out


def energy_and_gradient(R, T, u, lam):
    """E(u) and dE/du (exact away from integer sample positions)."""
    s, dsx, dsy = sample_displaced(T, u)
    r = s - R
    E = energy(R, T, u, lam)
    g = np.empty_like(u)
    g[0] = 2 * r * dsx + 2 * lam * neighbour_differences(u[0])
    g[1] = 2 * r * dsy + 2 * lam * neighbour_differences(u[1])
    return E, g


# ----------------------------------------------------------------------------
# Pyramid: restriction and prolongation
# ----------------------------------------------------------------------------

def restrict_image(F):
    """Next coarser pyramid level: mean over 2x2 blocks."""
    return 0.25 * (F[0::2, 0::2] + F[0::2, 1::2] + F[1::2, 0::2] + F[1::2, 1::2])


def restrict_field(u):
    """Displacement on the next coarser grid: half the 2x2 block mean (px shrink by 2)."""
    return np.stack([0.5 * restrict_image(u[0]), 0.5 * restrict_image(u[1])])


def pyramid(F, levels):
    """Stored frame pyramid: each level is the 2x2 block mean of the stored
    level below, rounded to float32."""
    out = [f32(F)]
    for _ in range(levels - 1):
        out.append(f32(restrict_image(out[-1])))
    return out


def prolong_field(uc, h, w):
    """Displacement on the finer h x w grid: 2 * u_c sampled at ((x-1/2)/2, (y-1/2)/2)."""
    yy, xx = np.mgrid[0:h, 0:w]
    px = (xx - 0.5) / 2.0
    py = (yy - 0.5) / 2.0
    x0 = np.floor(px).astype(np.int64)
    y0 = np.floor(py).astype(np.int64)
    wx, wy = px - x0, py - y0
    return np.stack([2.0 * bilinear(uc[c], x0, y0, wx, wy)[0] for c in range(2)])


# ----------------------------------------------------------------------------
# Gradient descent on one level, multilevel solve
# ----------------------------------------------------------------------------

@dataclass
class LevelResult:
    u: np.ndarray
    iters: int
    status: int
    energies: list


def solve_level(R, T, u0, tau, lam, max_iter, fixed_iter, rel_tol):
    """Gradient descent on one pyramid level.

    Iteration t evaluates E_t and g_t at u_t.  Unless the iteration count is
    fixed, the solve returns u_t as soon as t > 0 and the relative decrease
    E_{t-1} - E_t is at most rel_tol * E_{t-1} (this includes any increase);
    otherwise it steps u_{t+1} = u_t - tau g_t (stored in float32).  After
    max_iter steps it returns u_{max_iter}.  A non-finite energy stops the
    solve at once.
    """
    u = f32(u0)
    e_prev = None
    energies = []
    for t in range(max_iter):
        E, g = energy_and_gradient(R, T, u, lam)
        energies.append(E)
        if not np.isfinite(E):
            return LevelResult(u, t, STATUS_NONFINITE, energies)
        if not fixed_iter and e_prev is not None and (e_prev - E) <= rel_tol * e_prev:
            return LevelResult(u, t, STATUS_OK, energies)
        e_prev = E
        u = f32(u - tau * g)
    status = STATUS_OK if fixed_iter else STATUS_MAXITER
    return LevelResult(u, max_iter, status, energies)


@dataclass
class RegResult:
    u: np.ndarray          # [2][H][W] at full resolution
    iters: list            # per level, level 0 = finest
    status: int


def register(R_pyr, T_pyr, u0, params):
    """Multilevel registration Reg(R, T, u0).

    The initial guess (zero when u0 is None) is restricted to the coarsest
    level and solved there; each finer level starts from the prolongation of
    the coarser result.  The same tau and lam are used on every level.
    """
    L = params.levels
    if u0 is None:
        hc, wc = R_pyr[L - 1].shape
        u = np.zeros((2, hc, wc))
    else:
        u = np.array(u0, dtype=np.float64)
        for _ in range(L - 1):
            u = restrict_field(u)
        u = f32(u)
    iters = [0] * L
    status = STATUS_OK
    for lvl in range(L - 1, -1, -1):
        if lvl < L - 1:
            h, w = R_pyr[lvl].shape
            u = f32(prolong_field(u, h, w))
        res = solve_level(R_pyr[lvl], T_pyr[lvl], u, params.tau, params.lam,
                          params.max_iter, params.fixed_iter, params.rel_tol)
        u, iters[lvl] = res.u, res.iters
        status |= res.status
        if res.status & STATUS_NONFINITE:
            # a diverged registration has no meaningful field: report NaN
            h0, w0 = R_pyr[0].shape
            u = np.full((2, h0, w0), np.nan)
            break
    return RegResult(u, iters, status)


# ----------------------------------------------------------------------------
# Series operators A and B (Section 2.3.2) and the scan operator (Section 3)
# ----------------------------------------------------------------------------

def compose(u_ij, u_jk):
    """Displacement of phi_jk o phi_ij: u_ij(x) + u_jk(x + u_ij(x))."""
    h, w = u_ij.shape[1:]
    yy, xx = np.mgrid[0:h, 0:w]
    cx, fx = split_offset(u_ij[0])
    cy, fy = split_offset(u_ij[1])
    out = np.empty_like(u_ij, dtype=np.float64)
    for c in range(2):
        out[c] = u_ij[c] + bilinear(u_jk[c], xx + cx, yy + cy, fx, fy)[0]
    return out


def op_A(pyrs, i, params):
    """A(f_i, f_{i+1}): register consecutive frames from the identity."""
    return register(pyrs[i], pyrs[i + 1], None, params)


def op_B(pyrs, i, k, u_ij, u_jk, params):
    """B(phi_ij, phi_jk) = phi_ik: register f_i and f_k from the composition."""
    return register(pyrs[i], pyrs[k], compose(u_ij, u_jk), params)
