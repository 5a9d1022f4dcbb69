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

Frame pyramid.  Each coarser level of a frame is a separable binomial
low-pass of the level below, sampled at the centres of its 2x2 blocks (the
restriction of images is not specified by the paper beyond "multilevel";
a 2x2 block mean would alias periodic content that the coarse grid cannot
resolve, see ``restrict_frame``).  Displacements are restricted by half the
2x2 block mean.

Storage precision (two modes).  ``storage="f32"``: every value the solver
keeps - frame pyramid levels, the initial guess on the coarsest level, each
gradient-descent iterate, each prolongation - is the float64 result rounded
once to float32, and the integer cell of a bilinear sample is decided on the
float32 value of the displacement.  The paper fixes no precision for these
values; this mode exists so that a GPU implementation that stores its fields
in float32 (and computes in float64) can be compared with the oracle bit for
bit.  ``storage="f64"``: plain float64 throughout - the frames (given as
float32 data) are the only rounded values.  The two modes differ by the
float32 roundings of the stored fields and their consequences.
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


def store(a, storage="f32"):
    """A value as the solver keeps it: rounded to float32 (``"f32"``) or the
    float64 result itself (``"f64"``)."""
    if storage == "f32":
        return f32(a)
    if storage == "f64":
        return np.array(a, dtype=np.float64)
    raise ValueError(f"unknown storage mode {storage!r}")


def split_offset(off, storage="f32"):
    """Integer cell offset and the float64 remainder.  In float32 storage the
    cell is decided on the float32 value of the offset, else on the value."""
    off = np.asarray(off, dtype=np.float64)
    if storage == "f32":
        cell = np.floor(off.astype(np.float32)).astype(np.float64)
    else:
        cell = np.floor(off)
    return cell.astype(np.int64), off - cell


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


def sample_displaced(img, u, storage="f32"):
    """img(x + u(x)) for every pixel x of u's grid, with derivatives."""
    h, w = u.shape[1:]
    yy, xx = np.mgrid[0:h, 0:w]
    cx, fx = split_offset(u[0], storage)
    cy, fy = split_offset(u[1], storage)
    return bilinear(img, xx + cx, yy + cy, fx, fy)


def warp(T, u, storage="f32"):
    """(T o phi)(x) = T(x + u(x)) (the deformed template)."""
    return sample_displaced(T, u, storage)[0]


# ----------------------------------------------------------------------------
# Energy and gradient
# ----------------------------------------------------------------------------

def energy(R, T, u, lam, storage="f32"):
    """E(u): SSD of the warped template against R plus lam * |grad u|^2."""
    r = warp(T, u, storage) - R
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


def energy_and_gradient(R, T, u, lam, storage="f32"):
    """E(u) and dE/du (exact away from integer sample positions)."""
    s, dsx, dsy = sample_displaced(T, u, storage)
    r = s - R
    E = energy(R, T, u, lam, storage)
    g = np.empty_like(u)
    g[0] = 2 * r * dsx + 2 * lam * neighbour_differences(u[0])
    g[1] = 2 * r * dsy + 2 * lam * neighbour_differences(u[1])
    return E, g


# ----------------------------------------------------------------------------
# Pyramid: restriction and prolongation
# ----------------------------------------------------------------------------

def restrict_image(F):
    """Mean over 2x2 blocks (the restriction of displacement fields)."""
    return 0.25 * (F[0::2, 0::2] + F[0::2, 1::2] + F[1::2, 0::2] + F[1::2, 1::2])


def restrict_field(u):
    """Displacement on the next coarser grid: half the 2x2 block mean (px shrink by 2)."""
    return np.stack([0.5 * restrict_image(u[0]), 0.5 * restrict_image(u[1])])


# Per-axis weights of the frame restriction: the binomial coefficients of
# (1 + z)^5 over 32.  Their frequency response is cos(pi f)^5 (f in cycles per
# fine pixel): 1 at f = 0, 0.18 at f = 1/4 (the coarse grid's Nyquist
# frequency), 0 at f = 1/2; the 2x2 block mean, the binomial of order 1, has
# cos(pi f) = 0.71 at f = 1/4.
BINOMIAL6 = (1 / 32, 5 / 32, 10 / 32, 10 / 32, 5 / 32, 1 / 32)


def restrict_frame(F):
    """Next coarser level of a frame: at coarse pixel (Y, X)

        sum_{a=0..5} w_a sum_{b=0..5} w_b F[2Y + a - 2][2X + b - 2]

    with w = BINOMIAL6 and edge-clamped taps, i.e. the separable binomial
    low-pass centred on (2Y + 1/2, 2X + 1/2), the centre of the 2x2 block the
    coarse pixel covers (the geometry of the block mean and of the
    prolongation).  The paper's multilevel scheme (Section 2.3.1) does not say
    how images are coarsened.  A lattice whose period is at most two pixels
    of the coarse grid (at least 1/4 cycle per fine pixel) cannot be
    represented there: at exactly two pixels the sampled lattice no longer
    tells a shift from its mirror image, below two it aliases to a lattice
    that moves the other way, and a solve on that level pulls the
    displacement away from the true shift.  The 2x2 block mean passes such
    content at up to 71% of its amplitude, the order-5 binomial at most 18%,
    while it keeps 67% of a lattice of four coarse pixels per period.

    Evaluation order: per row a, the weighted taps summed over b in
    increasing order; then the weighted row sums over a in increasing order
    (every product is exact: the weights have three significant bits).
    """
    H, W = F.shape
    ys = np.arange(H // 2)
    xs = np.arange(W // 2)
    out = None
    for a in range(6):
        ya = np.clip(2 * ys + a - 2, 0, H - 1)
        row = None
        for b in range(6):
            xb = np.clip(2 * xs + b - 2, 0, W - 1)
            t = BINOMIAL6[b] * F[np.ix_(ya, xb)]
            row = t if row is None else row + t
        t = BINOMIAL6[a] * row
        out = t if out is None else out + t
    return out


def pyramid(F, levels, storage="f32"):
    """Stored frame pyramid: level 0 is the frame, each coarser level the
    binomial restriction of the stored level below, stored."""
    out = [store(F, storage)]
    for _ in range(levels - 1):
        out.append(store(restrict_frame(out[-1]), storage))
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


def solve_level(R, T, u0, tau, lam, max_iter, fixed_iter, rel_tol, storage="f32"):
    """Gradient descent on one pyramid level.

    Iteration t evaluates E_t and g_t at u_t.  Unless the iteration count is
    fixed, the solve returns u_t as soon as t > 0 and the relative decrease
    E_{t-1} - E_t is at most rel_tol * E_{t-1} (this includes any increase);
    otherwise it steps u_{t+1} = u_t - tau g_t (stored in float32).  After
    max_iter steps it returns u_{max_iter}.  A non-finite energy stops the
    solve at once.  Iterates are stored per ``storage``.
    """
    u = store(u0, storage)
    e_prev = None
    energies = []
    for t in range(max_iter):
        E, g = energy_and_gradient(R, T, u, lam, storage)
        energies.append(E)
        if not np.isfinite(E):
            return LevelResult(u, t, STATUS_NONFINITE, energies)
        if not fixed_iter and e_prev is not None and (e_prev - E) <= rel_tol * e_prev:
            return LevelResult(u, t, STATUS_OK, energies)
        e_prev = E
        u = store(u - tau * g, storage)
    status = STATUS_OK if fixed_iter else STATUS_MAXITER
    return LevelResult(u, max_iter, status, energies)


@dataclass
class RegResult:
    u: np.ndarray          # [2][H][W] at full resolution
    iters: list            # per level, level 0 = finest
    status: int


def register(R_pyr, T_pyr, u0, params, storage="f32"):
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
        u = store(u, storage)
    iters = [0] * L
    status = STATUS_OK
    for lvl in range(L - 1, -1, -1):
        if lvl < L - 1:
            h, w = R_pyr[lvl].shape
            u = store(prolong_field(u, h, w), storage)
        res = solve_level(R_pyr[lvl], T_pyr[lvl], u, params.tau, params.lam,
                          params.max_iter, params.fixed_iter, params.rel_tol, storage)
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

def compose(u_ij, u_jk, storage="f32"):
    """Displacement of phi_jk o phi_ij: u_ij(x) + u_jk(x + u_ij(x))."""
    h, w = u_ij.shape[1:]
    yy, xx = np.mgrid[0:h, 0:w]
    cx, fx = split_offset(u_ij[0], storage)
    cy, fy = split_offset(u_ij[1], storage)
    out = np.empty_like(u_ij, dtype=np.float64)
    for c in range(2):
        out[c] = u_ij[c] + bilinear(u_jk[c], xx + cx, yy + cy, fx, fy)[0]
    return out


def op_A(pyrs, i, params, storage="f32"):
    """A(f_i, f_{i+1}): register consecutive frames from the identity."""
    return register(pyrs[i], pyrs[i + 1], None, params, storage)


def op_B(pyrs, i, k, u_ij, u_jk, params, storage="f32"):
    """B(phi_ij, phi_jk) = phi_ik: register f_i and f_k from the composition."""
    return register(pyrs[i], pyrs[k], compose(u_ij, u_jk, storage), params, storage)
