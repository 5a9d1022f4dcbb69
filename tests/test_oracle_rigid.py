"""Pins of the rigid normalized-cross-correlation oracle (the paper's own
operator, Section 2.3.1) against facts it does not compute itself: SciPy's
bilinear interpolation and NumPy's correlation coefficient for the energy,
NumPy's rot90 for the direction and centre of the rotation, finite
differences for the gradient, direct application of the two maps for the
composition, brute force for the metric radius, and recovery of known
motions of the synthetic lattice."""
from dataclasses import replace

import numpy as np
import pytest
import torch
from scipy import ndimage

from oracle import plans
from oracle import rigid
from oracle.registration import pyramid
from synth import RIGID_TAU, SeriesSpec, get_config, lattice_image, rigid_pair, rigid_series
from synth.configs import SolverParams


def _smooth_image(h, w, seed):
    rng = np.random.default_rng(seed)
    img = rng.normal(size=(h, w))
    return ndimage.gaussian_filter(img, 2.0, mode="nearest")


def _lattice(h, w, origin=(3.3, 2.1), spacing=8.0):
    spec = SeriesSpec(1, h, w, spacing=spacing, noise=0.0)
    yy, xx = torch.meshgrid(torch.arange(h, dtype=torch.float64), torch.arange(w, dtype=torch.float64),
                            indexing="ij")
    return lattice_image(spec, np.array(origin), xx, yy).numpy()


# --------------------------------------------------------------- the energy

@pytest.mark.parametrize("theta", [(0.0, 0.0, 0.0), (0.13, 1.7, -2.4), (-0.6, -7.25, 3.5), (0.02, 40.0, -3.0)])
def test_energy_is_one_minus_pearson_of_scipy_warp(theta):
    """E = 1 - corrcoef(R, T o phi) with T o phi from scipy's order-1
    map_coordinates (edge-replicating), an independent bilinear sampler."""
    h, w = 28, 36
    R, T = _smooth_image(h, w, 1), _smooth_image(h, w, 2)
    px, py, _, _ = rigid.rigid_positions(np.array(theta), h, w)
    b = ndimage.map_coordinates(T, [py.ravel(), px.ravel()], order=1, mode="nearest").reshape(h, w)
    want = 1.0 - np.corrcoef(R.ravel(), b.ravel())[0, 1]
    E, _ = rigid.ncc_energy_grad(R, T, np.array(theta))
    assert abs(E - want) < 1e-12


def test_rotation_by_quarter_turn_about_centre_is_rot90():
    """alpha = pi/2 maps the pixel grid of a square image onto itself:
    T o phi is NumPy's counter-clockwise rot90 of T (this fixes the sign of
    the angle, the centre and the axis order)."""
    n = 17
    T = _smooth_image(n, n, 3)
    px, py, _, _ = rigid.rigid_positions(np.array([np.pi / 2, 0.0, 0.0]), n, n)
    b, _, _ = rigid.sample_at(T, px, py)
    np.testing.assert_allclose(b, np.rot90(T, 1), atol=1e-12)


def test_integer_translation_is_a_shift():
    h, w = 20, 24
    T = _smooth_image(h, w, 4)
    px, py, _, _ = rigid.rigid_positions(np.array([0.0, 3.0, -2.0]), h, w)
    b, _, _ = rigid.sample_at(T, px, py)
    np.testing.assert_allclose(b[2:, :w - 3], T[:h - 2, 3:], atol=1e-12)


def test_energy_invariances_and_extremes():
    h, w = 24, 24
    R, T = _smooth_image(h, w, 5), _smooth_image(h, w, 6)
    th = np.array([0.05, 0.7, -1.1])
    E, g = rigid.ncc_energy_grad(R, T, th)
    E2, g2 = rigid.ncc_energy_grad(3.0 * R - 1.0, 2.5 * T + 7.0, th)   # NCC is invariant to gain and offset
    assert abs(E - E2) < 1e-12
    np.testing.assert_allclose(g, g2, rtol=1e-9, atol=1e-13)
    E0, g0 = rigid.ncc_energy_grad(R, R, np.zeros(3))
    assert abs(E0) < 1e-14 and np.abs(g0).max() < 1e-9
    Em, _ = rigid.ncc_energy_grad(R, -R, np.zeros(3))
    assert abs(Em - 2.0) < 1e-14
    Ec, gc = rigid.ncc_energy_grad(R, np.full((h, w), 0.25), th)   # constant template: E = 1, no gradient
    assert Ec == 1.0 and not gc.any()


@pytest.mark.parametrize("theta", [(0.0, 0.3, -0.4), (0.21, 1.37, 0.62), (-0.4, -2.2, 5.3)])
def test_gradient_matches_central_differences(theta):
    h, w = 26, 30
    R, T = _smooth_image(h, w, 7), _smooth_image(h, w, 8)
    th = np.array(theta)
    _, g = rigid.ncc_energy_grad(R, T, th)
    for p, step in enumerate((1e-6, 1e-5, 1e-5)):
        e = np.zeros(3)
        e[p] = step
        fd = (rigid.ncc_energy_grad(R, T, th + e)[0] - rigid.ncc_energy_grad(R, T, th - e)[0]) / (2 * step)
        assert abs(fd - g[p]) <= 1e-5 * max(1.0, abs(g[p])), (p, fd, g[p])


def test_metric_radius_is_mean_squared_distance_from_centre():
    for h, w in ((8, 8), (17, 40), (256, 256)):
        yy, xx = np.mgrid[0:h, 0:w]
        cx, cy = rigid.centre(h, w)
        brute = np.mean((xx - cx) ** 2 + (yy - cy) ** 2)
        assert abs(rigid.radius2(h, w) - brute) < 1e-9 * brute


# ---------------------------------------------------------- the composition

@pytest.mark.parametrize("t1,t2", [((0.1, 2.0, -1.0), (0.0, 0.0, 0.0)), ((0.0, 0.0, 0.0), (-0.3, 1.5, 0.25)),
                                   ((0.37, -4.0, 2.5), (-0.12, 3.25, 1.75)), ((1.2, 0.5, 0.5), (2.1, -6.0, 0.0))])
def test_compose_is_the_map_phi_jk_after_phi_ij(t1, t2):
    """compose(theta_ij, theta_jk) moves every pixel where phi_jk moves the
    position phi_ij gave it (the maps applied one after the other)."""
    h, w = 15, 22
    px, py, _, _ = rigid.rigid_positions(np.array(t1), h, w)
    a, gx, gy = t2
    cx, cy = rigid.centre(h, w)
    qx = np.cos(a) * (px - cx) - np.sin(a) * (py - cy) + cx + gx
    qy = np.sin(a) * (px - cx) + np.cos(a) * (py - cy) + cy + gy
    rx, ry, _, _ = rigid.rigid_positions(rigid.compose(np.array(t1), np.array(t2)), h, w)
    np.testing.assert_allclose(rx, qx, atol=1e-12)
    np.testing.assert_allclose(ry, qy, atol=1e-12)


# ------------------------------------------------------------ the minimiser

def test_identical_frames_stay_at_identity():
    f = _lattice(32, 32)
    pyr = pyramid(f, 2)
    r = rigid.register(pyr, pyr, None, SolverParams(levels=2, max_iter=30, tau=RIGID_TAU))
    assert np.abs(r.theta).max() < 1e-9
    assert r.status == 0


def test_fixed_iterations_are_exact():
    f0, f1 = rigid_pair(SeriesSpec(2, 32, 32, noise=0.0), (0.01, 0.5, -0.3))
    p = SolverParams(levels=2, max_iter=7, fixed_iter=True, tau=RIGID_TAU)
    pa, pb = pyramid(f0.double().numpy(), 2), pyramid(f1.double().numpy(), 2)
    r = rigid.register(pa, pb, None, p)
    assert r.iters == [7, 7] and r.status == 0


@pytest.mark.parametrize("theta", [(0.02, 1.3, -0.7), (-0.035, -2.1, 0.4), (0.0, 0.45, 0.8)])
def test_recovers_known_motion_of_clean_lattice(theta):
    """Noise-free lattice moved by a known rigid motion: the multilevel flow
    lands within 0.05 px of it (angle measured as alpha * r at the mean
    radius); the residual is the bias of bilinear resampling.  Acceptance
    threshold proposed here, the paper prints none."""
    spec = SeriesSpec(2, 64, 64, spacing=8.0, sigma=1.5, noise=0.0, seed=17)
    R, T = rigid_pair(spec, theta)
    p = SolverParams(levels=2, max_iter=200, tau=RIGID_TAU)
    r = rigid.register(pyramid(R.double().numpy(), 2), pyramid(T.double().numpy(), 2), None, p)
    e = r.theta - np.array(theta)
    assert abs(e[0]) * np.sqrt(rigid.radius2(64, 64)) < 0.05
    assert np.abs(e[1:]).max() < 0.05
    assert r.status == 0


def test_result_is_a_local_minimum_of_the_energy():
    """Converged flow (fixed 400 iterations): no parameter step of 1e-3 px
    (1e-3 / r rad for the angle) lowers the energy."""
    spec = SeriesSpec(2, 48, 48, noise=0.05, seed=23)
    R, T = rigid_pair(spec, (0.015, -0.8, 1.1))
    Rd, Td = R.double().numpy(), T.double().numpy()
    p = SolverParams(levels=1, max_iter=400, fixed_iter=True, tau=RIGID_TAU)
    th = rigid.register([Rd], [Td], None, p).theta
    E0, _ = rigid.ncc_energy_grad(Rd, Td, th)
    r = np.sqrt(rigid.radius2(48, 48))
    for q, d in ((0, 1e-3 / r), (1, 1e-3), (2, 1e-3)):
        for s in (-1, 1):
            e = np.zeros(3)
            e[q] = s * d
            assert rigid.ncc_energy_grad(Rd, Td, th + e)[0] >= E0 - 1e-13


def test_brute_force_translation_search_agrees():
    """Pure translation: the flow's G is within half a grid step of the best
    point of an exhaustive 0.05 px grid search of the energy."""
    spec = SeriesSpec(2, 32, 32, noise=0.0, seed=29)
    R, T = rigid_pair(spec, (0.0, 0.85, -0.35))
    Rd, Td = R.double().numpy(), T.double().numpy()
    grid = np.arange(-1.5, 1.5001, 0.05)
    E = np.array([[rigid.ncc_energy_grad(Rd, Td, np.array([0.0, gx, gy]))[0] for gx in grid] for gy in grid])
    iy, ix = np.unravel_index(np.argmin(E), E.shape)
    th = rigid.register([Rd], [Td], None, SolverParams(levels=1, max_iter=400, fixed_iter=True, tau=RIGID_TAU)).theta
    assert abs(th[1] - grid[ix]) <= 0.025 + 1e-9 and abs(th[2] - grid[iy]) <= 0.025 + 1e-9
    assert abs(th[0]) < 1e-3


# ------------------------------------------------------------------ the scan

@pytest.mark.parametrize("algo", ["seq", "lf"])
def test_scan_prefixes_register_each_frame_to_frame_0(algo):
    """phi0[0] is the first pairwise result, and every prefix is within
    0.1 px of the series' known motion (0.05 px noise, 64x64)."""
    cfg = get_config(1, n_frames=7)
    S = rigid_series(cfg.series)
    p = replace(cfg.solver, levels=2, max_iter=200, fixed_iter=False, tau=RIGID_TAU)
    ops, _ = plans.make_plan(6, algo)
    phi0, pairs, iters = rigid.run_scan(S.frames.double().numpy(), p, ops, 6)
    np.testing.assert_array_equal(phi0[0], pairs[0])
    r = np.sqrt(rigid.radius2(64, 64))
    err = phi0 - S.theta[1:]
    assert np.abs(err[:, 0]).max() * r < 0.1 and np.abs(err[:, 1:]).max() < 0.1
    assert iters.shape == (6 + len(ops), 2)
