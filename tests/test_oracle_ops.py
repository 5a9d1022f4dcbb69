"""Pins of the oracle's warp, energy, gradient, pyramid, composition and
differentiation against closed forms, special cases and finite differences."""
import numpy as np
import pytest

from oracle import autodiff
from oracle import registration as reg

rng = np.random.default_rng(7)


def _grid(h, w):
    return np.mgrid[0:h, 0:w]


# ---------------------------------------------------------------- warp (T1)

def test_warp_zero_displacement_is_identity():
    T = rng.standard_normal((13, 17))
    assert np.array_equal(reg.warp(T, np.zeros((2, 13, 17))), T)


def test_warp_integer_shift():
    T = rng.standard_normal((12, 20))
    u = np.zeros((2, 12, 20))
    u[0] = 3.0
    u[1] = -2.0
    out = reg.warp(T, u)
    yy, xx = _grid(12, 20)
    ref = T[np.clip(yy - 2, 0, 11), np.clip(xx + 3, 0, 19)]
    assert np.array_equal(out, ref)


def test_warp_affine_image_interior_exact():
    h, w = 16, 18
    yy, xx = _grid(h, w)
    T = 0.7 * xx - 1.3 * yy + 2.0
    u = rng.uniform(-2.5, 2.5, size=(2, h, w))
    out = reg.warp(T, u)
    ref = 0.7 * (xx + u[0]) - 1.3 * (yy + u[1]) + 2.0
    inside = (xx + u[0] >= 0) & (xx + u[0] <= w - 1) & (yy + u[1] >= 0) & (yy + u[1] <= h - 1)
    assert inside.sum() > 100
    np.testing.assert_allclose(out[inside], ref[inside], rtol=0, atol=1e-12)


def test_warp_bilinear_mixed_term():
    # T = x*y is reproduced exactly by bilinear interpolation inside a cell
    h, w = 10, 10
    yy, xx = _grid(h, w)
    T = (xx * yy).astype(float)
    u = rng.uniform(-1, 1, size=(2, h, w))
    px, py = xx + u[0], yy + u[1]
    inside = (px >= 0) & (px <= w - 1) & (py >= 0) & (py <= h - 1)
    out, dsx, dsy = reg.sample_displaced(T, u)
    np.testing.assert_allclose(out[inside], (px * py)[inside], atol=1e-12)
    np.testing.assert_allclose(dsx[inside], py[inside], atol=1e-12)
    np.testing.assert_allclose(dsy[inside], px[inside], atol=1e-12)


def test_warp_clamps_outside():
    T = rng.standard_normal((8, 8))
    u = np.zeros((2, 8, 8))
    u[0] = 20.5
    s, dsx, dsy = reg.sample_displaced(T, u)
    np.testing.assert_array_equal(s, np.repeat(T[:, 7:8], 8, axis=1))
    assert np.all(dsx == 0)


def test_sample_derivative_matches_difference_quotient():
    T = rng.standard_normal((12, 12))
    u = rng.uniform(-3, 3, size=(2, 12, 12))
    h = 1e-7
    s, dsx, dsy = reg.sample_displaced(T, u)
    up = u.copy()
    up[0] += h
    fd = (reg.sample_displaced(T, up)[0] - s) / h
    same_cell = np.floor(up[0]) == np.floor(u[0])
    np.testing.assert_allclose(fd[same_cell], dsx[same_cell], atol=1e-6)
    up = u.copy()
    up[1] += h
    fd = (reg.sample_displaced(T, up)[0] - s) / h
    same_cell = np.floor(up[1]) == np.floor(u[1])
    np.testing.assert_allclose(fd[same_cell], dsy[same_cell], atol=1e-6)


# ------------------------------------------------------- energy, gradient (T2)

def test_regulariser_closed_form_for_linear_field():
    h, w = 9, 14
    yy, xx = _grid(h, w)
    a, b, c, d = 0.3, -0.2, 0.05, 0.4
    u = np.stack([a * xx + b * yy, c * xx + d * yy]).astype(float)
    R = np.zeros((h, w))
    T = np.zeros((h, w))
    lam = 0.37
    E = reg.energy(R, T, u, lam)
    want = lam * ((a * a + c * c) * (w - 1) * h + (b * b + d * d) * w * (h - 1))
    assert E == pytest.approx(want, rel=1e-13)


def test_data_term_closed_form():
    R = rng.standard_normal((7, 9))
    T = rng.standard_normal((7, 9))
    E = reg.energy(R, T, np.zeros((2, 7, 9)), 0.1)
    assert E == pytest.approx(np.sum((T - R) ** 2), rel=1e-14)


@pytest.mark.parametrize("lam", [0.0, 0.1, 2.0])
def test_gradient_matches_central_differences(lam):
    h, w = 11, 13
    R = rng.standard_normal((h, w))
    T = rng.standard_normal((h, w))
    u = rng.uniform(-2, 2, size=(2, h, w))
    # keep samples away from cell borders so the energy is smooth there
    frac = u - np.floor(u)
    u = np.floor(u) + np.clip(frac, 0.05, 0.95)
    E, g = reg.energy_and_gradient(R, T, u, lam)
    eps = 1e-6
    for _ in range(30):
        c, y, x = rng.integers(2), rng.integers(h), rng.integers(w)
        up, um = u.copy(), u.copy()
        up[c, y, x] += eps
        um[c, y, x] -= eps
        fd = (reg.energy(R, T, up, lam) - reg.energy(R, T, um, lam)) / (2 * eps)
        assert fd == pytest.approx(g[c, y, x], rel=1e-6, abs=1e-7)


def test_gradient_regulariser_sign_on_bump():
    # a single raised pixel must be pulled down by the smoothness term
    u = np.zeros((2, 5, 5))
    u[0, 2, 2] = 1.0
    Z = np.zeros((5, 5))
    _, g = reg.energy_and_gradient(Z, Z, u, 1.0)
    assert g[0, 2, 2] == pytest.approx(2 * 4 * 1.0)
    assert g[0, 2, 1] == pytest.approx(-2.0)
    assert g[0, 0, 0] == 0.0


# -------------------------------------------------------------------- pyramid

def test_restrict_constant_and_linear():
    h, w = 8, 12
    yy, xx = _grid(h, w)
    assert np.allclose(reg.restrict_image(np.full((h, w), 3.5)), 3.5)
    lin = 2.0 * xx + 0.5 * yy
    cy, cx = _grid(h // 2, w // 2)
    np.testing.assert_allclose(reg.restrict_image(lin), 2.0 * (2 * cx + 0.5) + 0.5 * (2 * cy + 0.5))


def test_frame_restriction_constant_linear_and_nyquist():
    h, w = 16, 20
    yy, xx = _grid(h, w)
    assert np.array_equal(reg.restrict_frame(np.full((h, w), 3.5)), np.full((h // 2, w // 2), 3.5))
    # symmetric about the block centre: a linear image is sampled at (2Y+1/2, 2X+1/2)
    lin = 2.0 * xx + 0.5 * yy - 1.0
    cy, cx = _grid(h // 2, w // 2)
    want = 2.0 * (2 * cx + 0.5) + 0.5 * (2 * cy + 0.5) - 1.0
    np.testing.assert_allclose(reg.restrict_frame(lin)[1:-1, 1:-1], want[1:-1, 1:-1], atol=1e-12)
    # the highest frequency of the fine grid is removed (columns, rows, checkerboard)
    for img in ((-1.0) ** xx, (-1.0) ** yy, (-1.0) ** (xx + yy)):
        assert np.all(reg.restrict_frame(img.astype(float))[1:-1, 1:-1] == 0.0)


@pytest.mark.parametrize("f", [1 / 16, 1 / 8, 1 / 6, 1 / 4, 1 / 3])
def test_frame_restriction_frequency_response_is_cos5(f):
    # closed form of the order-5 binomial: cos(2 pi f x + p) -> cos(pi f)^5 cos(2 pi f X' + p)
    h, w = 12, 40
    yy, xx = _grid(h, w)
    img = np.cos(2 * np.pi * f * xx + 0.3)
    cy, cx = _grid(h // 2, w // 2)
    want = np.cos(np.pi * f) ** 5 * np.cos(2 * np.pi * f * (2 * cx + 0.5) + 0.3)
    np.testing.assert_allclose(reg.restrict_frame(img)[:, 2:-2], want[:, 2:-2], atol=1e-13)


def test_frame_restriction_matches_scipy_and_box_of_binomial5():
    from scipy.ndimage import correlate1d
    F = rng.standard_normal((18, 14))
    wts = np.array([1, 5, 10, 10, 5, 1]) / 32.0
    ref = correlate1d(correlate1d(F, wts, axis=0, mode="nearest"), wts, axis=1, mode="nearest")
    np.testing.assert_allclose(reg.restrict_frame(F), ref[1::2, 1::2], atol=1e-14)
    # [1 5 10 10 5 1]/32 = [1 1]/2 * [1 4 6 4 1]/16: the block mean of the
    # 5-tap binomial smoothing (equal away from the clamped border)
    b5 = correlate1d(correlate1d(F, np.array([1, 4, 6, 4, 1]) / 16.0, axis=0, mode="nearest"),
                     np.array([1, 4, 6, 4, 1]) / 16.0, axis=1, mode="nearest")
    np.testing.assert_allclose(reg.restrict_frame(F)[1:-1, 1:-1], reg.restrict_image(b5)[1:-1, 1:-1],
                               atol=1e-14)


def test_prolong_restrict_linear_field_interior():
    # a linear displacement survives restriction + prolongation in the interior
    h, w = 16, 20
    yy, xx = _grid(h, w)
    u = np.stack([0.25 * xx - 0.5 * yy + 1.0, -0.1 * xx + 0.3 * yy - 2.0])
    back = reg.prolong_field(reg.restrict_field(u), h, w)
    np.testing.assert_allclose(back[:, 1:-1, 1:-1], u[:, 1:-1, 1:-1], atol=1e-12)


def test_prolong_constant_doubles():
    uc = np.full((2, 4, 5), 0.75)
    np.testing.assert_allclose(reg.prolong_field(uc, 8, 10), 1.5)


# -------------------------------------------------------------- compose (T6)

def test_compose_with_identity():
    u = rng.uniform(-3, 3, size=(2, 10, 12))
    z = np.zeros_like(u)
    assert np.array_equal(reg.compose(z, u), u)
    assert np.array_equal(reg.compose(u, z), u)


def test_compose_translations_add():
    u = np.zeros((2, 9, 9))
    v = np.zeros((2, 9, 9))
    u[0], u[1] = 1.25, -0.5
    v[0], v[1] = -0.75, 2.0
    np.testing.assert_allclose(reg.compose(u, v), u + v, atol=1e-15)


def test_compose_order():
    # u_ij constant, u_jk linear: u_ik(x) = s + A (x + s) in the interior,
    # which differs from the swapped composition s + A x
    h, w = 20, 20
    yy, xx = _grid(h, w)
    s = np.array([1.5, -0.75])
    u_ij = np.stack([np.full((h, w), s[0]), np.full((h, w), s[1])])
    u_jk = np.stack([0.1 * xx + 0.2 * yy, -0.05 * xx + 0.15 * yy])
    want = np.stack([s[0] + 0.1 * (xx + s[0]) + 0.2 * (yy + s[1]),
                     s[1] - 0.05 * (xx + s[0]) + 0.15 * (yy + s[1])])
    out = reg.compose(u_ij, u_jk)
    np.testing.assert_allclose(out[:, 3:-3, 3:-3], want[:, 3:-3, 3:-3], atol=1e-12)


# ------------------------------------------------------ differentiation (T9)

def test_adjoint_dot_product():
    H, W = 14, 11
    I = rng.standard_normal((H, W))
    v = rng.standard_normal((H, W))
    u = rng.uniform(-4, 4, size=(2, H, W))
    lhs = np.sum(reg.warp(I, u) * v)
    rhs = np.sum(I * autodiff.warp_adjoint(v, u, (H, W)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_restriction_adjoints():
    F = rng.standard_normal((8, 6))
    G = rng.standard_normal((4, 3))
    assert np.sum(reg.restrict_image(F) * G) == pytest.approx(
        np.sum(F * autodiff.restrict_image_adjoint(G)), rel=1e-13)
    F = rng.standard_normal((10, 8))
    G = rng.standard_normal((5, 4))
    assert np.sum(reg.restrict_frame(F) * G) == pytest.approx(
        np.sum(F * autodiff.restrict_frame_adjoint(G, F.shape)), rel=1e-13)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_pyramid_energy_gradients_finite_differences(levels):
    H = W = 16
    Ia = rng.standard_normal((H, W))
    Ib = rng.standard_normal((H, W))
    u = rng.uniform(-1.5, 1.5, size=(2, H, W))
    u = np.floor(u) + np.clip(u - np.floor(u), 0.1, 0.9)
    lam = 0.1
    E, gA, gU, gB = autodiff.pyramid_energy_grads(Ia, u, Ib, lam, levels)
    assert E == pytest.approx(autodiff.pyramid_energy(Ia, u, Ib, lam, levels), rel=1e-14)
    eps = 1e-6

    def fd(which, idx):
        args = [Ia.copy(), u.copy(), Ib.copy()]
        args[which][idx] += eps
        ep = autodiff.pyramid_energy(*args, lam, levels)
        args[which][idx] -= 2 * eps
        em = autodiff.pyramid_energy(*args, lam, levels)
        return (ep - em) / (2 * eps)

    for _ in range(12):
        y, x = rng.integers(H), rng.integers(W)
        assert fd(0, (y, x)) == pytest.approx(gA[y, x], rel=1e-5, abs=1e-6)
        assert fd(2, (y, x)) == pytest.approx(gB[y, x], rel=1e-5, abs=1e-6)
        c = rng.integers(2)
        assert fd(1, (c, y, x)) == pytest.approx(gU[c, y, x], rel=1e-5, abs=1e-6)


def test_single_level_gradient_matches_registration_gradient():
    Ia = rng.standard_normal((9, 9))
    Ib = rng.standard_normal((9, 9))
    u = rng.uniform(-1, 1, size=(2, 9, 9))
    E, _, gU, gB = autodiff.pyramid_energy_grads(Ia, u, Ib, 0.1, 1)
    E2, g2 = reg.energy_and_gradient(Ib, Ia, u, 0.1)
    assert E == E2
    np.testing.assert_array_equal(gU, g2)
    np.testing.assert_allclose(gB, -2 * (reg.warp(Ia, u) - Ib))
