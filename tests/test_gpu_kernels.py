"""GPU parity of the standalone kernels against the oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from oracle import autodiff as oad
from oracle import registration as oreg

from _helpers import announce, f64, gpu, host, smooth_field

pytestmark = pytest.mark.gpu

SIZES = [(8, 8), (13, 77), (64, 64), (70, 129), (128, 96)]


@pytest.fixture(scope="module")
def rs():
    import paper_2010_12478_amd as rs
    assert torch.cuda.is_available()
    return rs


@pytest.mark.parametrize("H,W", SIZES)
def test_warp_parity(rs, H, W):
    announce(f"warp {H}x{W}")
    rng = np.random.default_rng(H * 1000 + W)
    B = 3
    T = rng.standard_normal((B, H, W)).astype(np.float32)
    u = smooth_field(rng, B, H, W, 3.0)
    u[1] *= 4.0                     # far outside the image: clamped taps
    out = host(rs.warp(gpu(T), gpu(u)))
    for b in range(B):
        want = oreg.warp(T[b].astype(np.float64), u[b].astype(np.float64))
        np.testing.assert_allclose(out[b], want, atol=2e-5, rtol=0)


def test_warp_identity_is_exact(rs):
    announce("warp identity")
    T = torch.randn(2, 37, 61, device="cuda")
    u = torch.zeros(2, 2, 37, 61, device="cuda")
    assert torch.equal(rs.warp(T, u), T)


def test_warp_integer_shift_is_exact(rs):
    announce("warp integer shift")
    T = torch.randn(1, 20, 30, device="cuda")
    u = torch.zeros(1, 2, 20, 30, device="cuda")
    u[:, 0] = 2.0
    u[:, 1] = -1.0
    out = rs.warp(T, u)
    ref = oreg.warp(f64(T[0]), f64(u[0]))
    assert np.array_equal(host(out[0]).astype(np.float64), ref)


def test_warp_f64(rs):
    announce("warp f64")
    rng = np.random.default_rng(3)
    T = rng.standard_normal((2, 33, 45))
    u = smooth_field(rng, 2, 33, 45, 2.5).astype(np.float64) + 1e-3
    out = host(rs.warp(gpu(T, torch.float64), gpu(u, torch.float64)))
    for b in range(2):
        np.testing.assert_allclose(out[b], oreg.warp(T[b], u[b]), rtol=0, atol=1e-13)


@pytest.mark.parametrize("H,W", SIZES)
def test_compose_parity(rs, H, W):
    announce(f"compose {H}x{W}")
    rng = np.random.default_rng(H + 7 * W)
    a = smooth_field(rng, 2, H, W, 2.0)
    b = smooth_field(rng, 2, H, W, 2.0)
    out = host(rs.compose(gpu(a), gpu(b)))
    for q in range(2):
        want = oreg.compose(a[q].astype(np.float64), b[q].astype(np.float64))
        np.testing.assert_allclose(out[q], want, atol=2e-5, rtol=0)
    z = torch.zeros(2, 2, H, W, device="cuda")
    assert torch.equal(rs.compose(z, gpu(b)), gpu(b))
    assert torch.equal(rs.compose(gpu(a), z), gpu(a))


@pytest.mark.parametrize("H,W", [(8, 8), (64, 96), (130, 66)])
def test_restrict_prolong_pyramid(rs, H, W):
    announce(f"restrict/prolong {H}x{W}")
    rng = np.random.default_rng(11)
    F = rng.standard_normal((3, H, W)).astype(np.float32)
    got = host(rs.restrict(gpu(F)))
    for q in range(3):
        np.testing.assert_allclose(got[q], oreg.restrict_image(F[q].astype(np.float64)), atol=1e-6)
    u = smooth_field(rng, 2, H // 2, W // 2, 2.0)
    up = host(rs.prolong(gpu(u)))
    for q in range(2):
        np.testing.assert_allclose(up[q], oreg.prolong_field(u[q].astype(np.float64), H, W), atol=1e-5)
    if H % 4 == 0 and W % 4 == 0 and H >= 32 and W >= 32:
        lv = rs.pyramid(gpu(F), 3)
        ref = [oreg.pyramid(F[q].astype(np.float64), 3) for q in range(3)]
        for l in (1, 2):
            for q in range(3):
                np.testing.assert_allclose(host(lv[l - 1][q]), ref[q][l], atol=1e-6)


@pytest.mark.parametrize("H,W", SIZES)
def test_energy_grad_parity(rs, H, W):
    announce(f"energy_grad {H}x{W}")
    rng = np.random.default_rng(5 * H + W)
    B = 2
    R = rng.standard_normal((B, H, W)).astype(np.float32)
    T = rng.standard_normal((B, H, W)).astype(np.float32)
    u = smooth_field(rng, B, H, W, 2.0)
    E, g, gn = rs.energy_grad(gpu(R), gpu(T), gpu(u), 0.1, want_grad=True, want_gnorm=True)
    E, g, gn = host(E), host(g), host(gn)
    for b in range(B):
        Ew, gw = oreg.energy_and_gradient(R[b].astype(np.float64), T[b].astype(np.float64),
                                          u[b].astype(np.float64), 0.1)
        assert E[b] == pytest.approx(Ew, rel=2e-6)
        np.testing.assert_allclose(g[b], gw, atol=5e-5, rtol=1e-5)
        assert gn[b] == pytest.approx(np.sum(gw * gw), rel=1e-5)
    # bitwise reproducible
    E2, g2, _ = rs.energy_grad(gpu(R), gpu(T), gpu(u), 0.1)
    assert np.array_equal(host(E2), E) and np.array_equal(host(g2), g)


def test_energy_grad_tile_order_does_not_change_results(rs):
    """A batch large enough for the XCD-aware tile order to permute its
    blocks (5 items of 256x192 at 64-row tiles: 60 tiles, two full runs of
    8 x 3 and a tail of 12) gives every item bitwise the energy, gradient
    and gradient norm of that item alone (12 tiles: no permutation), and
    matches the oracle."""
    announce("energy_grad tile order")
    rng = np.random.default_rng(21)
    B, H, W = 5, 256, 192
    rs.set_tuning(64, 0)
    R = rng.standard_normal((B, H, W)).astype(np.float32)
    T = rng.standard_normal((B, H, W)).astype(np.float32)
    u = smooth_field(rng, B, H, W, 2.5)
    E, g, gn = rs.energy_grad(gpu(R), gpu(T), gpu(u), 0.1, want_grad=True, want_gnorm=True)
    E, g, gn = host(E), host(g), host(gn)
    for b in range(B):
        E1, g1, gn1 = rs.energy_grad(gpu(R[b:b + 1]), gpu(T[b:b + 1]), gpu(u[b:b + 1]), 0.1, want_grad=True,
                                     want_gnorm=True)
        assert host(E1)[0] == E[b] and host(gn1)[0] == gn[b]
        assert np.array_equal(host(g1)[0], g[b])
    Ew, gw = oreg.energy_and_gradient(R[3].astype(np.float64), T[3].astype(np.float64), u[3].astype(np.float64),
                                      0.1)
    assert E[3] == pytest.approx(Ew, rel=2e-6)
    np.testing.assert_allclose(g[3], gw, atol=5e-5, rtol=1e-5)


def test_energy_grad_f64(rs):
    announce("energy_grad f64")
    rng = np.random.default_rng(9)
    R = rng.standard_normal((2, 40, 70))
    T = rng.standard_normal((2, 40, 70))
    u = smooth_field(rng, 2, 40, 70, 1.5).astype(np.float64) + 1e-4
    E, g, _ = rs.energy_grad(gpu(R, torch.float64), gpu(T, torch.float64), gpu(u, torch.float64), 0.1)
    for b in range(2):
        Ew, gw = oreg.energy_and_gradient(R[b], T[b], u[b], 0.1)
        assert host(E)[b] == pytest.approx(Ew, rel=1e-12)
        np.testing.assert_allclose(host(g)[b], gw, atol=1e-11)


@pytest.mark.parametrize("H,W", [(16, 16), (45, 70)])
def test_warp_adjoint_parity(rs, H, W):
    announce(f"warp_adjoint {H}x{W}")
    rng = np.random.default_rng(H * W)
    v = rng.standard_normal((2, H, W)).astype(np.float32)
    u = smooth_field(rng, 2, H, W, 3.0)
    got = host(rs.warp_adjoint(gpu(v), gpu(u)))
    for b in range(2):
        want = oad.warp_adjoint(v[b].astype(np.float64), u[b].astype(np.float64), (H, W))
        np.testing.assert_allclose(got[b], want, atol=1e-4, rtol=1e-5)
    # dot-product test in float64
    I = rng.standard_normal((2, H, W))
    v64 = rng.standard_normal((2, H, W))
    u64 = smooth_field(rng, 2, H, W, 3.0).astype(np.float64) + 1e-3
    lhs = np.sum(host(rs.warp(gpu(I, torch.float64), gpu(u64, torch.float64))) * v64)
    rhs = np.sum(I * host(rs.warp_adjoint(gpu(v64, torch.float64), gpu(u64, torch.float64))))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("H,W,amp", [(150, 200, 3.0), (97, 130, 20.0), (64, 64, 9.0)])
def test_warp_adjoint_joined_and_separate_taps(rs, H, W, amp):
    """The adjoint joins shares that land on one cell (the lower taps of a
    row with the upper taps of the next, a lane's right tap with its right
    neighbour's left tap) before the atomic addition: groups of 16 rows with
    a ragged last group and partial last wavefronts; amp 3 makes the taps
    of neighbouring pixels mostly coincide, amp 9 and 20 (with the
    per-pixel noise of the field) make many of them differ, and one item
    mixes both."""
    announce(f"warp_adjoint joins {H}x{W} amp {amp}")
    rng = np.random.default_rng(H + W + int(amp))
    B = 3
    v = rng.standard_normal((B, H, W)).astype(np.float32)
    u = smooth_field(rng, B, H, W, amp)
    u[2, :, :, : W // 2] *= 0.1
    base = rng.standard_normal((B, H, W)).astype(np.float32)
    got = host(rs.warp_adjoint(gpu(v), gpu(u), gpu(base.copy())))
    for b in range(B):
        want = base[b].astype(np.float64) + oad.warp_adjoint(v[b].astype(np.float64), u[b].astype(np.float64),
                                                             (H, W))
        np.testing.assert_allclose(got[b], want, atol=2e-4, rtol=1e-5)


def test_warp_adjoint_dot_product_full_size(rs):
    """<warp(I), v> = <I, adjoint(v)> in float64 on the differentiation
    workload's shape (64 x 512x512, a +-3 px field as in the benchmark, one
    item with +-40 px): a property that holds at any size, checked per item."""
    announce("warp_adjoint dot product 64x512x512")
    B, H, W = 64, 512, 512
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    I = torch.randn((B, H, W), device="cuda", dtype=torch.float64, generator=g)
    v = torch.randn((B, H, W), device="cuda", dtype=torch.float64, generator=g)
    yy = torch.arange(H, device="cuda", dtype=torch.float64).view(1, H, 1)
    xx = torch.arange(W, device="cuda", dtype=torch.float64).view(1, 1, W)
    ph = torch.rand((B, 1, 1), device="cuda", dtype=torch.float64, generator=g) * 6.28
    u = torch.stack([3.0 * torch.sin(2 * np.pi * yy / H + ph) + 0.01 * xx,
                     3.0 * torch.sin(2 * np.pi * xx / W + ph) + 0.01 * yy], dim=1).contiguous()
    u[5] *= 13.0
    lhs = (rs.warp(I, u) * v).sum(dim=(1, 2))
    rhs = (I * rs.warp_adjoint(v, u)).sum(dim=(1, 2))
    torch.testing.assert_close(lhs, rhs, rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("levels,H,W,amp", [(1, 64, 48, 2.0), (2, 64, 48, 2.0), (3, 64, 48, 2.0),
                                            (2, 132, 200, 2.0), (2, 90, 150, 16.0)])
def test_pyramid_energy_and_backward_parity(rs, levels, H, W, amp):
    """The backward pass's dIa scatter joins shares on one cell as the warp's
    adjoint does: small and ragged shapes, smooth and rough fields."""
    announce(f"pyramid energy levels={levels} {H}x{W} amp {amp}")
    rng = np.random.default_rng(levels + H)
    B = 2
    Ia = rng.standard_normal((B, H, W)).astype(np.float32)
    Ib = rng.standard_normal((B, H, W)).astype(np.float32)
    u = smooth_field(rng, B, H, W, amp)
    gE = torch.tensor([1.0, -0.5], dtype=torch.float64, device="cuda")
    E = host(rs.pyramid_energy(gpu(Ia), gpu(u), gpu(Ib), 0.1, levels))
    dIa, du, dIb = (host(t) for t in rs.pyramid_energy_backward(gpu(Ia), gpu(u), gpu(Ib), 0.1, levels, gE))
    w = host(gE)
    for b in range(B):
        Ew, gA, gU, gB = oad.pyramid_energy_grads(Ia[b].astype(np.float64), u[b].astype(np.float64),
                                                  Ib[b].astype(np.float64), 0.1, levels)
        assert E[b] == pytest.approx(Ew, rel=2e-6)
        np.testing.assert_allclose(dIa[b], w[b] * gA, atol=1e-4, rtol=1e-5)
        np.testing.assert_allclose(du[b], w[b] * gU, atol=1e-4, rtol=1e-5)
        np.testing.assert_allclose(dIb[b], w[b] * gB, atol=1e-4, rtol=1e-5)


@pytest.mark.parametrize("levels", [1, 2])
def test_gradcheck_f64_on_crops(rs, levels):
    """FP64 gradcheck of the autograd Function on 32x32 crops of frame pairs
    from the 512x512 differentiation workload's generator."""
    announce(f"gradcheck levels={levels}")
    from synth import get_config, make_series
    cfg = get_config(4, n_frames=5)
    S = make_series(cfg.series)
    rng = np.random.default_rng(40 + levels)
    crops_a, crops_b = [], []
    for p in range(4):
        y, x = rng.integers(0, 512 - 32, size=2)
        crops_a.append(S.frames[p + 1, y:y + 32, x:x + 32].double().numpy())
        crops_b.append(S.frames[p, y:y + 32, x:x + 32].double().numpy())
    Ia = gpu(np.stack(crops_a), torch.float64).requires_grad_()
    Ib = gpu(np.stack(crops_b), torch.float64).requires_grad_()
    # 1.3 + 0.05 * smooth: every pyramid level's samples (u halved per level)
    # stay inside one bilinear cell, where the energy is differentiable
    u = 1.3 + 0.05 * smooth_field(rng, 4, 32, 32, 1.0).astype(np.float64)
    u = gpu(u, torch.float64).requires_grad_()
    assert torch.autograd.gradcheck(lambda a, v, b: rs.warp_energy(a, v, b, 0.1, levels),
                                    (Ia, u, Ib), eps=1e-6, atol=1e-6, rtol=1e-5,
                                    nondet_tol=1e-12)   # dE/dIa uses atomic additions


def test_autograd_f32_matches_oracle(rs):
    announce("autograd f32")
    rng = np.random.default_rng(77)
    Ia = rng.standard_normal((2, 48, 48)).astype(np.float32)
    Ib = rng.standard_normal((2, 48, 48)).astype(np.float32)
    u = smooth_field(rng, 2, 48, 48, 1.5)
    ta, tu, tb = (gpu(x).requires_grad_() for x in (Ia, u, Ib))
    E = rs.warp_energy(ta, tu, tb, 0.1, 2)
    E.sum().backward()
    for b in range(2):
        Ew, gA, gU, gB = oad.pyramid_energy_grads(Ia[b].astype(np.float64), u[b].astype(np.float64),
                                                  Ib[b].astype(np.float64), 0.1, 2)
        assert host(E)[b] == pytest.approx(Ew, rel=2e-6)
        np.testing.assert_allclose(host(ta.grad)[b], gA, atol=1e-4, rtol=1e-5)
        np.testing.assert_allclose(host(tu.grad)[b], gU, atol=1e-4, rtol=1e-5)
        np.testing.assert_allclose(host(tb.grad)[b], gB, atol=1e-4, rtol=1e-5)


def test_empty_batch_is_noop(rs):
    announce("empty batch")
    T = torch.zeros(0, 16, 16, device="cuda")
    u = torch.zeros(0, 2, 16, 16, device="cuda")
    assert rs.warp(T, u).shape == (0, 16, 16)
