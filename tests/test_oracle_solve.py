"""Pins of the oracle's gradient descent, multilevel solve and scan executor:
identity registration, brute-force shift search, recovery of known synthetic
deformations (proposed acceptance thresholds, the paper prints none)."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import registration as reg
from oracle.scan import run_scan
from synth import SeriesSpec, get_config, ground_truth, lattice_image, make_series
from synth.configs import SolverParams

import torch


def _lattice_pair(shift, size=24, spacing=8.0):
    spec = SeriesSpec(2, size, size, spacing=spacing, noise=0.0)
    origin = np.array([3.3, 2.1])
    yy, xx = torch.meshgrid(torch.arange(size, dtype=torch.float64),
                            torch.arange(size, dtype=torch.float64), indexing="ij")
    R = lattice_image(spec, origin, xx, yy).numpy()
    T = lattice_image(spec, origin, xx - shift[0], yy - shift[1]).numpy()
    return R, T          # T(x + shift) = R(x)


# ----------------------------------------------------------------- T3

@pytest.mark.parametrize("levels", [1, 2, 3])
def test_identity_registration_of_identical_frames(levels):
    cfg = get_config(1, n_frames=2, height=32, width=48)
    f = make_series(cfg.series).frames[0].numpy().astype(np.float64)
    pyr = reg.pyramid(f, levels)
    res = reg.register(pyr, pyr, None, SolverParams(levels=levels, max_iter=30))
    assert np.all(res.u == 0.0)
    # zero residual and zero gradient: the relative rule stops at t = 1
    assert res.iters == [1] * levels


def test_fixed_iterations_are_exact():
    R, T = _lattice_pair((0.4, -0.3))
    res = reg.solve_level(R, T, np.zeros((2, 24, 24)), 0.5, 0.1, 7, True, 1e-5)
    assert res.iters == 7 and len(res.energies) == 7


def test_stopping_rule_special_cases():
    R, T = _lattice_pair((0.6, 0.2))
    u0 = np.zeros((2, 24, 24))
    # a huge tolerance stops at the first check
    assert reg.solve_level(R, T, u0, 0.5, 0.1, 50, False, 1e9).iters == 1
    # tolerance 0 runs until the energy no longer decreases
    res = reg.solve_level(R, T, u0, 0.5, 0.1, 2000, False, 0.0)
    e = res.energies
    assert res.iters < 2000
    assert all(e[t] < e[t - 1] for t in range(1, len(e) - 1))
    assert e[-1] >= e[-2]


def test_nonfinite_energy_stops():
    R, T = _lattice_pair((0.5, 0.5))
    R = R.copy()
    R[3, 3] = np.nan
    res = reg.solve_level(R, T, np.zeros((2, 24, 24)), 0.5, 0.1, 20, False, 1e-5)
    assert res.status == reg.STATUS_NONFINITE and res.iters == 0


# ----------------------------------------------------------------- T4

def _exhaustive_shift(R, T, lam=0.1):
    """argmin of E over constant shifts on a 1/64 px grid in [-3, 3]^2."""
    def E(s):
        u = np.empty((2,) + R.shape)
        u[0], u[1] = s
        return reg.energy(R, T, u, lam)
    coarse = np.arange(-3, 3 + 1e-9, 1 / 8)
    best = min(((E((sx, sy)), sx, sy) for sx in coarse for sy in coarse))
    fine = np.arange(-8, 9) / 64
    best = min(((E((best[1] + dx, best[2] + dy)), best[1] + dx, best[2] + dy)
                for dx in fine for dy in fine))
    return np.array(best[1:])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_shift_search(seed):
    s_true = np.random.default_rng(100 + seed).uniform(-1.5, 1.5, size=2)
    R, T = _lattice_pair(s_true)
    s_star = _exhaustive_shift(R, T)
    assert np.all(np.abs(s_star - s_true) < 0.1)

    # (i) gradient descent restricted to constant fields lands on s*
    v = np.zeros(2)
    for _ in range(3000):
        u = np.empty((2, 24, 24))
        u[0], u[1] = v
        _, g = reg.energy_and_gradient(R, T, u, 0.1)
        v = v - 0.004 * g.reshape(2, -1).sum(axis=1)
    assert np.all(np.abs(v - s_star) <= 1 / 64 + 1e-12)

    # (ii) a stiff regulariser keeps the dense field near-constant at s*
    p = SolverParams(levels=1, max_iter=20000, tau=0.05, lam=2.0, rel_tol=1e-12)
    res = reg.register([R], [T], None, p)
    assert np.all(np.abs(res.u[:, 4:-4, 4:-4].reshape(2, -1).mean(axis=1) - s_star) < 0.02)

    # (iii) the default operator from the identity stays in s*'s basin
    # (shift below half a lattice period, Section 2.3.2)
    res = reg.register([R], [T], None, SolverParams(levels=1, max_iter=500))
    assert np.all(np.abs(res.u[:, 4:-4, 4:-4].reshape(2, -1).mean(axis=1) - s_star) < 0.1)


# ----------------------------------------------------------------- T5

def _atom_mask(series, clean_spec, i):
    clean = make_series(clean_spec).frames[i].numpy()
    b = int(series.spec.drift + 2)
    m = np.zeros(clean.shape, bool)
    m[b:-b, b:-b] = True
    return m & (clean >= np.exp(-2.0))   # within ~2 sigma of an atom centre


@pytest.mark.parametrize("levels", [1, 2])
def test_recovery_of_synthetic_deformation_noise_free(levels):
    cfg = get_config(1, n_frames=6, noise=0.0, levels=levels, max_iter=500, fixed_iter=False)
    S = make_series(cfg.series)
    fr = S.frames.numpy().astype(np.float64)
    res = run_scan(fr, cfg.solver, "seq")
    mask = _atom_mask(S, cfg.series, 0)
    for k in (1, 3, 5):
        e = np.abs(res.phi0[k - 1] - ground_truth(S, 0, k))[:, mask]
        assert e.max() <= 0.1 and np.sqrt((e ** 2).mean()) <= 0.03, k
    assert np.all(np.abs(S.drift[1:] - S.drift[:-1]) < cfg.series.spacing / 2)


def test_recovery_of_synthetic_deformation_noisy():
    cfg = get_config(1, n_frames=4, noise=0.05, levels=1, max_iter=500, fixed_iter=False)
    S = make_series(cfg.series)
    res = run_scan(S.frames.numpy().astype(np.float64), cfg.solver, "seq")
    mask = _atom_mask(S, replace(cfg.series, noise=0.0), 0)
    for k in (1, 3):
        e = np.abs(res.phi0[k - 1] - ground_truth(S, 0, k))[:, mask]
        assert np.sqrt((e ** 2).mean()) <= 0.12


def test_scan_plans_agree_with_sequential_recursion_on_clean_series():
    # Associativity in practice (Section 2.3.3): tree orders land on the same
    # deformation as the sequential recursion up to the solver's accuracy.
    cfg = get_config(1, n_frames=9, noise=0.0, levels=1, max_iter=300, fixed_iter=False)
    S = make_series(cfg.series)
    fr = S.frames.numpy().astype(np.float64)
    seq = run_scan(fr, cfg.solver, "seq")
    mask = _atom_mask(S, cfg.series, 0)
    for algo in ("dissemination", "lf", "bk"):
        tree = run_scan(fr, cfg.solver, algo)
        assert np.array_equal(tree.u_pair, seq.u_pair)
        dev = np.abs(tree.phi0 - seq.phi0)[:, :, mask]
        print(f"{algo}: max deviation from the sequential order {dev.max():.4f} px")
        assert dev.max() < 0.05


# ------------------------------------------- flexible segments (Algorithm 1)

def test_flex_orders_accepts_algorithm1_schedules_and_rejects_others():
    from oracle.scan import flex_orders, flex_start
    M, W = 9, 3
    assert [flex_start(M, W, w) for w in range(W)] == [0, 4, 8]
    # worker 0: 0 -> 1 -> 2; worker 1: 4 -> 5 (right first) -> 3; worker 2: 8 -> 7 -> 6
    seg = [(0, 2), (3, 5), (6, 8)]
    step = np.array([0, 1, 2, 2, 0, 1, 2, 1, 0])
    orders = flex_orders(seg, step, M)
    assert orders == [(0, [1, 2]), (4, [5, 3]), (8, [7, 6])]
    bad = step.copy()
    bad[3], bad[5] = 1, 2          # worker 1 stepped left first
    with pytest.raises(ValueError):
        flex_orders(seg, bad, M)
    with pytest.raises(ValueError):
        flex_orders([(0, 2), (4, 5), (6, 8)], step, M)    # element 3 uncovered
    # worker 0 taking element 3 instead is legal too
    assert flex_orders([(0, 3), (4, 5), (6, 8)], np.array([0, 1, 2, 3, 0, 1, 2, 1, 0]), M)[0] == (0, [1, 2, 3])
    jump = np.array([0, 2, 1, 2, 0, 1, 2, 1, 0])           # worker 0 absorbs 2 before 1
    with pytest.raises(ValueError):
        flex_orders(seg, jump, M)


def test_flex_scan_agrees_with_sequential_recursion_on_clean_series():
    # any legal combination order lands on the same deformation as the
    # sequential recursion up to the solver's accuracy (Section 2.3.3)
    from oracle.scan import run_flex_scan
    cfg = get_config(1, n_frames=10, noise=0.0, levels=1, max_iter=300, fixed_iter=False)
    S = make_series(cfg.series)
    fr = S.frames.numpy().astype(np.float64)
    seq = run_scan(fr, cfg.solver, "seq")
    seg = [(0, 2), (3, 5), (6, 8)]
    step = np.array([0, 1, 2, 2, 0, 1, 2, 1, 0])
    phi0, u_pair = run_flex_scan(fr, cfg.solver, seg, step, "lf")
    assert np.array_equal(u_pair, seq.u_pair)
    assert np.array_equal(phi0[:3], seq.phi0[:3])       # worker 0 is the sequential recursion
    mask = _atom_mask(S, cfg.series, 0)
    dev = np.abs(phi0 - seq.phi0)[:, :, mask]
    assert dev.max() < 0.05


# ------------------------------------------- storage precision of the oracle

def test_float64_storage_keeps_unrounded_iterates():
    # "f64" is plain float64: iterates are not float32 values; "f32" rounds
    # every stored field (the mode the GPU is compared with bit for bit)
    R, T = _lattice_pair((0.45, -0.35))
    u0 = np.zeros((2, 24, 24))
    a = reg.solve_level(R, T, u0, 0.5, 0.1, 12, True, 1e-5, storage="f32")
    b = reg.solve_level(R, T, u0, 0.5, 0.1, 12, True, 1e-5, storage="f64")
    assert np.array_equal(a.u, reg.f32(a.u))
    assert not np.array_equal(b.u, reg.f32(b.u))
    assert np.abs(a.u - b.u).max() < 1e-5
    f = make_series(get_config(1, n_frames=1, height=32, width=32).series).frames[0].numpy().astype(np.float64)
    p32, p64 = reg.pyramid(f, 3, "f32"), reg.pyramid(f, 3, "f64")
    assert np.array_equal(p32[0], p64[0]) and np.array_equal(p32[2], reg.f32(p32[2]))
    assert np.abs(p32[2] - p64[2]).max() < 1e-6 and not np.array_equal(p32[2], p64[2])


# ------------------------- recovery along chains at the 512 and 1024 settings

def _window_series(index, n, size):
    cfg = get_config(index, n_frames=n)
    H, W = cfg.series.height, cfg.series.width
    win = ((H - size) // 2, (W - size) // 2, size, size)
    return cfg, win, make_series(cfg.series, window=win)


@pytest.mark.parametrize("index", [3, 5])
def test_recovery_along_a_chain_keeps_every_prefix_registered(index):
    """Recovery of known deformations through the scan (Section 2.3.2: each
    frame registered to frame 0 from the composition of its neighbours).
    Settings of the 1024 x 512x512 series (spacing 8, 3 levels, drift 8 px,
    distortion 1.5 px, one extra-noise frame) and of the 4096 x 1024x1024
    series (spacing 12, 4 levels, drift 16 px, distortion 2 px): 16 frames
    on a central 128x128 window of the full-size frames (same drift walk and
    distortion field; the coarsest grid keeps its 2 px and 1.5 px lattice
    period).  Bounds on the interior (D + 2 px from the border), for every
    prefix phi_{0,k}: rms <= 0.35 px, about twice the noise-limited accuracy
    of a single registration (0.1-0.25 px measured), and max <= 2 px, half
    of the half period of the 8 px lattice: a prefix that lost the lattice
    anywhere would be off by a period there (8 or 12 px)."""
    cfg, win, S = _window_series(index, 17, 128)
    assert np.all(np.abs(np.diff(S.drift, axis=0)) <= cfg.series.spacing / 4)
    res = run_scan(S.frames.numpy().astype(np.float64), cfg.solver, "seq",
                   workers=min(8, len(__import__("os").sched_getaffinity(0))))
    m = int(cfg.series.drift + 2)
    moved = 0.0
    for k in range(1, 17):
        gt = ground_truth(S, 0, k, window=win)
        d = (res.phi0[k - 1] - gt)[:, m:-m, m:-m]
        rms, mx = np.sqrt(np.mean(d ** 2)), np.abs(d).max()
        print(f"phi_0,{k}: rms {rms:.3f} px, max {mx:.2f} px, |drift| {np.abs(S.drift[k]).max():.1f} px")
        assert rms <= 0.35 and mx <= 2.0, k
        moved = max(moved, np.abs(gt).max())
    # the chain reaches beyond half a lattice period from frame 0 (so it is
    # the chaining, not one registration from the identity, that recovers it)
    assert moved > cfg.series.spacing / 2


def test_block_mean_pyramid_loses_the_lattice_where_the_binomial_keeps_it(monkeypatch):
    """Why frames are coarsened by the binomial low-pass: on the 512x512
    settings (3 levels: the coarsest grid samples the 8 px lattice with 2 px
    per period), pair (7, 8) of the series registered from the identity on a
    256x256 window.  With the 2x2 block mean the coarsest level pulls the
    shift to its mirror image and the finer levels cannot recover it."""
    cfg, win, S = _window_series(3, 9, 256)
    win = (0, 0, 256, 256)
    S = make_series(cfg.series, window=win)
    fr = S.frames.numpy().astype(np.float64)
    gt = ground_truth(S, 7, 8, window=win)

    def run():
        p = [reg.pyramid(fr[i], cfg.solver.levels) for i in (7, 8)]
        u = reg.register(p[0], p[1], None, cfg.solver).u
        return np.sqrt(np.mean((u - gt)[:, 10:-10, 10:-10] ** 2))

    good = run()
    monkeypatch.setattr(reg, "restrict_frame", reg.restrict_image)
    bad = run()
    print(f"binomial pyramid {good:.3f} px rms, block-mean pyramid {bad:.3f} px rms")
    assert good <= 0.35 and bad >= 2.0
