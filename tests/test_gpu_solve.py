"""GPU parity of the registration solver (reg_solve_batch) against the oracle,
plain vs batched execution, and edge cases."""
from dataclasses import replace

import numpy as np
import pytest
import torch

from oracle import registration as oreg
from synth import get_config, make_series
from synth.configs import SolverParams

from _helpers import announce, gpu, host, smooth_field

pytestmark = pytest.mark.gpu

TOL_PX = 1e-3   # final displacements, max-abs


@pytest.fixture(scope="module")
def rs():
    import paper_2010_12478_amd as rs
    return rs


@pytest.fixture(autouse=True)
def _default_tuning(rs):
    rs.set_tuning(32, 16, resident=True)
    yield
    rs.set_tuning(32, 16, resident=True)


def _series(index, **kw):
    cfg = get_config(index, **kw)
    S = make_series(cfg.series)
    return cfg, S.frames


def _oracle_batch(frames, ref, tmpl, params, u0=None):
    fr = frames.double().numpy()
    pyrs = {f: oreg.pyramid(fr[f], params.levels) for f in set(ref) | set(tmpl)}
    out = []
    for b, (i, k) in enumerate(zip(ref, tmpl)):
        out.append(oreg.register(pyrs[i], pyrs[k], None if u0 is None else u0[b].astype(np.float64), params))
    return out


@pytest.mark.parametrize("mode", ["plain", "batched"])
@pytest.mark.parametrize("levels", [1, 2])
def test_identity_registration_is_exactly_zero(rs, mode, levels):
    announce(f"identity solve {mode} L={levels}")
    cfg, frames = _series(1, n_frames=2, height=64, width=80)
    p = SolverParams(levels=levels, max_iter=30)
    u, iters, status = rs.solve_batch(frames.cuda(), [0, 1], [0, 1], p, mode=mode)
    assert torch.count_nonzero(u).item() == 0
    assert host(iters).tolist() == [[1] * levels] * 2
    assert host(status).tolist() == [0, 0]


@pytest.mark.parametrize("mode", ["plain", "batched"])
@pytest.mark.parametrize("levels,iters", [(1, 1), (1, 2), (1, 17), (2, 5), (3, 9)])
def test_stored_iterates_bitwise_equal_to_oracle(rs, mode, levels, iters):
    """Storage-precision reading: every stored value is the same sequence of
    rounded float64 operations on both sides, so after any fixed number of
    updates the float32 field equals the oracle's bit for bit (from the
    identity and from a composed initial guess with negative and positive
    displacements, which exercises the in-cell fraction of u in (-1, 0))."""
    announce(f"bitwise {mode} L={levels} iters={iters}")
    cfg, frames = _series(1, n_frames=3, height=64, width=96)
    p = replace(cfg.solver, levels=levels, max_iter=iters, fixed_iter=True)
    rng = np.random.default_rng(11 + levels)
    u0 = smooth_field(rng, 1, 64, 96, 1.2)
    for init in (None, u0):
        u, it, st = rs.solve_batch(frames.cuda(), [0], [2], p,
                                   u0=None if init is None else gpu(init), mode=mode)
        want = _oracle_batch(frames, [0], [2], p, init)[0]
        got = host(u)[0].astype(np.float64)
        print(f"init={'identity' if init is None else 'smooth'}: "
              f"{int((got != want.u).sum())} of {got.size} values differ")
        assert np.array_equal(got, want.u)
        assert host(it)[0].tolist() == want.iters


@pytest.mark.parametrize("H,W,levels", [(64, 64, 1), (64, 96, 2), (72, 40, 1), (128, 128, 3)])
def test_solve_batch_matches_oracle(rs, H, W, levels):
    announce(f"solve_batch vs oracle {H}x{W} L={levels}")
    cfg, frames = _series(2, n_frames=5, height=H, width=W)
    p = replace(cfg.solver, levels=levels)
    ref, tmpl = [0, 1, 2, 3], [1, 2, 3, 4]
    u, iters, status = rs.solve_batch(frames.cuda(), ref, tmpl, p, mode="batched")
    want = _oracle_batch(frames, ref, tmpl, p)
    u, iters, status = host(u), host(iters), host(status)
    for b, w in enumerate(want):
        err = np.abs(u[b] - w.u).max()
        print(f"pair {b}: iters gpu {iters[b].tolist()} oracle {w.iters} max-abs {err:.2e} px")
        assert err <= TOL_PX
        assert iters[b].tolist() == list(w.iters)
        assert status[b] == w.status


def test_plain_and_batched_are_bitwise_identical(rs):
    announce("plain vs batched")
    cfg, frames = _series(2, n_frames=6, height=64, width=64)
    p = replace(cfg.solver, levels=2, max_iter=60)
    ref, tmpl = [0, 1, 2, 3, 4], [1, 2, 3, 4, 5]
    a = rs.solve_batch(frames.cuda(), ref, tmpl, p, mode="plain")
    b = rs.solve_batch(frames.cuda(), ref, tmpl, p, mode="batched")
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("max_group", [1, 2, 4, 16])
def test_group_size_does_not_change_results(rs, max_group):
    announce(f"group size {max_group}")
    cfg, frames = _series(2, n_frames=4, height=128, width=128)
    p = replace(cfg.solver, levels=2, max_iter=40)
    ref, tmpl = [0, 1, 2], [1, 2, 3]
    rs.set_tuning(32, 1)
    base = rs.solve_batch(frames.cuda(), ref, tmpl, p)
    rs.set_tuning(32, max_group)
    got = rs.solve_batch(frames.cuda(), ref, tmpl, p)
    for x, y in zip(base, got):
        assert torch.equal(x, y)


@pytest.mark.parametrize("tile_rows", [4, 16, 24, 56, 64])
def test_tile_rows_match_oracle(rs, tile_rows):
    """Streamed tiles of several heights against the oracle; 24 and 56 rows
    give each wavefront a ragged last batch after batches that pass their
    shared rows of u on, and 56 a ragged last row of tiles."""
    announce(f"tile rows {tile_rows}")
    cfg, frames = _series(2, n_frames=3, height=96, width=80)
    p = replace(cfg.solver, levels=1, max_iter=80)
    rs.set_tuning(tile_rows, 4)
    u, iters, _ = rs.solve_batch(frames.cuda(), [0, 1], [1, 2], p)
    want = _oracle_batch(frames, [0, 1], [1, 2], p)
    for b, w in enumerate(want):
        assert np.abs(host(u)[b] - w.u).max() <= TOL_PX


@pytest.mark.parametrize("tile_rows", [4, 8, 16, 32, 64])
@pytest.mark.parametrize("H,W,levels", [(64, 64, 1), (128, 192, 2), (256, 128, 3)])
def test_resident_levels_match_streaming_bitwise(rs, tile_rows, H, W, levels):
    """Register-resident levels (one workgroup per tile) give the same bits
    as the streaming sweep with the same tiles, and match the oracle."""
    announce(f"resident vs streaming {H}x{W} L={levels} th={tile_rows}")
    cfg, frames = _series(2, n_frames=4, height=H, width=W)
    p = replace(cfg.solver, levels=levels, max_iter=60)
    ref, tmpl = [0, 1, 2], [1, 2, 3]
    rs.set_tuning(tile_rows, 128, resident=False)
    a = rs.solve_batch(frames.cuda(), ref, tmpl, p)
    rs.set_tuning(tile_rows, 128, resident=True)
    b = rs.solve_batch(frames.cuda(), ref, tmpl, p)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    if tile_rows == 32:
        want = _oracle_batch(frames, ref, tmpl, p)
        for k, w in enumerate(want):
            assert np.abs(host(b[0])[k] - w.u).max() <= TOL_PX
            assert host(b[1])[k].tolist() == list(w.iters)


@pytest.mark.parametrize("H,W,levels,tile_rows,group",
                         [(128, 256, 2, 64, 128), (256, 512, 1, 16, 1), (64, 256, 1, 4, 1)])
def test_rows_of_four_tiles_match_resident_bitwise(rs, H, W, levels, tile_rows, group):
    """A streamed level whose width in tiles is a multiple of 4 is swept with
    every wavefront on a whole tile, the four of a workgroup side by side;
    its energies add the same quarter sums in the same order as the
    register-resident form, so the bits agree.  With one workgroup per
    registration the 256x512 level is 32 rows of four tiles (two flushes of
    the tile sums); 4-row tiles make every quarter one row."""
    announce(f"rows of four vs resident {H}x{W} L={levels} th={tile_rows} g={group}")
    cfg, frames = _series(2, n_frames=3, height=H, width=W)
    p = replace(cfg.solver, levels=levels, max_iter=60)
    ref, tmpl = [0, 1], [1, 2]
    rs.set_tuning(tile_rows, group, resident=False)
    a = rs.solve_batch(frames.cuda(), ref, tmpl, p)
    rs.set_tuning(tile_rows, 128, resident=True)
    b = rs.solve_batch(frames.cuda(), ref, tmpl, p)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    want = _oracle_batch(frames, ref, tmpl, p)
    for k, w in enumerate(want):
        assert np.abs(host(a[0])[k] - w.u).max() <= TOL_PX
        assert host(a[1])[k].tolist() == list(w.iters)


@pytest.mark.parametrize("H,W", [(100, 200), (70, 260)])
def test_rows_of_four_tiles_ragged_match_oracle(rs, H, W):
    """Streamed levels with a last column and a last row of tiles partly
    outside the image: 200 columns are 4 tiles (swept as a row of four), 260
    are 5 (swept by quarters)."""
    announce(f"rows of four ragged {H}x{W}")
    cfg, frames = _series(2, n_frames=3, height=H, width=W)
    p = replace(cfg.solver, levels=1, max_iter=60)
    rs.set_tuning(16, 2, resident=False)
    u, iters, _ = rs.solve_batch(frames.cuda(), [0, 1], [1, 2], p)
    want = _oracle_batch(frames, [0, 1], [1, 2], p)
    for b, w in enumerate(want):
        assert np.abs(host(u)[b] - w.u).max() <= TOL_PX
        assert host(iters)[b].tolist() == list(w.iters)


def test_resident_stop_keeps_previous_state_and_nonfinite(rs):
    """A level that stops on the energy test returns the state its last
    iteration started from (the LDS copy); a non-finite frame still flags the
    registration and fills it with NaN."""
    announce("resident stop/nonfinite")
    cfg, frames = _series(2, n_frames=4, height=128, width=128)
    frames = frames.clone()
    frames[3, 5, 70] = float("inf")
    p = replace(cfg.solver, levels=2, max_iter=150)
    rs.set_tuning(32, 16, resident=True)
    u, iters, status = rs.solve_batch(frames.cuda(), [0, 1, 2], [1, 2, 3], p)
    want = _oracle_batch(frames, [0, 1, 2], [1, 2, 3], p)
    st = host(status)
    for k in range(2):
        assert np.abs(host(u)[k] - want[k].u).max() <= TOL_PX
        assert host(iters)[k].tolist() == list(want[k].iters)
        assert st[k] == want[k].status
    assert st[2] & 2 and want[2].status & 2
    assert torch.isnan(u[2]).all()


def test_given_initial_guess(rs):
    announce("solve with u0")
    cfg, frames = _series(2, n_frames=3, height=64, width=64)
    p = replace(cfg.solver, levels=2, max_iter=100)
    rng = np.random.default_rng(1)
    u0 = smooth_field(rng, 2, 64, 64, 0.8)
    u, iters, _ = rs.solve_batch(frames.cuda(), [0, 0], [1, 2], p, u0=gpu(u0))
    want = _oracle_batch(frames, [0, 0], [1, 2], p, u0=u0)
    for b, w in enumerate(want):
        assert np.abs(host(u)[b] - w.u).max() <= TOL_PX
        assert host(iters)[b].tolist() == list(w.iters)


def test_fixed_iterations(rs):
    announce("fixed iterations")
    cfg, frames = _series(1, n_frames=3)
    p = cfg.solver   # 50 fixed updates, one level
    u, iters, status = rs.solve_batch(frames.cuda(), [0, 1], [1, 2], p)
    assert host(iters).tolist() == [[50], [50]]
    assert host(status).tolist() == [0, 0]
    want = _oracle_batch(frames, [0, 1], [1, 2], p)
    for b, w in enumerate(want):
        assert np.abs(host(u)[b] - w.u).max() <= TOL_PX


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_nonfinite_frame_is_flagged_and_isolated(rs, mode):
    announce(f"nonfinite {mode}")
    cfg, frames = _series(2, n_frames=4, height=64, width=64)
    frames = frames.clone()
    frames[2, 10, 10] = float("nan")
    p = replace(cfg.solver, levels=2, max_iter=50)
    u, iters, status = rs.solve_batch(frames.cuda(), [0, 1, 2], [1, 2, 3], p, mode=mode)
    st = host(status)
    assert st[0] == 0 or st[0] == 1
    assert st[1] & 2 and st[2] & 2
    assert torch.isnan(u[1]).all() and torch.isnan(u[2]).all()
    assert torch.isfinite(u[0]).all()
    want = _oracle_batch(frames, [0, 1, 2], [1, 2, 3], p)
    assert [w.status & 2 for w in want] == [0, 2, 2]
    assert host(iters)[1].tolist() == want[1].iters


def test_invalid_indices_rejected(rs):
    announce("invalid index")
    cfg, frames = _series(1, n_frames=3)
    with pytest.raises(rs.RegError):
        rs.solve_batch(frames.cuda(), [0], [7], cfg.solver)


def test_autotune_picks_a_candidate_and_keeps_results(rs):
    announce("autotune 64x64")
    cfg, frames = _series(2, n_frames=5, height=64, width=64)
    p = replace(cfg.solver, levels=2, max_iter=40)
    ref, tmpl = [0, 1, 2, 3], [1, 2, 3, 4]
    th, mg = rs.autotune(64, 64, 2, 8)
    assert th in (16, 32, 64) and mg in (1, 4, 8, 16, 32, 64, 128)
    assert rs.autotune(64, 64, 2, 8) == (th, mg)          # cached per shape
    u, iters, status = rs.solve_batch(frames.cuda(), ref, tmpl, p)
    want = _oracle_batch(frames, ref, tmpl, p)
    for b, w in enumerate(want):
        assert np.abs(host(u)[b] - w.u).max() <= TOL_PX
        assert host(iters)[b].tolist() == list(w.iters)
