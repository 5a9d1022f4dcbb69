"""GPU reduce-then-scan with flexible segment boundaries (scan_run_flex,
Algorithm 1) against the oracle replaying the same combination order.

The boundaries depend on run-time speeds, so they are not unique: the test
checks that the recorded schedule is one Algorithm 1 can produce (segments
tile the series in worker order, each holds its worker's start, every step
absorbs an adjacent element, the first step goes right), then recomputes
every prefix on the CPU in that order from the frames alone."""
from dataclasses import replace

import numpy as np
import pytest
import torch

from oracle import plans as oplans
from oracle import registration as oreg
from oracle.scan import flex_orders, run_flex_scan
from synth import get_config, make_series

from _helpers import announce, host

pytestmark = pytest.mark.gpu

TOL_PX = 1e-3


@pytest.fixture(scope="module")
def rs():
    import paper_2010_12478_amd as rs
    rs.set_tuning(64, 64, resident=True)
    return rs


@pytest.mark.parametrize("N,workers,glob,levels", [(10, 2, "lf", 1), (14, 3, "lf", 2), (20, 5, "dissemination", 2),
                                                   (26, 8, "bk", 1), (13, 12, "seq", 1)])
def test_flex_scan_matches_oracle_replay(rs, N, workers, glob, levels):
    announce(f"flex N={N} workers={workers} {glob} L={levels}")
    cfg = get_config(2, n_frames=N, height=64, width=96, levels=levels)
    p = replace(cfg.solver, max_iter=80)
    S = make_series(cfg.series)
    phi0, u_pair, seg, step, counts, ms = rs.scan_run_flex(S.frames.cuda(), p, workers, glob)
    torch.cuda.synchronize()
    M = N - 1
    flex_orders(seg[:, :2], step, M)          # a schedule Algorithm 1 can produce
    want_phi0, want_pair = run_flex_scan(S.frames.double().numpy(), p, seg[:, :2], step, glob)
    e_pair = float(np.abs(host(u_pair) - want_pair).max())
    e_phi = float(np.abs(host(phi0) - want_phi0).max())
    print(f"segments {seg[:, :2].tolist()}: max-abs phi0 {e_phi:.2e} px, u_pair {e_pair:.2e} px")
    assert e_pair <= TOL_PX and e_phi <= TOL_PX
    gops, _ = oplans.make_plan(workers, glob)
    n3 = sum(int(seg[w][1] - seg[w][0]) for w in range(1, workers))
    assert counts == [M - workers, len(gops), n3, M + (M - workers) + len(gops) + n3]
    assert [int(x) for x in seg[:, 2]] == [int(seg[w][1] - seg[w][0]) for w in range(workers)]


def test_flex_scan_rejects_bad_arguments(rs):
    from paper_2010_12478_amd import RegError
    cfg = get_config(1, n_frames=5)
    fr = make_series(cfg.series).frames.cuda()
    with pytest.raises(RegError):
        rs.scan_run_flex(fr, cfg.solver, 1)
    with pytest.raises(RegError):
        rs.scan_run_flex(fr, cfg.solver, 5)       # more workers than elements
    with pytest.raises(RegError):
        rs.scan_run_flex(fr[:2].contiguous(), cfg.solver, 2)


def test_flex_scan_full_size_series256(rs):
    """The benchmark's series (256 frames 256x256, 2 levels, relative-decrease
    stopping) on 64 workers: a valid schedule, worker 0's first prefixes
    (the sequential recursion) and sampled pairwise registrations against the
    oracle."""
    announce("flex full size series256")
    cfg = get_config(2)
    p = cfg.solver
    S = make_series(cfg.series)
    phi0, u_pair, seg, step, counts, ms = rs.scan_run_flex(S.frames.cuda(), p, 64, "lf")
    torch.cuda.synchronize()
    M = 255
    orders = flex_orders(seg[:, :2], step, M)
    assert bool(torch.isfinite(phi0).all())
    fr = S.frames.double().numpy()
    P = {f: oreg.pyramid(fr[f], p.levels) for f in range(5)}
    y = oreg.register(P[0], P[1], None, p).u
    assert np.abs(host(u_pair[0]) - y).max() <= TOL_PX
    for k in (2, 3):
        if int(seg[0][1]) < k - 1:
            break
        x = oreg.register(P[k - 1], P[k], None, p).u
        assert np.abs(host(u_pair[k - 1]) - x).max() <= TOL_PX
        y = oreg.register(P[0], P[k], oreg.compose(y, x), p).u
        err = float(np.abs(host(phi0[k - 1]) - y).max())
        print(f"phi_0,{k}: max-abs {err:.2e} px")
        assert err <= TOL_PX
    print(f"segment lengths {[int(s[1] - s[0] + 1) for s in seg]}, ms {ms}")
