"""Pins of the mock-operator oracle (the paper's microbenchmarks, Section 5):
the counter-based operator times, the range semantics of every plan, and the
simulated execution forms, including Algorithm 1 (Section 4.3)."""
import numpy as np
import pytest

from oracle import mock, plans


def test_splitmix64_reference_outputs():
    # splitmix64 seeded with 0 (state advanced by the golden gamma before each
    # output): its first outputs as published with the generator
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    got = [mock.splitmix64_finalizer(mock.GOLDEN * n) for n in range(1, 5)]
    assert got == want
    # the counter of application (i, k) = (n - 1, 0) with seed 0 is that state
    assert mock.uniform(0, 0, 0) == (want[0] >> 11) * 2.0 ** -53


def test_operator_time_distributions():
    n = 200_000
    exp = np.array([mock.op_time(10.0, "exp", 1410, i, i + 3) for i in range(n)])
    assert abs(exp.mean() - 10.0) < 0.1            # mean t (std error 0.022)
    assert abs(np.median(exp) - 10.0 * np.log(2)) < 0.1
    assert exp.max() <= mock.CAP * 10.0
    frame = np.array([mock.op_time(10.0, "frame", 1410, i, i + 3) for i in range(n)])
    assert abs(frame.mean() - 10.0) < 0.1          # mean of two draws of mean t
    assert mock.op_time(10.0, "static", 1410, 3, 9) == 10.0
    # frame model: every application touching frame f shares its difficulty
    d = mock.exp_draw(10.0, 1410, 5, 5)
    assert mock.op_time(10.0, "frame", 1410, 5, 5) == d
    # deterministic in the application, different between applications
    assert mock.op_time(10.0, "exp", 7, 2, 9) == mock.op_time(10.0, "exp", 7, 2, 9)
    assert mock.op_time(10.0, "exp", 7, 2, 9) != mock.op_time(10.0, "exp", 7, 2, 10)


def test_apply_checks_adjacency():
    assert mock.apply((0, 3), (3, 8)) == (0, 8)
    with pytest.raises(ValueError):
        mock.apply((0, 3), (4, 8))


@pytest.mark.parametrize("algo,chunk,glob", [("seq", 0, "lf"), ("dissemination", 0, "lf"), ("lf", 0, "lf"),
                                             ("bk", 0, "lf"), ("hier", 5, "lf"), ("hier", 3, "dissemination")])
@pytest.mark.parametrize("M", [1, 2, 7, 64, 100])
def test_every_plan_yields_every_prefix(algo, chunk, glob, M):
    ops, _ = plans.make_plan(M, algo, chunk, glob)
    assert np.array_equal(mock.run_plan(M, ops), mock.expected_prefixes(M))


def test_level_simulation_with_static_times():
    M, P = 64, 1000
    for algo in ("dissemination", "lf", "bk"):
        ops, nl = plans.make_plan(M, algo)
        # every level fits the workers: one operator time per level
        assert mock.simulate_levels(M, ops, P, 2.0, "static", 0, queued=False) == 2.0 * nl
        assert mock.simulate_levels(M, ops, P, 2.0, "static", 0, queued=True) == 2.0 * nl
    ops, nl = plans.make_plan(M, "seq")
    assert mock.simulate_dataflow(M, ops, 4, 1.0, "static", 0)[0] == M - 1


@pytest.mark.parametrize("steal", [False, True])
@pytest.mark.parametrize("M,P", [(2, 2), (9, 2), (100, 7), (1000, 16)])
def test_phase1_segments_are_valid(steal, M, P):
    for dist in ("static", "exp", "frame"):
        fin, segs, res = mock.simulate_phase1(M, P, 1.0, dist, 1410, steal)
        assert mock.valid_segments(segs, M, P, steal)
        for (a, b), r in zip(segs, res):
            assert r == (a, b + 1)


def test_static_segments_take_their_length():
    fin, segs, _ = mock.simulate_phase1(100, 4, 1.0, "static", 0, steal=False)
    assert fin == [24.0, 24.0, 24.0, 24.0]


def test_two_workers_meet_in_the_middle():
    # Algorithm 1 with equal operator times: worker 0 starts at element 0
    # (moves right), worker 1 at the last (moves left); they split the gap
    for M in (2, 3, 10, 11, 101):
        _, segs, _ = mock.simulate_phase1(M, 2, 1.0, "static", 0, steal=True)
        n0, n1 = segs[0][1] - segs[0][0] + 1, segs[1][1] - segs[1][0] + 1
        assert n0 + n1 == M and abs(n0 - n1) <= 1


def test_stealing_balances_phase1_under_frame_difficulty():
    # a slow segment hands elements to its neighbours: the slowest worker of
    # phase 1 finishes earlier than with static segments
    M, P = 4096, 64
    t_static, _, _ = mock.simulate_phase1(M, P, 1.0, "frame", 1410, steal=False)
    t_flex, _, _ = mock.simulate_phase1(M, P, 1.0, "frame", 1410, steal=True)
    assert max(t_flex) < 0.8 * max(t_static)
