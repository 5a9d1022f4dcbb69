"""Pins of the oracle's scan plans against the paper's counts (Table 1, the
dissemination figure, the Work columns of the full-registration table)."""
import json
import math
import os

import pytest

from oracle import plans

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "scan_work_counts.json")
SIZES = list(range(1, 40)) + [63, 64, 65, 100, 255, 256, 1023]


@pytest.mark.parametrize("algo", ["seq", "dissemination", "lf", "bk"])
def test_plans_compute_every_prefix(algo):
    for M in SIZES:
        ops, _ = plans.make_plan(M, algo)
        plans.check_plan(ops, M)


@pytest.mark.parametrize("glob", ["seq", "dissemination", "lf", "bk"])
@pytest.mark.parametrize("chunk", [0, 1, 2, 5, 16, 64])
def test_hier_plans_compute_every_prefix(glob, chunk):
    for M in [1, 2, 3, 7, 16, 33, 255, 300]:
        ops, _ = plans.make_plan(M, "hier", chunk, glob)
        plans.check_plan(ops, M)


def test_table1_work_and_depth():
    # Table 1 (Section 2.1): sequential N-1 / N-1; dissemination log2 N /
    # N log2 N - N + 1; Ladner-Fischer log2 N / < 4N - 5 (exact recursion).
    for m in range(1, 11):
        N = 1 << m
        ops, depth = plans.make_plan(N, "seq")
        assert (len(ops), depth) == (N - 1, N - 1)
        ops, depth = plans.make_plan(N, "dissemination")
        assert (len(ops), depth) == (N * m - N + 1, m)
        ops, depth = plans.make_plan(N, "lf")
        assert depth == m
        assert len(ops) == plans.lf_work(N)
        if N >= 4:
            assert len(ops) < 4 * N - 5
        # closed form of the same recursion: 4N - F(log2 N + 5) + 1
        if N >= 2:
            assert len(ops) == 4 * N - plans.fib(m + 5) + 1
        ops, depth = plans.make_plan(N, "bk")
        assert len(ops) == 2 * N - 2 - m
        assert depth <= 2 * m - 1


def test_dissemination_figure():
    g = json.load(open(GOLDEN))
    ops, depth = plans.make_plan(8, "dissemination")
    assert len(ops) == g["dissemination_8_ops"]
    assert depth == g["dissemination_8_rounds"]
    # round i performs N - 2^i applications
    per_level = [int((ops[:, 0] == l).sum()) for l in (1, 2, 3)]
    assert per_level == [7, 6, 4]


def test_table5_work_counts():
    g = json.load(open(GOLDEN))
    N = g["n_elements"]
    for P, wd, wl in zip(g["ranks"], g["work_dissemination"], g["work_ladner_fischer"]):
        for algo, want in (("dissemination", wd), ("lf", wl)):
            w_gs = len(plans.make_plan(P, algo)[0])
            assert N + (2 * N - P + w_gs) == want, (algo, P)


def test_hier_work():
    # reduce-then-scan with the chunk-0 fold reused and the chunk-end prefixes
    # taken from the global phase: (M - C) + W_GS(C) + (M - S) - (C - 1)
    for M, S in [(255, 16), (1023, 32), (4095, 64), (100, 7)]:
        C = math.ceil(M / S)
        w_gs = len(plans.make_plan(C, "lf")[0])
        ops, _ = plans.make_plan(M, "hier", S, "lf")
        last = M - (C - 1) * S
        want = (M - C) + w_gs + sum(S - 1 for _ in range(C - 2)) + (last - 1 if C > 1 else 0)
        assert len(ops) == want


def test_plan_ordering_is_canonical():
    ops, _ = plans.make_plan(100, "hier", 8, "dissemination")
    keys = [(r[0], r[6], r[4], r[5]) for r in ops]
    assert keys == sorted(keys)
    assert list(ops[:, 1]) == list(range(100, 100 + len(ops)))


def test_invalid_arguments():
    with pytest.raises(ValueError):
        plans.make_plan(0, "seq")
    with pytest.raises(ValueError):
        plans.make_plan(5, "nope")
