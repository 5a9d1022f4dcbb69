"""GPU mock-operator scan (scan_mock_run) against the oracle: every execution
form computes every prefix (0, e + 1) with no adjacency violation, the level
forms apply exactly the plan's operators, the segment forms leave a valid
partition of the elements (static bounds, or the flexible boundaries of
Algorithm 1 around each worker's start), and the waits really happen."""
import numpy as np
import pytest
import torch

from oracle import mock, plans

from _helpers import announce, host

pytestmark = pytest.mark.gpu

LEVEL_FORMS = ["level_static", "level_queued", "dataflow"]


@pytest.fixture(scope="module")
def rs():
    import paper_2010_12478_amd as rs
    return rs


@pytest.mark.parametrize("form", LEVEL_FORMS)
@pytest.mark.parametrize("algo,chunk,glob", [("seq", 0, "lf"), ("dissemination", 0, "lf"), ("lf", 0, "lf"),
                                             ("bk", 0, "lf"), ("hier", 16, "lf"), ("hier", 5, "dissemination")])
@pytest.mark.parametrize("M", [1, 2, 37, 1000])
def test_level_forms_compute_every_prefix(rs, form, algo, chunk, glob, M):
    if algo == "seq" and M > 100:
        M = 100
    announce(f"mock {form} {algo}/{chunk}/{glob} M={M}")
    prefix, _, counts, ms = rs.scan_mock(M, form, 64, 0.2, "exp", 1410, algo, chunk, glob)
    torch.cuda.synchronize()
    ops, _ = plans.make_plan(M, algo, chunk, glob)
    assert np.array_equal(host(prefix).astype(np.int64), mock.expected_prefixes(M))
    assert counts[4] == 0
    assert counts[0] == len(ops) and counts[3] == len(ops)


@pytest.mark.parametrize("form", ["segments", "flex"])
@pytest.mark.parametrize("glob", ["seq", "dissemination", "lf", "bk"])
@pytest.mark.parametrize("M,P", [(2, 2), (9, 2), (100, 7), (5000, 64)])
@pytest.mark.parametrize("dist", ["static", "exp", "frame"])
def test_segment_forms(rs, form, glob, M, P, dist):
    announce(f"mock {form} {glob} M={M} P={P} {dist}")
    prefix, seg, counts, ms = rs.scan_mock(M, form, P, 0.5, dist, 1410, "lf", 0, glob, want_seg=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(prefix).astype(np.int64), mock.expected_prefixes(M))
    assert counts[4] == 0
    segs = host(seg)
    assert mock.valid_segments(segs, M, P, steal=form == "flex")
    gops, _ = plans.make_plan(P, glob)
    assert counts[0] == M - P and counts[1] == len(gops)
    assert counts[2] == M - (segs[0][1] - segs[0][0] + 1)
    assert counts[3] == counts[0] + counts[1] + counts[2]


def test_single_worker_segments(rs):
    prefix, seg, counts, _ = rs.scan_mock(50, "segments", 1, 0.1, "exp", 3, "lf", 0, "lf", want_seg=True)
    assert np.array_equal(host(prefix).astype(np.int64), mock.expected_prefixes(50))
    assert counts[:4] == [49, 0, 0, 49]


def test_waits_take_their_time(rs):
    # static operator time t: a static segment of L elements takes (L - 1) t,
    # and the sequential plan M - 1 applications of t
    M, P, t = 4096, 16, 20.0
    _, _, counts, ms = rs.scan_mock(M, "segments", P, t, "static", 0, "lf", 0, "lf")
    assert ms[0] * 1000.0 >= (M // P - 1) * t * 0.999
    assert ms[0] * 1000.0 <= (M // P - 1) * t * 1.5 + 200.0
    _, _, counts, ms = rs.scan_mock(200, "dataflow", 64, t, "static", 0, "seq")
    assert ms[3] * 1000.0 >= 199 * t * 0.999


def test_full_size_microbenchmark_shapes(rs):
    # the paper's 98,304 elements on 1024 workers, dynamic operator times
    M, P = 98304, 1024
    for form in ("segments", "flex"):
        announce(f"mock full size {form}")
        prefix, seg, counts, ms = rs.scan_mock(M, form, P, 2.0, "frame", 1410, "lf", 0, "lf", want_seg=True)
        torch.cuda.synchronize()
        assert np.array_equal(host(prefix).astype(np.int64), mock.expected_prefixes(M))
        assert counts[4] == 0
        assert mock.valid_segments(host(seg), M, P, steal=form == "flex")
    for form in LEVEL_FORMS:
        announce(f"mock full size {form}")
        prefix, _, counts, _ = rs.scan_mock(M, form, P, 2.0, "exp", 1410, "lf")
        assert np.array_equal(host(prefix).astype(np.int64), mock.expected_prefixes(M))
        assert counts[4] == 0


def test_invalid_arguments_rejected(rs):
    from paper_2010_12478_amd import RegError
    with pytest.raises(RegError):
        rs.scan_mock(10, "flex", 1, 1.0)          # stealing needs two workers
    with pytest.raises(RegError):
        rs.scan_mock(10, "segments", 11, 1.0)     # more workers than elements
    with pytest.raises(RegError):
        rs.scan_mock(0, "dataflow", 4, 1.0)
    with pytest.raises(RegError):
        rs.scan_mock(10, "dataflow", 10 ** 7, 1.0)  # more workers than can be resident
