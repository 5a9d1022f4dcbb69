"""Host-side checks of the C ABI: the library loads, exports every entry point
the header declares, validates arguments, and its scan planner reproduces the
oracle's plans bit for bit (no GPU needed)."""
import ctypes
import os
import re
import sys

import numpy as np
import pytest

from oracle import plans as oplans

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "regscan.h")


@pytest.fixture(scope="module")
def rs():
    import paper_2010_12478_amd as rs
    return rs


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:reg|scan)_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("reg_warp", "reg_energy_grad", "reg_solve_batch", "scan_run", "scan_plan",
                     "reg_warp_adjoint", "reg_last_error", "reg_release"):
        assert required in names


def test_library_exports_every_declared_symbol(rs):
    lib = ctypes.CDLL(rs.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2010_12478_amd._lib import EXPORTS
    assert sorted(EXPORTS) == declared_functions()


def test_version(rs):
    assert rs.lib.reg_version() == 100


CASES = ([(algo, M, 0, "lf") for algo in ("seq", "dissemination", "lf", "bk")
          for M in list(range(1, 34)) + [63, 64, 65, 127, 255, 256, 1000, 1023]]
         + [("hier", M, S, g) for g in ("seq", "dissemination", "lf", "bk")
            for M in (1, 2, 5, 16, 17, 100, 255, 1023) for S in (0, 1, 3, 8, 16, 32)])


@pytest.mark.parametrize("algo,M,S,glob", CASES)
def test_scan_plan_bit_exact_against_oracle(rs, algo, M, S, glob):
    got, nl = rs.plan(M, algo, S, glob)
    want, nl_want = oplans.make_plan(M, algo, S, glob)
    assert nl == nl_want
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def test_scan_plan_large(rs):
    for algo, S in (("hier", 64), ("lf", 0), ("dissemination", 0)):
        got, _ = rs.plan(4095, algo, S, "lf")
        want, _ = oplans.make_plan(4095, algo, S, "lf")
        assert np.array_equal(got, want)


def test_scan_plan_errors(rs):
    lib = rs.lib
    n, l = ctypes.c_int(), ctypes.c_int()
    assert lib.scan_plan(0, 0, 0, 0, None, 0, ctypes.byref(n), ctypes.byref(l)) == -1
    assert b"M = 0" in lib.reg_last_error()
    assert lib.scan_plan(10, 7, 0, 0, None, 0, ctypes.byref(n), ctypes.byref(l)) == -1
    assert lib.scan_plan(10, 4, 4, 9, None, 0, ctypes.byref(n), ctypes.byref(l)) == -1
    # capacity too small: size still reported
    buf = (ctypes.c_int32 * 7)()
    assert lib.scan_plan(8, 1, 0, 0, ctypes.cast(buf, ctypes.c_void_p), 1, ctypes.byref(n),
                         ctypes.byref(l)) == -1
    assert n.value == 17


def test_invalid_arguments_rejected_before_any_gpu_use(rs):
    lib = rs.lib
    from paper_2010_12478_amd._lib import params_struct
    from synth.configs import SolverParams
    p = params_struct(SolverParams(levels=3))
    # 18x18 is not divisible by 4 -> rejected on the host
    rc = lib.scan_run(ctypes.c_void_p(16), 4, 18, 18, ctypes.byref(p), 0, 0, 0, 1, 0,
                      ctypes.c_void_p(16), None, None, None, None)
    assert rc == -1 and b"divisible" in lib.reg_last_error()
    bad = params_struct(SolverParams(levels=1, tau=-1.0))
    rc = lib.scan_run(ctypes.c_void_p(16), 4, 16, 16, ctypes.byref(bad), 0, 0, 0, 1, 0,
                      ctypes.c_void_p(16), None, None, None, None)
    assert rc == -1 and b"tau" in lib.reg_last_error()
    rc = lib.scan_run(ctypes.c_void_p(16), 1, 16, 16, ctypes.byref(p), 0, 0, 0, 1, 0,
                      ctypes.c_void_p(16), None, None, None, None)
    assert rc == -1
    assert lib.reg_set_tuning(6, 0, -1) == -1
    assert lib.reg_set_tuning(0, 129, -1) == -1
    assert lib.reg_set_tuning(0, 0, 2) == -1


def test_rigid_arguments_rejected_before_any_gpu_use(rs):
    lib = rs.lib
    from paper_2010_12478_amd._lib import params_struct
    from synth import RIGID_TAU
    from synth.configs import SolverParams
    p = params_struct(SolverParams(levels=2, tau=RIGID_TAU))
    ref = (ctypes.c_int32 * 1)(0)
    bad_idx = (ctypes.c_int32 * 1)(5)
    out = ctypes.c_void_p(16)
    # template index outside [0, N)
    rc = lib.reg_rigid_solve_batch(ctypes.c_void_p(16), 2, 32, 32, ref, bad_idx, None, out, None, None, 1,
                                   ctypes.byref(p), None)
    assert rc == -1 and b"out of range" in lib.reg_last_error()
    # 18x18 is not divisible by 2^(levels-1) = 4
    p3 = params_struct(SolverParams(levels=3, tau=RIGID_TAU))
    rc = lib.reg_rigid_solve_batch(ctypes.c_void_p(16), 2, 18, 18, ref, ref, None, out, None, None, 1,
                                   ctypes.byref(p3), None)
    assert rc == -1 and b"divisible" in lib.reg_last_error()
    # theta aliasing theta0
    rc = lib.reg_rigid_solve_batch(ctypes.c_void_p(16), 2, 32, 32, ref, ref, out, out, None, None, 1,
                                   ctypes.byref(p), None)
    assert rc == -1 and b"alias" in lib.reg_last_error()
    # scan: a single frame, an unknown mode, an unknown algorithm
    rc = lib.scan_run_rigid(ctypes.c_void_p(16), 1, 32, 32, ctypes.byref(p), 0, 0, 0, 1, out, None, None, None,
                            None)
    assert rc == -1
    rc = lib.scan_run_rigid(ctypes.c_void_p(16), 4, 32, 32, ctypes.byref(p), 0, 0, 0, 0, out, None, None, None,
                            None)
    assert rc == -1 and b"mode" in lib.reg_last_error()
    rc = lib.scan_run_rigid(ctypes.c_void_p(16), 4, 32, 32, ctypes.byref(p), 9, 0, 0, 1, out, None, None, None,
                            None)
    assert rc == -1 and b"algorithm" in lib.reg_last_error()


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_algorithmic_counts():
    """The roofline's per-step counts from iteration counts: the rigid pixel
    passes (t + 1 evaluations for a level stopped at t, max_iter when capped)
    and the dense bytes for a hand-counted case."""
    import numpy as np
    b = _bench()
    it = np.array([[3, 0], [200, 5]])          # two registrations, 2 levels, cap 200
    assert b.pixel_passes(it, 8, 8, 2, 200) == (4 + 200) * 64 + (1 + 6) * 16
    one = b.algorithmic_bytes(np.array([[2]]), 1, 4, 4, 1, 50)
    two = b.algorithmic_bytes(np.array([[3]]), 1, 4, 4, 1, 50)
    assert two - one == b.SWEEP_BYTES * 16      # one more kept update of a 4x4 field


def test_bench_traffic_records(tmp_path, monkeypatch):
    """The roofline's traffic fields from the committed counter records: a
    direct record gives bytes per launch, a per-level record composes bytes
    per pixel pass with the launch's pixel passes per level, and a record
    taken on other kernel sources gives nothing."""
    import json
    import numpy as np
    b = _bench()
    sha = b.kernel_sources_sha256()
    monkeypatch.setattr(b, "traffic_file", lambda name: str(tmp_path / f"{name}.json"))
    assert b.measured_traffic("none") is None and b.traffic_estimate("none", None, 1, 1, 1, 1, 1) is None
    (tmp_path / "direct.json").write_text(json.dumps({"sources_sha256": sha, "hbm_bytes_per_dispatch": 1234}))
    assert b.measured_traffic("direct") == 1234
    (tmp_path / "stale.json").write_text(json.dumps({"sources_sha256": "0" * 64, "hbm_bytes_per_dispatch": 1}))
    assert b.measured_traffic("stale") is None
    (tmp_path / "levels.json").write_text(json.dumps({"sources_sha256": sha, "bytes_per_pixel_pass": [30.0, 20.0]}))
    assert b.measured_traffic("levels") is None            # no direct figure for that launch
    it = np.array([[3, 200], [0, 7]])                       # two registrations, 2 levels, cap 200
    est = b.traffic_estimate("levels", it, 8, 8, 2, 200, 1000)
    passes = [(4 + 1) * 64, (200 + 8) * 16]                 # t + 1 evaluations, max_iter when capped
    assert est["bytes"] == int(30.0 * passes[0] + 20.0 * passes[1])
    assert est["per_algorithmic"] == round(est["bytes"] / 1000, 4)


def test_size_limits_rejected_before_any_gpu_use(rs):
    """Largest accepted frame: 16384 px per side and 2^26 pixels; beyond that,
    and for non-positive sizes or batches, every entry point fails on the host."""
    lib = rs.lib
    from paper_2010_12478_amd._lib import params_struct
    from synth.configs import SolverParams
    p = params_struct(SolverParams(levels=1))
    ref = (ctypes.c_int32 * 1)(0)
    out = ctypes.c_void_p(16)
    for H, W in ((16385, 64), (64, 16385), (8192, 16384), (0, 64), (64, -1)):
        rc = lib.reg_solve_batch(ctypes.c_void_p(16), 1, H, W, ref, ref, None, out, None, None, 1,
                                 ctypes.byref(p), 1, None)
        assert rc == -1, (H, W)
        rc = lib.reg_rigid_solve_batch(ctypes.c_void_p(16), 1, H, W, ref, ref, None, out, None, None, 1,
                                       ctypes.byref(p), None)
        assert rc == -1, (H, W)
        rc = lib.scan_run(ctypes.c_void_p(16), 4, H, W, ctypes.byref(p), 0, 0, 0, 1, 0, out, None, None, None, None)
        assert rc == -1, (H, W)
    rc = lib.reg_solve_batch(ctypes.c_void_p(16), 1, 64, 64, ref, ref, None, out, None, None, -1,
                             ctypes.byref(p), 1, None)
    assert rc == -1 and b"batch" in lib.reg_last_error()
