"""ctypes binding of libregscan.so: argument marshalling only.

Every computation happens in the library's HIP kernels.  Torch tensors supply
device memory and the current HIP stream; nothing here falls back to a CPU or
PyTorch implementation: if the library is missing, importing this package
fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch's HIP runtime first: the library then binds to the runtime already in
# the process (loaded the other way round, two runtimes end up in one process
# and the library finds no device)
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libregscan.so")

REG_OK, REG_E_INVALID, REG_E_NOMEM, REG_E_HIP, REG_E_NODEVICE = 0, -1, -2, -3, -4
REG_S_OK, REG_S_MAXITER, REG_S_NONFINITE, REG_S_ABORTED = 0, 1, 2, 4
SCAN_ALGOS = {"seq": 0, "dissemination": 1, "lf": 2, "bk": 3, "hier": 4}
MODES = {"plain": 0, "batched": 1, "dataflow": 2}
SCAN_F_GRAPH = 1

EXPORTS = (
    "reg_last_error", "reg_version", "reg_pyramid", "reg_warp", "reg_warp_f64",
    "reg_warp_adjoint", "reg_warp_adjoint_f64", "reg_energy_grad", "reg_energy_grad_f64", "reg_energy_grad_noalloc",
    "reg_pyramid_energy", "reg_pyramid_energy_f64", "reg_pyramid_energy_backward",
    "reg_pyramid_energy_backward_f64", "reg_compose", "reg_restrict", "reg_prolong",
    "reg_solve_batch", "scan_plan", "scan_run", "reg_last_solve_timing", "reg_last_solve_launch_ms",
    "reg_set_tuning",
    "reg_autotune", "reg_release", "scan_mock_run", "scan_run_flex", "reg_rigid_solve_batch", "scan_run_rigid",
)


class RegError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"regscan error {code}: {message}")
        self.code = code


class reg_params_t(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("fixed_iter", ctypes.c_int32), ("tau", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("rel_tol", ctypes.c_double)]


class mock_params_t(ctypes.Structure):
    _fields_ = [("mean_us", ctypes.c_double), ("dist", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


MOCK_DISTS = {"static": 0, "exp": 1, "frame": 2}
MOCK_MODES = {"level_static": 0, "level_queued": 1, "dataflow": 2, "segments": 3, "flex": 4}


class scan_op_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("level", "out", "a", "b", "i", "j", "k")]


_P = ctypes.c_void_p
_I = ctypes.c_int
_F = ctypes.c_float
_D = ctypes.c_double

_SIGS = {
    "reg_last_error": (ctypes.c_char_p, []),
    "reg_version": (_I, []),
    "reg_pyramid": (_I, [_P, _P, _I, _I, _I, _I, _P]),
    "reg_warp": (_I, [_P, _P, _P, _I, _I, _I, _P]),
    "reg_warp_f64": (_I, [_P, _P, _P, _I, _I, _I, _P]),
    "reg_warp_adjoint": (_I, [_P, _P, _P, _I, _I, _I, _P]),
    "reg_warp_adjoint_f64": (_I, [_P, _P, _P, _I, _I, _I, _P]),
    "reg_energy_grad": (_I, [_P, _P, _P, _D, _P, _P, _P, _I, _I, _I, _P]),
    "reg_energy_grad_f64": (_I, [_P, _P, _P, _D, _P, _P, _P, _I, _I, _I, _P]),
    "reg_energy_grad_noalloc": (_I, [_P, _P, _P, _D, _P, _P, _P, _I, _I, _I, _P]),
    "reg_pyramid_energy": (_I, [_P, _P, _P, _D, _I, _P, _I, _I, _I, _P]),
    "reg_pyramid_energy_f64": (_I, [_P, _P, _P, _D, _I, _P, _I, _I, _I, _P]),
    "reg_pyramid_energy_backward": (_I, [_P, _P, _P, _D, _I, _P, _P, _P, _P, _I, _I, _I, _P]),
    "reg_pyramid_energy_backward_f64": (_I, [_P, _P, _P, _D, _I, _P, _P, _P, _P, _I, _I, _I, _P]),
    "reg_compose": (_I, [_P, _P, _P, _I, _I, _I, _P]),
    "reg_restrict": (_I, [_P, _P, _D, _I, _I, _I, _P]),
    "reg_prolong": (_I, [_P, _P, _I, _I, _I, _P]),
    "reg_solve_batch": (_I, [_P, _I, _I, _I, _P, _P, _P, _P, _P, _P, _I,
                             ctypes.POINTER(reg_params_t), _I, _P]),
    "scan_plan": (_I, [_I, _I, _I, _I, _P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "scan_run": (_I, [_P, _I, _I, _I, ctypes.POINTER(reg_params_t), _I, _I, _I, _I, _I,
                      _P, _P, _P, _P, _P]),
    "reg_last_solve_timing": (_I, [ctypes.POINTER(_D), ctypes.POINTER(_I)]),
    "reg_set_tuning": (_I, [_I, _I, _I]),
    "reg_last_solve_launch_ms": (_I, [ctypes.POINTER(ctypes.c_double), _I, ctypes.POINTER(_I)]),
    "reg_autotune": (_I, [_I, _I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), _P]),
    "reg_release": (None, []),
    "scan_mock_run": (_I, [_I, _I, _I, _I, _I, _I, _P, _P, _P, _P, _P, _P]),
    "scan_run_flex": (_I, [_P, _I, _I, _I, _P, _I, _I, _P, _P, _P, _P, _P, _P, _P]),
    "reg_rigid_solve_batch": (_I, [_P, _I, _I, _I, _P, _P, _P, _P, _P, _P, _I, _P, _P]),
    "scan_run_rigid": (_I, [_P, _I, _I, _I, _P, _I, _I, _I, _I, _P, _P, _P, _P, _P]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built: run `python -m paper_2010_12478_amd.build` "
            "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(code):
    if code != REG_OK:
        raise RegError(code, lib.reg_last_error().decode())
    return code


def params_struct(p) -> reg_params_t:
    """reg_params_t from any object with levels, max_iter, fixed_iter, tau, lam, rel_tol."""
    return reg_params_t(int(p.levels), int(p.max_iter), int(bool(p.fixed_iter)),
                        float(p.tau), float(p.lam), float(p.rel_tol))


def plan(M: int, algo: str, chunk: int = 0, global_algo: str = "lf") -> np.ndarray:
    """scan_plan through the C ABI (host only): int64 array [n_ops][7]."""
    a, gl = SCAN_ALGOS[algo], SCAN_ALGOS[global_algo]
    n_ops, n_lv = _I(0), _I(0)
    check(lib.scan_plan(M, a, chunk, gl, None, 0, ctypes.byref(n_ops), ctypes.byref(n_lv)))
    buf = (scan_op_t * max(1, n_ops.value))()
    check(lib.scan_plan(M, a, chunk, gl, ctypes.cast(buf, _P), n_ops.value,
                        ctypes.byref(n_ops), ctypes.byref(n_lv)))
    out = np.zeros((n_ops.value, 7), dtype=np.int64)
    for n in range(n_ops.value):
        o = buf[n]
        out[n] = (o.level, o.out, o.a, o.b, o.i, o.j, o.k)
    return out, n_lv.value
