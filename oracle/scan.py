"""Series registration as a prefix scan, CPU oracle.  TEST INFRASTRUCTURE ONLY.

Runs the paper's two phases (Section 3): the pairwise registrations
phi_{k-1,k} = A(f_{k-1}, f_k), then the plan's operator applications level by
level, each phi_ik = B(phi_ij, phi_jk).  Independent applications of one plan
level may be spread over worker processes (one per host core).
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

from . import plans
from .registration import op_A, op_B, pyramid

_POOL_STATE = {}


def _init_worker(pyrs, params):
    _POOL_STATE["pyrs"] = pyrs
    _POOL_STATE["params"] = params


def _run_A(i):
    r = op_A(_POOL_STATE["pyrs"], i, _POOL_STATE["params"])
    return r.u, r.iters, r.status


def _run_B(args):
    i, k, u_ij, u_jk = args
    r = op_B(_POOL_STATE["pyrs"], i, k, u_ij, u_jk, _POOL_STATE["params"])
    return r.u, r.iters, r.status


@dataclass
class ScanResult:
    phi0: np.ndarray      # [M][2][H][W]: u_{0,k}, k = 1..M
    u_pair: np.ndarray    # [M][2][H][W]: u_{k-1,k}
    iters: np.ndarray     # [M + n_ops][levels]: A ops first, then plan ops
    status: np.ndarray    # [M + n_ops]
    ops: np.ndarray       # the plan


def frame_pyramids(frames, levels):
    return [pyramid(np.asarray(f, dtype=np.float64), levels) for f in frames]


def _map(fn, items, workers, pyrs, params):
    if workers <= 1 or len(items) <= 1:
        _init_worker(pyrs, params)
        return [fn(x) for x in items]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(min(workers, len(items)), initializer=_init_worker,
                  initargs=(pyrs, params)) as pool:
        return pool.map(fn, items)


def run_scan(frames, params, algo="seq", chunk=0, global_algo="lf", workers=1,
             pyrs=None):
    """Register every frame of ``frames`` ([N][H][W]) to frame 0."""
    N = len(frames)
    M = N - 1
    if pyrs is None:
        pyrs = frame_pyramids(frames, params.levels)
    A = _map(_run_A, list(range(M)), workers, pyrs, params)
    ops, n_levels = plans.make_plan(M, algo, chunk, global_algo)
    node = {m: A[m][0] for m in range(M)}
    iters = [A[m][1] for m in range(M)] + [None] * len(ops)
    status = [A[m][2] for m in range(M)] + [None] * len(ops)
    for lvl in range(1, n_levels + 1):
        rows = [n for n in range(len(ops)) if ops[n, 0] == lvl]
        args = [(int(ops[n, 4]), int(ops[n, 6]), node[int(ops[n, 2])], node[int(ops[n, 3])])
                for n in rows]
        res = _map(_run_B, args, workers, pyrs, params)
        for n, (u, it, st) in zip(rows, res):
            node[int(ops[n, 1])] = u
            iters[M + n] = it
            status[M + n] = st
    fin = plans.final_nodes(ops, M)
    phi0 = np.stack([node[int(fin[k])] for k in range(M)])
    u_pair = np.stack([A[m][0] for m in range(M)])
    return ScanResult(phi0, u_pair, np.array(iters, dtype=np.int64),
                      np.array(status, dtype=np.int64), ops)


def host_cores():
    return len(os.sched_getaffinity(0))
