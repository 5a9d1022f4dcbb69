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


def _init_worker(pyrs, params, storage="f32"):
    _POOL_STATE["pyrs"] = pyrs
    _POOL_STATE["params"] = params
    _POOL_STATE["storage"] = storage


def _run_A(i):
    r = op_A(_POOL_STATE["pyrs"], i, _POOL_STATE["params"], _POOL_STATE["storage"])
    return r.u, r.iters, r.status


def _run_B(args):
    i, k, u_ij, u_jk = args
    r = op_B(_POOL_STATE["pyrs"], i, k, u_ij, u_jk, _POOL_STATE["params"], _POOL_STATE["storage"])
    return r.u, r.iters, r.status


@dataclass
class ScanResult:
    phi0: np.ndarray      # [M][2][H][W]: u_{0,k}, k = 1..M
    u_pair: np.ndarray    # [M][2][H][W]: u_{k-1,k}
    iters: np.ndarray     # [M + n_ops][levels]: A ops first, then plan ops
    status: np.ndarray    # [M + n_ops]
    ops: np.ndarray       # the plan


def frame_pyramids(frames, levels, storage="f32"):
    return [pyramid(np.asarray(f, dtype=np.float64), levels, storage) for f in frames]


def _map(fn, items, workers, pyrs, params, storage="f32"):
    if workers <= 1 or len(items) <= 1:
        _init_worker(pyrs, params, storage)
        return [fn(x) for x in items]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(min(workers, len(items)), initializer=_init_worker,
                  initargs=(pyrs, params, storage)) as pool:
        return pool.map(fn, items)


def run_scan(frames, params, algo="seq", chunk=0, global_algo="lf", workers=1,
             pyrs=None, storage="f32"):
    """Register every frame of ``frames`` ([N][H][W]) to frame 0 (``storage``:
    see ``oracle.registration``)."""
    N = len(frames)
    M = N - 1
    if pyrs is None:
        pyrs = frame_pyramids(frames, params.levels, storage)
    A = _map(_run_A, list(range(M)), workers, pyrs, params, storage)
    ops, n_levels = plans.make_plan(M, algo, chunk, global_algo)
    node = {m: A[m][0] for m in range(M)}
    iters = [A[m][1] for m in range(M)] + [None] * len(ops)
    status = [A[m][2] for m in range(M)] + [None] * len(ops)
    for lvl in range(1, n_levels + 1):
        rows = [n for n in range(len(ops)) if ops[n, 0] == lvl]
        args = [(int(ops[n, 4]), int(ops[n, 6]), node[int(ops[n, 2])], node[int(ops[n, 3])])
                for n in rows]
        res = _map(_run_B, args, workers, pyrs, params, storage)
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


# ------------------------------------------------ flexible segment boundaries

def flex_start(M, workers, w):
    """Algorithm 1's starting element of worker w (Section 4.3): the first
    element for worker 0, the last for the last worker, otherwise the middle
    of the static segment [w M / workers, (w + 1) M / workers)."""
    if w == 0:
        return 0
    if w == workers - 1:
        return M - 1
    s0, s1 = w * M // workers, (w + 1) * M // workers
    return (s0 + s1 - 1) // 2


def flex_orders(seg, step, M):
    """Per worker, the elements absorbed after its start in the order they
    were absorbed (step 1, 2, ...); checks that the schedule is one the
    algorithm can produce: segments tile [0, M) in worker order, each holds
    its worker's start (step 0), every step extends the segment by the
    adjacent element, and the first step goes right when it can."""
    workers = len(seg)
    orders = []
    for w in range(workers):
        pl, pr = int(seg[w][0]), int(seg[w][1])
        if w == 0 and pl != 0 or w == workers - 1 and pr != M - 1:
            raise ValueError("segments do not cover the series")
        if w > 0 and int(seg[w - 1][1]) + 1 != pl:
            raise ValueError(f"segments {w - 1} and {w} are not adjacent")
        start = flex_start(M, workers, w)
        if not pl <= start <= pr or step[start] != 0:
            raise ValueError(f"worker {w} did not start at element {start}")
        rest = sorted((int(step[e]), e) for e in range(pl, pr + 1) if e != start)
        if [s for s, _ in rest] != list(range(1, len(rest) + 1)):
            raise ValueError(f"worker {w} steps are not 1..{len(rest)}")
        lo = hi = start
        for n, (_, e) in enumerate(rest):
            if e == hi + 1:
                hi = e
            elif e == lo - 1:
                lo = e
            else:
                raise ValueError(f"worker {w} absorbed non-adjacent element {e}")
            if n == 0 and w < workers - 1 and e != start + 1:
                raise ValueError(f"worker {w} did not step right first")
        orders.append((start, [e for _, e in rest]))
    return orders


def run_flex_scan(frames, params, seg, step, global_algo="lf", pyrs=None):
    """The reduce-then-scan over flexible segments in the combination order a
    run recorded (segments and per-element steps): each worker's segment
    reduced from its start outward (B(res, x_e) to the right, B(x_e, res) to
    the left; worker 0's partial results are the prefixes), the global plan
    over the segment totals, then each later segment rescanned from the prefix
    before it.  Every value is computed here from the frames."""
    N = len(frames)
    M = N - 1
    if pyrs is None:
        pyrs = frame_pyramids(frames, params.levels)
    orders = flex_orders(seg, step, M)
    A = [op_A(pyrs, i, params).u for i in range(M)]
    phi0 = [None] * M
    phi0[0] = A[0]
    totals = []
    for w, (start, order) in enumerate(orders):
        res, lo, hi = A[start], start, start
        for e in order:
            if e == hi + 1:
                res = op_B(pyrs, lo, e + 1, res, A[e], params).u
                hi = e
                if w == 0:
                    phi0[e] = res
            else:
                res = op_B(pyrs, e, hi + 1, A[e], res, params).u
                lo = e
        totals.append(res)
    workers = len(orders)
    ops, _ = plans.make_plan(workers, global_algo)
    node = {w: totals[w] for w in range(workers)}
    for r in ops:
        i, k = int(r[4]), int(r[6])
        u = op_B(pyrs, int(seg[i][0]), int(seg[k - 1][1]) + 1, node[int(r[2])], node[int(r[3])], params).u
        node[int(r[1])] = u
        if i == 0:
            phi0[int(seg[k - 1][1])] = u
    for w in range(1, workers):
        cur = phi0[int(seg[w][0]) - 1]
        for e in range(int(seg[w][0]), int(seg[w][1])):
            cur = op_B(pyrs, 0, e + 1, cur, A[e], params).u
            phi0[e] = cur
    return np.stack(phi0), np.stack(A)
