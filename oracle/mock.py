"""Mock-operator prefix scan, CPU oracle.  TEST INFRASTRUCTURE ONLY.

The paper's microbenchmarks (Section 5) run the scan algorithms on an
artificial operator whose application takes a static time t or a time drawn
from an exponential distribution with rate 1/t.  Here a scan node is the frame
range (i, k) it covers (element e = (e, e + 1)); the operator maps (i, j) and
(j, k) to (i, k).  The time of the application yielding (i, k) comes from a
counter-based generator, so it is the same wherever and whenever the
application is executed:

    z = seed + 0x9E3779B97F4A7C15 * (1 + i + 2^32 k)   (mod 2^64)
    u = splitmix64_finalizer(z) >> 11, scaled by 2^-53
    time = t (static)  or  -t ln(1 - u) (exponential), at most 64 t
    frame model: time = (d_i + d_k) / 2 with d_f the exponential draw of (f, f)

(splitmix64: Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", 2014).

Besides the outputs every execution form must produce (the prefixes (0, e+1))
and its operator counts, this module simulates the execution forms in
virtual time with these operator times: list scheduling of plan levels
(static round robin or a shared queue), the dataflow ready queue, and the
reduce-then-scan over static or flexible segments, the latter following
Algorithm 1 (Section 4.3): each worker starts in the middle of its segment,
steps right once, then extends toward whichever neighbour is slower (time
per application so far), or toward the only side with unclaimed elements.
"""
from __future__ import annotations

import heapq
import math

import numpy as np

from . import plans

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
CAP = 64.0


def splitmix64_finalizer(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def uniform(seed: int, i: int, k: int) -> float:
    z = (seed + GOLDEN * (1 + i + (k << 32))) & MASK64
    return (splitmix64_finalizer(z) >> 11) * 2.0 ** -53


def exp_draw(mean: float, seed: int, i: int, k: int) -> float:
    return min(-mean * math.log1p(-uniform(seed, i, k)), CAP * mean)


def op_time(mean: float, dist: str, seed: int, i: int, k: int) -> float:
    """Time of the application yielding (i, k), in the unit of `mean`:
    static t; "exp": exponential with rate 1/t, independent per application;
    "frame": the mean of the difficulties of frames i and k, each exponential
    with rate 1/t (the draw keyed (f, f)), so that every application touching
    a slow frame is slow."""
    if dist == "static":
        return mean
    if dist == "frame":
        return 0.5 * (exp_draw(mean, seed, i, i) + exp_draw(mean, seed, k, k))
    return exp_draw(mean, seed, i, k)


def apply(left, right):
    """(i, j) (.) (j, k) = (i, k); raises on non-adjacent operands."""
    if left[1] != right[0]:
        raise ValueError(f"operands {left} and {right} are not adjacent")
    return (left[0], right[1])


def expected_prefixes(M: int) -> np.ndarray:
    return np.stack([np.zeros(M, np.int64), np.arange(1, M + 1)], axis=1)


def run_plan(M: int, ops: np.ndarray) -> np.ndarray:
    """Executes a plan on range nodes; returns the range computed for every
    element's final node (the prefix (0, e + 1) when the plan is correct)."""
    node = {m: (m, m + 1) for m in range(M)}
    for r in ops:
        node[int(r[1])] = apply(node[int(r[2])], node[int(r[3])])
    fin = plans.final_nodes(ops, M)
    return np.array([node[int(fin[e])] for e in range(M)], dtype=np.int64)


# ----------------------------------------------------------------- simulation

def simulate_levels(M, ops, workers, mean, dist, seed, queued):
    """Level-synchronous execution: per level, static round robin (op q on
    worker q mod workers, in order) or list scheduling from a shared queue."""
    total = 0.0
    for lvl in range(1, int(ops[:, 0].max()) + 1 if len(ops) else 1):
        rows = ops[ops[:, 0] == lvl]
        times = [op_time(mean, dist, seed, int(r[4]), int(r[6])) for r in rows]
        if queued:
            heap = [0.0] * min(workers, len(times))
            for t in times:
                heapq.heappush(heap, heapq.heappop(heap) + t)
            total += max(heap) if heap else 0.0
        else:
            load = np.zeros(workers)
            for q, t in enumerate(times):
                load[q % workers] += t
            total += load.max()
    return total


def simulate_dataflow(n_base, ops, workers, mean, dist, seed, start=None):
    """One pass over the plan: an op becomes ready when its inputs are done;
    free workers take ready ops in the order they became ready (FIFO).
    `start` gives the availability time of every element (default 0)."""
    n = len(ops)
    avail = {m: (0.0 if start is None else start[m]) for m in range(n_base)}
    deps = {}
    cons = {}
    for q, r in enumerate(ops):
        a, b = int(r[2]), int(r[3])
        deps[q] = sum(1 for x in (a, b) if x >= n_base)
        for x in (a, b):
            if x >= n_base:
                cons.setdefault(x, []).append(q)
    ready = []   # (ready time, sequence, op)
    seq = 0
    for q, r in enumerate(ops):
        if deps[q] == 0:
            heapq.heappush(ready, (max(avail[int(r[2])], avail[int(r[3])]), seq, q))
            seq += 1
    free = [0.0] * workers
    heapq.heapify(free)
    done_at = {}
    end = 0.0
    while ready:
        t_ready, _, q = heapq.heappop(ready)
        w = heapq.heappop(free)
        r = ops[q]
        t0 = max(w, t_ready)
        t1 = t0 + op_time(mean, dist, seed, int(r[4]), int(r[6]))
        heapq.heappush(free, t1)
        out = int(r[1])
        done_at[out] = t1
        end = max(end, t1)
        for c in cons.get(out, []):
            deps[c] -= 1
            if deps[c] == 0:
                rc = ops[c]
                ta = done_at.get(int(rc[2]), avail.get(int(rc[2]), 0.0))
                tb = done_at.get(int(rc[3]), avail.get(int(rc[3]), 0.0))
                heapq.heappush(ready, (max(ta, tb), seq, c))
                seq += 1
    return end, done_at


def static_bounds(M, workers):
    return [(w * M // workers, (w + 1) * M // workers) for w in range(workers)]


def flex_start(M, workers, w):
    s0, s1 = static_bounds(M, workers)[w]
    if w == 0:
        return 0
    if w == workers - 1:
        return M - 1
    return (s0 + s1 - 1) // 2


def simulate_phase1(M, workers, mean, dist, seed, steal):
    """Phase 1 in virtual time.  Returns (finish time per worker, final
    segment [pl, pr] per worker, the range each worker ends with)."""
    if not steal:
        finish, segs, res = [], [], []
        for s0, s1 in static_bounds(M, workers):
            t, cur = 0.0, (s0, s0 + 1)
            for e in range(s0 + 1, s1):
                cur = apply(cur, (e, e + 1))
                t += op_time(mean, dist, seed, cur[0], cur[1])
            finish.append(t)
            segs.append((s0, s1 - 1))
            res.append(cur)
        return finish, segs, res
    start = [flex_start(M, workers, w) for w in range(workers)]
    gap = [[start[w] + 1, start[w + 1] - 1] for w in range(workers - 1)]   # [lo, hi]
    pl, pr = list(start), list(start)
    cur = [(s, s + 1) for s in start]
    ops = [0] * workers
    busy = [0.0] * workers
    clock = [0.0] * workers
    finished = [False] * workers
    events = [(0.0, w) for w in range(workers)]   # (time, worker): the worker decides its next step
    heapq.heapify(events)

    def size(g):
        return gap[g][1] - gap[g][0] + 1

    def rate(w):
        return busy[w] / ops[w] if ops[w] else 0.0

    while events:
        t, w = heapq.heappop(events)
        sl = size(w - 1) if w > 0 else 0
        sr = size(w) if w < workers - 1 else 0
        if sl <= 0 and sr <= 0:
            finished[w] = True
            clock[w] = t
            continue
        if ops[w] == 0 and sr > 0:
            right = True
        elif sl > 0 and sr > 0:
            right = not (rate(w - 1) > rate(w + 1))
        else:
            right = sl <= 0
        if right:
            e = gap[w][0]
            gap[w][0] += 1
            cur[w] = apply(cur[w], (e, e + 1))
            pr[w] = e
        else:
            e = gap[w - 1][1]
            gap[w - 1][1] -= 1
            cur[w] = apply((e, e + 1), cur[w])
            pl[w] = e
        dt = op_time(mean, dist, seed, cur[w][0], cur[w][1])
        ops[w] += 1
        busy[w] += dt
        heapq.heappush(events, (t + dt, w))
    return clock, list(zip(pl, pr)), cur


def simulate_segments(M, workers, mean, dist, seed, steal, global_algo="lf"):
    """Reduce-then-scan over static or flexible segments, each phase one
    launch (it starts when the previous one has finished): phase 1, the global
    scan of the segment totals (dataflow on `workers` workers), phase 3 (worker
    w >= 1 rescans its segment from the global prefix).  Returns the makespan
    and the phase durations and segments."""
    fin1, segs, res = simulate_phase1(M, workers, mean, dist, seed, steal)
    t1 = max(fin1)
    gops, _ = plans.make_plan(workers, global_algo)
    # the global plan's ranges are in segment numbers; its operator times are
    # those of the frame ranges the segments cover
    lo = [s[0] for s in segs]
    hi = [s[1] + 1 for s in segs]
    g = np.array(gops, dtype=np.int64).reshape(-1, 7).copy()
    if len(g):
        g[:, 4] = [lo[int(i)] for i in gops[:, 4]]
        g[:, 6] = [hi[int(k) - 1] for k in gops[:, 6]]
    t2, _ = simulate_dataflow(workers, g, workers, mean, dist, seed)
    t3 = 0.0
    for w in range(1, workers):
        t = 0.0
        for e in range(segs[w][0], segs[w][1] + 1):
            t += op_time(mean, dist, seed, 0, e + 1)
        t3 = max(t3, t)
    return t1 + t2 + t3, {"phase1": t1, "global": t2, "phase3": t3, "segments": segs, "totals": res}


def valid_segments(segs, M, workers, steal):
    """Segments partition [0, M) in worker order; static ones are the static
    bounds, flexible ones contain their worker's start element."""
    segs = [tuple(int(v) for v in s) for s in segs]
    if segs[0][0] != 0 or segs[-1][1] != M - 1:
        return False
    for w in range(workers - 1):
        if segs[w][1] + 1 != segs[w + 1][0]:
            return False
    for w, (a, b) in enumerate(segs):
        if a > b:
            return False
        if steal:
            if not a <= flex_start(M, workers, w) <= b:
                return False
        elif (a, b + 1) != static_bounds(M, workers)[w]:
            return False
    return True
