"""Prefix-scan plans, CPU oracle.  TEST INFRASTRUCTURE ONLY.

A plan is the list of operator applications (i, j) . (j, k) -> (i, k) that
turns the elements x_k = phi_{k-1,k}, k = 1..M, into the inclusive prefixes
y_k = phi_{0,k} (Section 3: phi_{0,j} = phi_{0,1} . ... . phi_{j-1,j}).

Nodes 0..M-1 are the elements x_1..x_M; node M + n is the output of op n.
Every op carries (level, out, a, b, i, j, k): a and b are its input nodes with
ranges (i, j) and (j, k).  Levels are as-soon-as-possible: 1 + the larger
level of the two inputs, elements at level 0.  Ops are ordered by level, then
by k, i, j, and outputs are numbered in that order.

Algorithms (Section 2.1, Table 1; Section 4.1-4.2):
  seq            left fold, M-1 ops, depth M-1
  dissemination  round d = 1, 2, 4, ...: z_k <- z_{k-d} . z_k for k > d
                 (Fig. "dissemination": 17 ops for 8 elements in 3 rounds)
  lf             Ladner-Fischer P_0 circuit, depth log2 M
  bk             Brent-Kung: up-sweep then down-sweep, depth 2 log2 M - 1
  hier           reduce-then-scan over chunks of S elements (Section 4.1/4.2):
                 each chunk reduces left to right (chunk 0's partial results
                 are already its prefixes), a global scan over the chunk totals
                 with the chosen algorithm, then every later chunk rescans
                 from the previous chunk's global prefix; the last prefix of a
                 chunk is the global result itself and is not recomputed.
For lf and bk with M not a power of two the circuit is built for the next
power of two and every op whose range ends beyond M is dropped.
"""
from __future__ import annotations

import math

import numpy as np

ALGOS = ("seq", "dissemination", "lf", "bk", "hier")
ALGO_ID = {name: n for n, name in enumerate(ALGOS)}

OP_FIELDS = ("level", "out", "a", "b", "i", "j", "k")


class _Builder:
    def __init__(self, n_elems):
        self.rng = [(m, m + 1) for m in range(n_elems)]   # node -> (i, k)
        self.lvl = [0] * n_elems
        self.ops = []                                      # (a, b, provisional out)

    def op(self, a, b):
        ia, ja = self.rng[a]
        jb, kb = self.rng[b]
        assert ja == jb, f"non-adjacent operands {self.rng[a]} . {self.rng[b]}"
        out = len(self.rng)
        self.rng.append((ia, kb))
        self.lvl.append(1 + max(self.lvl[a], self.lvl[b]))
        self.ops.append((a, b, out))
        return out


def _seq(b, nodes):
    out = [nodes[0]]
    for nd in nodes[1:]:
        out.append(b.op(out[-1], nd))
    return out


def _dissemination(b, nodes):
    z = list(nodes)
    d = 1
    while d < len(z):
        z = [z[k] if k < d else b.op(z[k - d], z[k]) for k in range(len(z))]
        d *= 2
    return z


def _lf0(b, nodes):
    n = len(nodes)
    if n == 1:
        return list(nodes)
    half = n // 2
    left = _lf1(b, nodes[:half])
    right = _lf0(b, nodes[half:])
    return left + [b.op(left[-1], r) for r in right]


def _lf1(b, nodes):
    n = len(nodes)
    if n == 1:
        return list(nodes)
    pairs = [b.op(nodes[2 * q], nodes[2 * q + 1]) for q in range(n // 2)]
    inner = _lf0(b, pairs)
    out = [None] * n
    out[0] = nodes[0]
    for q in range(n // 2):
        out[2 * q + 1] = inner[q]
        if q > 0:
            out[2 * q] = b.op(inner[q - 1], nodes[2 * q])
    return out


def _bk(b, nodes):
    z = list(nodes)       # z[p] holds position p + 1
    n = len(z)
    d = 1
    while 2 * d <= n:     # up-sweep
        for p in range(2 * d, n + 1, 2 * d):
            z[p - 1] = b.op(z[p - d - 1], z[p - 1])
        d *= 2
    d //= 2
    while d >= 1:         # down-sweep
        for p in range(3 * d, n + 1, 2 * d):
            z[p - 1] = b.op(z[p - d - 1], z[p - 1])
        d //= 2
    return z


def _pow2_then_drop(fn):
    def run(b, nodes):
        n = len(nodes)
        m = 1 << max(0, math.ceil(math.log2(n))) if n > 1 else 1
        if m == n:
            return fn(b, nodes)
        # virtual elements extend the ranges beyond the real ones
        base = len(b.rng)
        last_k = b.rng[nodes[-1]][1]
        virt = []
        for q in range(m - n):
            b.rng.append((last_k + q, last_k + q + 1))
            b.lvl.append(0)
            virt.append(base + q)
        out = fn(b, list(nodes) + virt)
        return out[:n]
    return run


GLOBAL = {
    "seq": _seq,
    "dissemination": _dissemination,
    "lf": _pow2_then_drop(_lf0),
    "bk": _pow2_then_drop(_bk),
}


def _hier(b, nodes, chunk, global_algo):
    n = len(nodes)
    S = n if chunk <= 0 else min(chunk, n)
    chunks = [nodes[s:s + S] for s in range(0, n, S)]
    # phase 1: left-to-right reduction of every chunk
    prefix0 = _seq(b, chunks[0])
    totals = [prefix0[-1]]
    for ch in chunks[1:]:
        t = ch[0]
        for nd in ch[1:]:
            t = b.op(t, nd)
        totals.append(t)
    # phase 2: global scan over the chunk totals
    G = GLOBAL[global_algo](b, totals)
    # phase 3: rescan every later chunk from the previous global prefix
    out = list(prefix0)
    for c in range(1, len(chunks)):
        ch = chunks[c]
        y = G[c - 1]
        for nd in ch[:-1]:
            y = b.op(y, nd)
            out.append(y)
        out.append(G[c])
    return out


def make_plan(M, algo, chunk=0, global_algo="lf"):
    """Build the plan for M elements.  Returns (ops int64 [n][7], n_levels)."""
    if M < 1:
        raise ValueError("M must be >= 1")
    if algo not in ALGOS:
        raise ValueError(f"unknown algorithm {algo}")
    if algo == "hier" and global_algo not in GLOBAL:
        raise ValueError(f"unknown global algorithm {global_algo}")
    b = _Builder(M)
    nodes = list(range(M))
    if algo == "hier":
        _hier(b, nodes, chunk, global_algo)
    else:
        GLOBAL[algo](b, nodes)
    # drop ops whose range ends beyond M (power-of-two padding)
    keep = [(a, bb, o) for (a, bb, o) in b.ops if b.rng[o][1] <= M]
    # order by (level, k, i, j) and renumber outputs
    def key(t):
        a, bb, o = t
        return (b.lvl[o], b.rng[o][1], b.rng[o][0], b.rng[a][1])
    keep.sort(key=key)
    new_id = {m: m for m in range(M)}
    for n, (_, _, o) in enumerate(keep):
        new_id[o] = M + n
    ops = np.zeros((len(keep), 7), dtype=np.int64)
    for n, (a, bb, o) in enumerate(keep):
        i, k = b.rng[o]
        j = b.rng[a][1]
        ops[n] = (b.lvl[o], new_id[o], new_id[a], new_id[bb], i, j, k)
    n_levels = int(ops[:, 0].max()) if len(ops) else 0
    return ops, n_levels


def final_nodes(ops, M):
    """Node holding phi_{0,k} for k = 1..M (index k-1)."""
    out = np.full(M, -1, dtype=np.int64)
    out[0] = 0
    for row in ops:
        if row[4] == 0:
            k = int(row[6])
            assert out[k - 1] == -1, f"prefix (0,{k}) produced twice"
            out[k - 1] = row[1]
    return out


def check_plan(ops, M):
    """Verify that a plan is a correct inclusive scan; returns the final nodes."""
    rng = {m: (m, m + 1) for m in range(M)}
    lvl = {m: 0 for m in range(M)}
    for row in ops:
        level, out, a, b, i, j, k = (int(v) for v in row)
        assert a in rng and b in rng, "operand used before it is produced"
        assert rng[a] == (i, j) and rng[b] == (j, k), "range bookkeeping mismatch"
        assert level == 1 + max(lvl[a], lvl[b]), "level is not as-soon-as-possible"
        assert out not in rng, "node produced twice"
        rng[out] = (i, k)
        lvl[out] = level
    fin = final_nodes(ops, M)
    for k in range(1, M + 1):
        assert fin[k - 1] >= 0 and rng[int(fin[k - 1])] == (0, k), f"prefix {k} missing"
    return fin


# ----------------------------------------------------------------------------
# Closed-form work and depth (Table 1; Section 4.1, reduce-then-scan)
# ----------------------------------------------------------------------------

def fib(n):
    a, b = 0, 1
    for _ in range(n):
        a, b = b, a + b
    return a


def lf_work(n):
    """Exact Ladner-Fischer P_0 work for n a power of two (recursion of Table 1)."""
    s0 = {1: 0, 2: 1}
    s1 = {1: 0, 2: 1}
    m = 4
    while m <= n:
        s1[m] = s0[m // 2] + m - 1
        s0[m] = s1[m // 2] + s0[m // 2] + m // 2
        m *= 2
    return s0[n]
