// Prefix-scan planner (host only).
//
// Builds the DAG of operator applications (i, j) (.) (j, k) -> (i, k) that
// turns x_1..x_M into the inclusive prefixes (Section 3), for the scan
// algorithms of Table 1 and the hierarchical reduce-then-scan of
// Sections 4.1-4.2, then levels it as-soon-as-possible and orders it by
// (level, k, i, j).  Ladner-Fischer and Brent-Kung circuits (also as the
// global phase of the hierarchical plan) are built for the next power of two;
// ops whose range ends beyond the last real element are dropped.
#include "plan.h"

#include <algorithm>
#include <stdexcept>

namespace rs {

namespace {

struct Builder {
  std::vector<int> lo, hi, lvl;        // per node: range (lo, hi], level
  struct Op { int a, b, out; };
  std::vector<Op> ops;

  explicit Builder(int m) {
    for (int q = 0; q < m; ++q) add_leaf(q, q + 1);
  }
  int add_leaf(int i, int k) {
    lo.push_back(i);
    hi.push_back(k);
    lvl.push_back(0);
    return (int)lo.size() - 1;
  }
  int apply(int a, int b) {
    if (hi[a] != lo[b]) throw std::logic_error("plan: operands are not adjacent");
    const int out = (int)lo.size();
    lo.push_back(lo[a]);
    hi.push_back(hi[b]);
    lvl.push_back(1 + std::max(lvl[a], lvl[b]));
    ops.push_back({a, b, out});
    return out;
  }
};

using Nodes = std::vector<int>;

Nodes fold(Builder& B, const Nodes& x) {
  Nodes y{x[0]};
  for (size_t q = 1; q < x.size(); ++q) y.push_back(B.apply(y.back(), x[q]));
  return y;
}

Nodes dissemination(Builder& B, const Nodes& x) {
  Nodes z = x;
  for (size_t d = 1; d < z.size(); d *= 2) {
    Nodes nz(z.size());
    for (size_t q = 0; q < z.size(); ++q) nz[q] = q < d ? z[q] : B.apply(z[q - d], z[q]);
    z.swap(nz);
  }
  return z;
}

Nodes lf1(Builder& B, const Nodes& x);

// Ladner-Fischer P_0: P_1 on the left half, P_0 on the right half, then the
// last left prefix is applied to every right output.
Nodes lf0(Builder& B, const Nodes& x) {
  const size_t n = x.size();
  if (n == 1) return x;
  const Nodes left = lf1(B, Nodes(x.begin(), x.begin() + n / 2));
  const Nodes right = lf0(B, Nodes(x.begin() + n / 2, x.end()));
  Nodes y = left;
  for (int r : right) y.push_back(B.apply(left.back(), r));
  return y;
}

// Ladner-Fischer P_1: combine neighbouring pairs, P_0 over the pair results,
// then fill the even positions from the preceding pair prefix.
Nodes lf1(Builder& B, const Nodes& x) {
  const size_t n = x.size();
  if (n == 1) return x;
  Nodes pairs;
  for (size_t q = 0; q < n / 2; ++q) pairs.push_back(B.apply(x[2 * q], x[2 * q + 1]));
  const Nodes inner = lf0(B, pairs);
  Nodes y(n);
  y[0] = x[0];
  for (size_t q = 0; q < n / 2; ++q) {
    y[2 * q + 1] = inner[q];
    if (q > 0) y[2 * q] = B.apply(inner[q - 1], x[2 * q]);
  }
  return y;
}

Nodes brent_kung(Builder& B, const Nodes& x) {
  Nodes z = x;   // z[p - 1] covers up to position p
  const size_t n = z.size();
  size_t d = 1;
  for (; 2 * d <= n; d *= 2)
    for (size_t p = 2 * d; p <= n; p += 2 * d) z[p - 1] = B.apply(z[p - d - 1], z[p - 1]);
  for (d /= 2; d >= 1; d /= 2)
    for (size_t p = 3 * d; p <= n; p += 2 * d) z[p - 1] = B.apply(z[p - d - 1], z[p - 1]);
  return z;
}

Nodes padded(Builder& B, const Nodes& x, Nodes (*circuit)(Builder&, const Nodes&)) {
  size_t m = 1;
  while (m < x.size()) m *= 2;
  if (m == x.size()) return circuit(B, x);
  Nodes ext = x;
  const int last = B.hi[x.back()];
  for (size_t q = 0; q < m - x.size(); ++q) ext.push_back(B.add_leaf(last + (int)q, last + (int)q + 1));
  Nodes y = circuit(B, ext);
  y.resize(x.size());
  return y;
}

Nodes global_scan(Builder& B, const Nodes& x, int algo) {
  switch (algo) {
    case 0: return fold(B, x);
    case 1: return dissemination(B, x);
    case 2: return padded(B, x, lf0);
    case 3: return padded(B, x, brent_kung);
    default: throw std::invalid_argument("plan: unknown algorithm");
  }
}

void hierarchical(Builder& B, const Nodes& x, int chunk, int global_algo) {
  const size_t n = x.size();
  const size_t S = (chunk <= 0 || (size_t)chunk >= n) ? n : (size_t)chunk;
  std::vector<Nodes> chunks;
  for (size_t s = 0; s < n; s += S) chunks.emplace_back(x.begin() + s, x.begin() + std::min(n, s + S));
  // local phase: reduce every chunk left to right (chunk 0 yields prefixes)
  const Nodes prefix0 = fold(B, chunks[0]);
  Nodes totals{prefix0.back()};
  for (size_t c = 1; c < chunks.size(); ++c) {
    int t = chunks[c][0];
    for (size_t q = 1; q < chunks[c].size(); ++q) t = B.apply(t, chunks[c][q]);
    totals.push_back(t);
  }
  // global phase over the chunk totals
  const Nodes G = global_scan(B, totals, global_algo);
  // second local phase: rescan every later chunk from the previous prefix
  for (size_t c = 1; c < chunks.size(); ++c) {
    int y = G[c - 1];
    for (size_t q = 0; q + 1 < chunks[c].size(); ++q) y = B.apply(y, chunks[c][q]);
  }
}

}  // namespace

int build_plan(int M, int algo, int chunk, int global_algo, std::vector<PlanOp>& out, int& n_levels) {
  out.clear();
  n_levels = 0;
  if (M < 1 || algo < 0 || algo > 4) return -1;
  if (algo == 4 && (global_algo < 0 || global_algo > 3)) return -1;
  Builder B(M);
  Nodes x(M);
  for (int q = 0; q < M; ++q) x[q] = q;
  if (algo == 4)
    hierarchical(B, x, chunk, global_algo);
  else
    global_scan(B, x, algo);

  std::vector<Builder::Op> keep;
  for (const auto& op : B.ops)
    if (B.hi[op.out] <= M) keep.push_back(op);
  std::stable_sort(keep.begin(), keep.end(), [&](const Builder::Op& p, const Builder::Op& q) {
    if (B.lvl[p.out] != B.lvl[q.out]) return B.lvl[p.out] < B.lvl[q.out];
    if (B.hi[p.out] != B.hi[q.out]) return B.hi[p.out] < B.hi[q.out];
    if (B.lo[p.out] != B.lo[q.out]) return B.lo[p.out] < B.lo[q.out];
    return B.hi[p.a] < B.hi[q.a];
  });
  std::vector<int> id(B.lo.size(), -1);
  for (int q = 0; q < M; ++q) id[q] = q;
  for (size_t n = 0; n < keep.size(); ++n) id[keep[n].out] = M + (int)n;
  for (const auto& op : keep) {
    PlanOp p;
    p.level = B.lvl[op.out];
    p.out = id[op.out];
    p.a = id[op.a];
    p.b = id[op.b];
    p.i = B.lo[op.out];
    p.j = B.hi[op.a];
    p.k = B.hi[op.out];
    out.push_back(p);
    n_levels = std::max(n_levels, p.level);
  }
  return 0;
}

}  // namespace rs
