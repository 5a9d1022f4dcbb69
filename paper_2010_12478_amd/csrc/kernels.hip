// Standalone kernels (double arithmetic, float or double storage): pyramid restriction / prolongation, composition, warp
// and its adjoint, energy + gradient, and the backward pass of the
// differentiable warp + energy step.
#include "internal.h"
#include "sweep.h"

namespace rs {

namespace {

constexpr int kEW = 256;   // threads per block of the elementwise kernels

inline int ew_blocks(size_t n) {
  size_t b = (n + kEW - 1) / kEW;
  return (int)(b < 65535u * 16u ? b : 65535u * 16u);
}

// out[b][Y][X] = scale * (1/4) * sum of the 2x2 block of in[b]
template <typename S>
__global__ void __launch_bounds__(kEW) k_restrict(const S* __restrict__ in, S* __restrict__ out, double scale,
                                                  int B, int H, int W) {
  const int h = H >> 1, w = W >> 1;
  const size_t n = (size_t)B * h * w;
  for (size_t t = blockIdx.x * (size_t)kEW + threadIdx.x; t < n; t += (size_t)gridDim.x * kEW) {
    const size_t b = t / ((size_t)h * w);
    const int r = (int)(t - b * h * w);
    const int Y = r / w, X = r - Y * w;
    const S* p = in + b * H * W + (size_t)(2 * Y) * W + 2 * X;
    const double sum = (((double)p[0] + (double)p[1]) + (double)p[W]) + (double)p[W + 1];
    out[t] = (S)(scale * (0.25 * sum));
  }
}

// Per-axis weights of the frame restriction: the binomial coefficients of
// (1 + z)^5 over 32 (exact binary fractions; a product with a float32 tap is
// exact in float64).
constexpr double kBinom6[6] = {1.0 / 32, 5.0 / 32, 10.0 / 32, 10.0 / 32, 5.0 / 32, 1.0 / 32};

// Coarse pixel (Y, X) of the frame restriction of an h2 x w2 level `src`
// (row pitch sp): the separable order-5 binomial low-pass centred on the
// 2x2 block (2Y + 1/2, 2X + 1/2),
//   sum_{a=0..5} w_a (sum_{b=0..5} w_b src[clamp(2Y+a-2)][clamp(2X+b-2)]),
// each row's sum in increasing b, then the weighted rows in increasing a,
// one rounded float64 operation each (no contraction).  It removes the
// lattice content a coarser grid cannot represent (an atom lattice of two
// coarse pixels per period or less would otherwise come through aliased or
// sign-ambiguous) instead of passing 71% of it like the 2x2 block mean.
template <typename S>
__device__ __forceinline__ double binom6_pixel(const S* __restrict__ src, int sp, int h2, int w2, int Y, int X) {
#pragma clang fp contract(off)
  int xo[6];
#pragma unroll
  for (int b = 0; b < 6; ++b) xo[b] = clampi(2 * X + b - 2, 0, w2 - 1);
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const S* r = src + (size_t)clampi(2 * Y + a - 2, 0, h2 - 1) * sp;
    double row = kBinom6[0] * (double)r[xo[0]];
#pragma unroll
    for (int b = 1; b < 6; ++b) row = row + kBinom6[b] * (double)r[xo[b]];
    acc = a == 0 ? kBinom6[0] * row : acc + kBinom6[a] * row;
  }
  return acc;
}

// out[b] = frame restriction of in[b] (H x W -> H/2 x W/2)
template <typename S>
__global__ void __launch_bounds__(kEW) k_restrict_frame(const S* __restrict__ in, S* __restrict__ out, int B,
                                                        int H, int W) {
  const int h = H >> 1, w = W >> 1;
  const size_t n = (size_t)B * h * w;
  for (size_t t = blockIdx.x * (size_t)kEW + threadIdx.x; t < n; t += (size_t)gridDim.x * kEW) {
    const size_t b = t / ((size_t)h * w);
    const int r = (int)(t - b * h * w);
    const int Y = r / w, X = r - Y * w;
    out[t] = (S)binom6_pixel(in + b * H * W, W, H, W, Y, X);
  }
}

// Weights with which fine row y (of n2 = 2 n) enters coarse rows Y0 .. Y0 + 3
// of the frame restriction: w[i] = sum of kBinom6[a] over the taps a of
// coarse row Y0 + i whose clamped index is y (zero past the last row).
__device__ __forceinline__ int binom6_adjoint_rows(int y, int n2, double w[4]) {
  const int n = n2 >> 1;
  const int Y0 = max((y - 3) >> 1, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int Y = Y0 + i;
    double s = 0.0;
    if (Y < n) {
#pragma unroll
      for (int a = 0; a < 6; ++a)
        if (clampi(2 * Y + a - 2, 0, n2 - 1) == y) s += kBinom6[a];
    }
    w[i] = s;
  }
  return Y0;
}

// dF[b] = transpose of the frame restriction applied to dC[b]
// (H/2 x W/2 -> H x W), gathered per fine pixel; dC == nullptr: zeros.
template <typename S>
__global__ void __launch_bounds__(kEW) k_restrict_frame_adjoint(const S* __restrict__ dC, S* __restrict__ dF,
                                                                int B, int H, int W) {
  const int h = H >> 1, w = W >> 1;
  const size_t HW = (size_t)H * W, n = (size_t)B * HW;
  for (size_t t = blockIdx.x * (size_t)kEW + threadIdx.x; t < n; t += (size_t)gridDim.x * kEW) {
    const size_t b = t / HW;
    if (!dC) {
      dF[t] = S(0);
      continue;
    }
    const int r = (int)(t - b * HW);
    const int y = r / W, x = r - y * W;
    double wy[4], wx[4];
    const int Y0 = binom6_adjoint_rows(y, H, wy);
    const int X0 = binom6_adjoint_rows(x, W, wx);
    const S* c = dC + b * (size_t)h * w;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (wy[i] == 0.0) continue;
      double row = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (wx[j] != 0.0) row += wx[j] * (double)c[(size_t)(Y0 + i) * w + X0 + j];
      acc += wy[i] * row;
    }
    dF[t] = (S)acc;
  }
}

// Padded pyramid level: element (Y, X), Y in [-1, h], X in [-1, w], of frame
// f holds pixel (clamp(Y), clamp(X)) of the level: a copy of the frame
// (COPY) or the frame restriction (binom6_pixel) of the level below.
template <bool COPY>
__global__ void __launch_bounds__(kEW) k_pad_level(const float* __restrict__ src, int sp, size_t sfs,
                                                   float* __restrict__ dst, int pitch, int N, int h, int w) {
  const int hp = h + 2, wp = w + 2;
  const size_t n = (size_t)N * hp * wp;
  const size_t fstride = (size_t)hp * pitch;
  for (size_t t = blockIdx.x * (size_t)kEW + threadIdx.x; t < n; t += (size_t)gridDim.x * kEW) {
    const size_t f = t / ((size_t)hp * wp);
    const int r = (int)(t - f * hp * wp);
    const int Y = r / wp - 1, X = r - (Y + 1) * wp - 1;
    const int yc = clampi(Y, 0, h - 1), xc = clampi(X, 0, w - 1);
    float v;
    if (COPY)
      v = src[f * h * w + (size_t)yc * w + xc];
    else
      v = (float)binom6_pixel(src + f * sfs, sp, 2 * h, 2 * w, yc, xc);
    dst[f * fstride + (size_t)(Y + 1) * pitch + kPadLeft + X] = v;
  }
}

__global__ void __launch_bounds__(kEW) k_prolong(const float* __restrict__ uc, float* __restrict__ uf,
                                                 int B, int Hf, int Wf) {
  const int hc = Hf >> 1, wc = Wf >> 1;
  const size_t n = (size_t)B * Hf * Wf;
  for (size_t t = blockIdx.x * (size_t)kEW + threadIdx.x; t < n; t += (size_t)gridDim.x * kEW) {
    const size_t b = t / ((size_t)Hf * Wf);
    const int r = (int)(t - b * Hf * Wf);
    const int y = r / Wf, x = r - y * Wf;
    double vx, vy;
    prolong_pixel<false>(uc + b * 2 * hc * wc, hc, wc, x, y, vx, vy);   // base varies per lane
    float* o = uf + b * 2 * Hf * Wf;
    o[r] = (float)vx;
    o[(size_t)Hf * Wf + r] = (float)vy;
  }
}

__global__ void __launch_bounds__(kEW) k_compose(const float* __restrict__ uij, const float* __restrict__ ujk,
                                                 float* __restrict__ out, int B, int H, int W) {
  const size_t HW = (size_t)H * W, n = (size_t)B * HW;
  for (size_t t = blockIdx.x * (size_t)kEW + threadIdx.x; t < n; t += (size_t)gridDim.x * kEW) {
    const size_t b = t / HW;
    const int r = (int)(t - b * HW);
    const int y = r / W, x = r - y * W;
    double vx, vy;
    init_pixel<float>(1, uij + b * 2 * HW, ujk + b * 2 * HW, H, W, 1, x, y, vx, vy);
    out[b * 2 * HW + r] = (float)vx;
    out[b * 2 * HW + HW + r] = (float)vy;
  }
}

// Rows of the batch (index b * H + y) are spread over blockIdx.y in groups of
// kWarpRows (grid-strided), columns over blockIdx.x and the threads: no
// per-pixel division, and each thread keeps kWarpRows independent
// load-gather-store chains in flight.
constexpr int kWarpRows = 4;

template <typename S>
__global__ void __launch_bounds__(kEW) k_warp(const S* __restrict__ T, const S* __restrict__ u,
                                              S* __restrict__ out, int B, int H, int W) {
  const size_t HW = (size_t)H * W;
  const int x = blockIdx.x * kEW + threadIdx.x;
  if (x >= W) return;
  const int n_rows = B * H;
  for (int row0 = blockIdx.y * kWarpRows; row0 < n_rows; row0 += gridDim.y * kWarpRows) {
    // the group's rows as (batch item, row), wave-uniform; a short last
    // group repeats its last row for the loads
    int bk[kWarpRows], yk[kWarpRows];
    {
      int b = row0 / H, y = row0 - b * H;
#pragma unroll
      for (int k = 0; k < kWarpRows; ++k) {
        bk[k] = b;
        yk[k] = y;
        if (row0 + k + 1 < n_rows && ++y == H) y = 0, ++b;
      }
    }
    S ux[kWarpRows], uy[kWarpRows];
#pragma unroll
    for (int k = 0; k < kWarpRows; ++k) {
      const BufView<0> ub(u + (size_t)bk[k] * 2 * HW);
      const int o = yk[k] * W + x;
      ux[k] = ub.load<S>(o);
      uy[k] = ub.load<S>((int)HW + o);
    }
#pragma unroll
    for (int k = 0; k < kWarpRows; ++k) {
      if (row0 + k >= n_rows) break;
      const BufView<0> tb(T + (size_t)bk[k] * HW);
      int ix, iy;
      double fx, fy;
      cell_of(ux[k], ix, fx);
      cell_of(uy[k], iy, fy);
      const int x0 = x + ix, y0 = yk[k] + iy;
      const int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
      const int ya = clampi(y0, 0, H - 1) * W, yb = clampi(y0 + 1, 0, H - 1) * W;
      out[(size_t)bk[k] * HW + (size_t)yk[k] * W + x] =
          (S)bilin_taps(tb.load<S>(ya + xa), tb.load<S>(ya + xb), tb.load<S>(yb + xa), tb.load<S>(yb + xb), fx, fy);
    }
  }
}

__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// Scatters of the adjoint kernels.  A thread takes a group of consecutive
// rows of one column (kWarpAdjRows for the warp's adjoint, kBackRows for
// the energy's backward pass); the bilinear shares of a pixel go to two
// upper taps (row ya) and two lower taps (row yb).  Shares that land on one
// cell are added in registers before the single atomic addition that
// carries them:
//  - rows: the lower taps of row y are held back and joined to the upper
//    taps of row y + 1 when those are the same two cells (the common case of
//    a smooth field); otherwise they are added to the destination;
//  - columns: a lane adds its left neighbour's right share into its own left
//    share when both are the same cell, and the neighbour then leaves it out.
// On smooth fields that leaves about one full-wavefront atomic per row of
// pixels instead of four.  The order of the additions is not fixed (as with
// any atomic sum).
// measured best of 4, 8, 16 rows (adjoint) and of 2, 4, 8 (backward)
constexpr int kWarpAdjRows = 16, kBackRows = 8;

template <typename S>
struct TapPair {   // two horizontally adjacent taps of one row; y < 0: none
  int y, xa, xb;
  S va, vb;
};

template <typename S>
__device__ __forceinline__ TapPair<S> no_taps() {
  TapPair<S> t;
  t.y = t.xa = t.xb = -1;
  t.va = t.vb = S(0);
  return t;
}

// Adds every lane's pair to dst (row pitch W).  Called by all lanes of the
// wavefront together (the column join reads the neighbours' registers).
template <typename S>
__device__ __forceinline__ void emit_taps(S* __restrict__ dst, int W, TapPair<S> t) {
  const int ly = wave_shift<0x138>(t.y, -1), lxb = wave_shift<0x138>(t.xb, -1);
  const S lvb = wave_from_left(t.vb, S(0));
  const bool take = t.y >= 0 && ly == t.y && lxb == t.xa;
  if (take) t.va += lvb;
  const int given = wave_shift<0x130>((int)take, 0);
  if (t.y >= 0) {
    atomic_add(dst + t.y * W + t.xa, t.va);
    if (!given) atomic_add(dst + t.y * W + t.xb, t.vb);
  }
}

// The row-by-row scatter of one thread's column (see above).
template <typename S>
struct RowScatter {
  TapPair<S> low = no_taps<S>();   // lower taps held back from the previous row

  // v(x, y) into the four clamped taps of (x, y) + (ux, uy) with bilinear
  // weights; a lane without a pixel (valid false) still takes part
  __device__ __forceinline__ void pixel(S* __restrict__ dst, int H, int W, bool valid, int x, int y, S ux, S uy,
                                        double v) {
    TapPair<S> up = no_taps<S>(), lo = no_taps<S>();
    if (valid) {
      int ix, iy;
      double fx, fy;
      cell_of(ux, ix, fx);
      cell_of(uy, iy, fy);
      const int xa = clampi(x + ix, 0, W - 1), xb = clampi(x + ix + 1, 0, W - 1);
      const double ox = 1.0 - fx, oy = 1.0 - fy;
      up.y = clampi(y + iy, 0, H - 1);
      lo.y = clampi(y + iy + 1, 0, H - 1);
      up.xa = lo.xa = xa;
      up.xb = lo.xb = xb;
      up.va = (S)(v * ox * oy);
      up.vb = (S)(v * fx * oy);
      lo.va = (S)(v * ox * fy);
      lo.vb = (S)(v * fx * fy);
    }
    const bool join = low.y >= 0 && up.y == low.y && up.xa == low.xa && up.xb == low.xb;
    if (join) {
      up.va += low.va;
      up.vb += low.vb;
    }
    emit_taps(dst, W, join ? no_taps<S>() : low);
    emit_taps(dst, W, up);
    low = lo;
  }
  __device__ __forceinline__ void finish(S* __restrict__ dst, int W) {
    emit_taps(dst, W, low);
    low = no_taps<S>();
  }
};

// Grid of the adjoint kernels: column blocks x (item, group of `rows` rows),
// at most 65535 groups (grid-strided beyond).
inline dim3 adjoint_grid(int B, int H, int W, int rows) {
  const long long groups = (long long)B * ((H + rows - 1) / rows);
  return dim3((unsigned)((W + kEW - 1) / kEW), (unsigned)(groups < 65535 ? groups : 65535));
}

// gT[b] += adjoint of the warp of item b applied to g[b] (grid: adjoint_grid)
template <typename S>
__global__ void __launch_bounds__(kEW) k_warp_adjoint(const S* __restrict__ g, const S* __restrict__ u,
                                                      S* __restrict__ gT, int B, int H, int W) {
  const size_t HW = (size_t)H * W;
  const int x = blockIdx.x * kEW + threadIdx.x;
  const bool col = x < W;
  const int xl = col ? x : W - 1;   // loads of lanes past the last column: any pixel
  const int gpi = (H + kWarpAdjRows - 1) / kWarpAdjRows;
  for (long long t = blockIdx.y; t < (long long)B * gpi; t += gridDim.y) {   // wave-uniform
    const int b = (int)(t / gpi), y0 = (int)(t - (long long)b * gpi) * kWarpAdjRows;
    const S* ub = u + (size_t)b * 2 * HW;
    const S* gb = g + (size_t)b * HW;
    S vx[kWarpAdjRows], vy[kWarpAdjRows], vg[kWarpAdjRows];
#pragma unroll
    for (int k = 0; k < kWarpAdjRows; ++k) {
      const int r = min(y0 + k, H - 1) * W + xl;
      vx[k] = ub[r];
      vy[k] = ub[HW + r];
      vg[k] = gb[r];
    }
    RowScatter<S> sc;
    S* tb = gT + (size_t)b * HW;
#pragma unroll
    for (int k = 0; k < kWarpAdjRows; ++k)
      sc.pixel(tb, H, W, col && y0 + k < H, x, y0 + k, vx[k], vy[k], (double)vg[k]);
    sc.finish(tb, W);
  }
}

// Energy (+ gradient) of one tile of one batch item (grid: tiles x items, in
// XCD-aware order: the tiles of a row of tiles meet in one L2, which serves
// the halo columns and gather lines they share).
template <typename S, int WRITE, bool GNORM>
__global__ void __launch_bounds__(kWG) k_energy_tiles(const S* __restrict__ R, const S* __restrict__ T,
                                                      const S* __restrict__ u, double lam, S* grad,
                                                      double* part, double* gpart, int H, int W, int th) {
  __shared__ double red[sweep_red_doubles<true>(1)];
  const size_t HW = (size_t)H * W;
  const int nt = tiles_of(H, W, th);
  const int item = xcd_item(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y, tiles_x(W));
  const int b = item / nt, tile = item - b * nt;
  LevelView<S> L;
  L.R = R + b * HW;
  L.T = T + b * HW;
  L.u = u + b * 2 * HW;
  L.out = grad ? grad + b * 2 * HW : nullptr;
  L.h = H;
  L.w = W;
  L.pitch = W;
  L.tau = 0.0;
  L.lam = lam;
  // four rows per register batch here (measured 11% faster than two, and
  // faster than six or eight, which leave fewer waves per SIMD), two inside
  // the persistent solver's instantiation with resident levels
  sweep_tiles<S, WRITE, GNORM, false, 4>(L, tile, nt, th, red, part + (size_t)b * nt, gpart + (size_t)b * nt);
}

__global__ void __launch_bounds__(kWave) k_sum_tiles(const double* part, const double* gpart, int nt,
                                                     double* E, double* gn) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const double e = wave_sum_array(part + (size_t)b * nt, nt, lane);
  if (lane == 0) E[b] = e;
  if (gn) {
    const double g = wave_sum_array(gpart + (size_t)b * nt, nt, lane);
    if (lane == 0) gn[b] = g;
  }
}

// One level of the backward pass.  Per pixel x of item b:
//   r = Ia(x + u(x)) - Ib(x), g = dE_l/du(x)
//   du(x)  = gE g(x)     + 1/8 du_c(parent)     (adjoint of half the block mean)
//   dIb(x) = -2 r gE     (+ dIb(x) if carry: it holds the adjoint of the
//                          frame restriction applied to the coarser dIb)
//   dIa   += 2 r gE * bilinear weights at the taps (dIa pre-initialised)
template <typename S>
__global__ void __launch_bounds__(kEW) k_energy_backward(const S* __restrict__ Ia, const S* __restrict__ u,
                                                         const S* __restrict__ Ib, double lam,
                                                         const double* __restrict__ gE, S* dIa, S* du,
                                                         S* dIb, const S* du_c, bool carry,
                                                         int B, int H, int W) {
  const size_t HW = (size_t)H * W;
  const int hc = H >> 1, wc = W >> 1;
  const size_t HWc = (size_t)hc * wc;
  const int x = blockIdx.x * kEW + threadIdx.x;
  const bool col = x < W;
  const int gpi = (H + kBackRows - 1) / kBackRows;
  for (long long t = blockIdx.y; t < (long long)B * gpi; t += gridDim.y) {   // wave-uniform
    const int b = (int)(t / gpi), y0 = (int)(t - (long long)b * gpi) * kBackRows;
    const S* ux = u + (size_t)b * 2 * HW;
    const S* uy = ux + HW;
    const double w = gE[b];
    // u on the rows y0 - 1 .. y0 + kBackRows (clamped to the image; lanes
    // past the last column read column W - 1): the rows above and below a
    // pixel come from these registers, the columns left and right from the
    // neighbouring lanes, and lanes 0 and 63 load the columns beyond the
    // wavefront's 64
    const int lane = threadIdx.x & (kWave - 1);
    const int xl = col ? x : W - 1;
    S cu[kBackRows + 2], cv[kBackRows + 2], eu[kBackRows], ev[kBackRows];
#pragma unroll
    for (int k = 0; k < kBackRows + 2; ++k) {
      const int r = clampi(y0 - 1 + k, 0, H - 1) * W + xl;
      cu[k] = ux[r];
      cv[k] = uy[r];
    }
    const int xe = lane == 0 ? x - 1 : x + 1;   // lane 0: the column left of it, lane 63: right
    const bool edge = col && (lane == 0 || lane == kWave - 1) && xe >= 0 && xe < W;
#pragma unroll
    for (int k = 0; k < kBackRows; ++k) {
      const int r = min(y0 + k, H - 1) * W + xe;
      eu[k] = edge ? ux[r] : S(0);
      ev[k] = edge ? uy[r] : S(0);
    }
    // the rows' outputs du and dIb first (their loads free to overlap: the
    // inputs are restrict), the scatters of dIa after them
    S sx[kBackRows], sy[kBackRows];
    double sv[kBackRows];
#pragma unroll
    for (int k = 0; k < kBackRows; ++k) {
      sx[k] = sy[k] = S(0);
      sv[k] = 0.0;
      const S cxs = cu[k + 1], cys = cv[k + 1];
      // all lanes take part in the lane shifts
      const S lxs = wave_from_left(cxs, eu[k]), lys = wave_from_left(cys, ev[k]);
      const S rxs = wave_from_right(cxs, eu[k]), rys = wave_from_right(cys, ev[k]);
      const int y = y0 + k;
      if (!col || y >= H) continue;
      const int r = y * W + x;
      const size_t q = (size_t)b * HW + r;
      int ix, iy;
      double fx, fy;
      cell_of(cxs, ix, fx);
      cell_of(cys, iy, fy);
      double s, dsx, dsy;
      bilin(Ia + (size_t)b * HW, H, W, x + ix, y + iy, fx, fy, s, dsx, dsy);
      const double res = s - (double)Ib[q];
      const double cx = cxs, cy = cys;
      double nbx = 0.0, nby = 0.0;
      if (x > 0) { nbx += cx - (double)lxs; nby += cy - (double)lys; }
      if (x + 1 < W) { nbx += cx - (double)rxs; nby += cy - (double)rys; }
      if (y > 0) { nbx += cx - (double)cu[k]; nby += cy - (double)cv[k]; }
      if (y + 1 < H) { nbx += cx - (double)cu[k + 2]; nby += cy - (double)cv[k + 2]; }
      double gx = w * (2.0 * res * dsx + 2.0 * lam * nbx);
      double gy = w * (2.0 * res * dsy + 2.0 * lam * nby);
      double gb = w * (-2.0 * res);
      if (du_c) {
        const size_t pc = (size_t)b * 2 * HWc + (size_t)(y >> 1) * wc + (x >> 1);
        gx += 0.125 * (double)du_c[pc];
        gy += 0.125 * (double)du_c[pc + HWc];
      }
      if (carry) gb += (double)dIb[q];
      du[(size_t)b * 2 * HW + r] = (S)gx;
      du[(size_t)b * 2 * HW + HW + r] = (S)gy;
      dIb[q] = (S)gb;
      sx[k] = cxs;
      sy[k] = cys;
      sv[k] = w * 2.0 * res;
    }
    RowScatter<S> sc;
    S* db = dIa + (size_t)b * HW;
#pragma unroll
    for (int k = 0; k < kBackRows; ++k) sc.pixel(db, H, W, col && y0 + k < H, x, y0 + k, sx[k], sy[k], sv[k]);
    sc.finish(db, W);
  }
}

// Autotuner input: a square lattice of period 8 px (sum of two cosines per
// axis), frame f shifted by (0.37 f, -0.29 f) px.
__global__ void __launch_bounds__(kEW) k_synth_frames(float* out, int F, int H, int W) {
  const size_t n = (size_t)F * H * W;
  for (size_t t = blockIdx.x * (size_t)kEW + threadIdx.x; t < n; t += (size_t)gridDim.x * kEW) {
    const size_t f = t / ((size_t)H * W);
    const int r = (int)(t - f * H * W);
    const int y = r / W, x = r - y * W;
    const double px = x - 0.37 * (double)f, py = y + 0.29 * (double)f;
    const double k = 6.283185307179586 / 8.0;
    out[t] = (float)(0.25 * (1.0 + cos(k * px)) * (1.0 + cos(k * py)));
  }
}

__global__ void k_add_energy(const double* Ein, double* Eacc, int B, int first) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) Eacc[b] = first ? Ein[b] : Eacc[b] + Ein[b];
}

}  // namespace

hipError_t launch_restrict(const void* in, void* out, double scale, int B, int H, int W, bool f64,
                           hipStream_t s) {
  const size_t n = (size_t)B * (H / 2) * (W / 2);
  if (n == 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_restrict<double>, dim3(ew_blocks(n)), dim3(kEW), 0, s, (const double*)in,
                       (double*)out, scale, B, H, W);
  else
    hipLaunchKernelGGL(k_restrict<float>, dim3(ew_blocks(n)), dim3(kEW), 0, s, (const float*)in,
                       (float*)out, scale, B, H, W);
  return hipGetLastError();
}

hipError_t launch_restrict_frame(const void* in, void* out, int B, int H, int W, bool f64, hipStream_t s) {
  const size_t n = (size_t)B * (H / 2) * (W / 2);
  if (n == 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_restrict_frame<double>, dim3(ew_blocks(n)), dim3(kEW), 0, s, (const double*)in,
                       (double*)out, B, H, W);
  else
    hipLaunchKernelGGL(k_restrict_frame<float>, dim3(ew_blocks(n)), dim3(kEW), 0, s, (const float*)in,
                       (float*)out, B, H, W);
  return hipGetLastError();
}

hipError_t launch_restrict_frame_adjoint(const void* dC, void* dF, int B, int H, int W, bool f64, hipStream_t s) {
  const size_t n = (size_t)B * H * W;
  if (n == 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_restrict_frame_adjoint<double>, dim3(ew_blocks(n)), dim3(kEW), 0, s, (const double*)dC,
                       (double*)dF, B, H, W);
  else
    hipLaunchKernelGGL(k_restrict_frame_adjoint<float>, dim3(ew_blocks(n)), dim3(kEW), 0, s, (const float*)dC,
                       (float*)dF, B, H, W);
  return hipGetLastError();
}

hipError_t launch_pad_level(const float* src, int sp, size_t sfs, bool copy, float* dst, int pitch, int N, int h,
                            int w, hipStream_t s) {
  const size_t n = (size_t)N * (h + 2) * (w + 2);
  if (n == 0) return hipSuccess;
  if (copy)
    hipLaunchKernelGGL(k_pad_level<true>, dim3(ew_blocks(n)), dim3(kEW), 0, s, src, sp, sfs, dst, pitch, N, h, w);
  else
    hipLaunchKernelGGL(k_pad_level<false>, dim3(ew_blocks(n)), dim3(kEW), 0, s, src, sp, sfs, dst, pitch, N, h, w);
  return hipGetLastError();
}

hipError_t launch_prolong(const float* uc, float* uf, int B, int Hf, int Wf, hipStream_t s) {
  const size_t n = (size_t)B * Hf * Wf;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prolong, dim3(ew_blocks(n)), dim3(kEW), 0, s, uc, uf, B, Hf, Wf);
  return hipGetLastError();
}

hipError_t launch_compose(const float* uij, const float* ujk, float* out, int B, int H, int W, hipStream_t s) {
  const size_t n = (size_t)B * H * W;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compose, dim3(ew_blocks(n)), dim3(kEW), 0, s, uij, ujk, out, B, H, W);
  return hipGetLastError();
}

// Grid of the row-wise elementwise kernels: column blocks x row groups (at
// most 65535, grid-strided beyond).
inline dim3 row_grid(int B, int H, int W, int rows_per_block = 1) {
  const long long rows = ((long long)B * H + rows_per_block - 1) / rows_per_block;
  return dim3((unsigned)((W + kEW - 1) / kEW), (unsigned)(rows < 65535 ? rows : 65535));
}

hipError_t launch_warp(const void* T, const void* u, void* out, int B, int H, int W, bool f64, hipStream_t s) {
  if ((size_t)B * H * W == 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_warp<double>, row_grid(B, H, W, kWarpRows), dim3(kEW), 0, s, (const double*)T,
                       (const double*)u, (double*)out, B, H, W);
  else
    hipLaunchKernelGGL(k_warp<float>, row_grid(B, H, W, kWarpRows), dim3(kEW), 0, s, (const float*)T,
                       (const float*)u, (float*)out, B, H, W);
  return hipGetLastError();
}

hipError_t launch_warp_adjoint(const void* g, const void* u, void* gT, int B, int H, int W, bool f64,
                               hipStream_t s) {
  if ((size_t)B * H * W == 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_warp_adjoint<double>, adjoint_grid(B, H, W, kWarpAdjRows), dim3(kEW), 0, s, (const double*)g,
                       (const double*)u, (double*)gT, B, H, W);
  else
    hipLaunchKernelGGL(k_warp_adjoint<float>, adjoint_grid(B, H, W, kWarpAdjRows), dim3(kEW), 0, s, (const float*)g,
                       (const float*)u, (float*)gT, B, H, W);
  return hipGetLastError();
}

template <typename S>
static void energy_dispatch(const S* R, const S* T, const S* u, double lam, S* grad, double* part, double* gpart,
                            bool gnorm, int B, int H, int W, int th, hipStream_t s) {
  const dim3 grid(tiles_of(H, W, th), B);
  if (grad && gnorm)
    hipLaunchKernelGGL((k_energy_tiles<S, SW_GRAD, true>), grid, dim3(kWG), 0, s, R, T, u, lam, grad, part,
                       gpart, H, W, th);
  else if (grad)
    hipLaunchKernelGGL((k_energy_tiles<S, SW_GRAD, false>), grid, dim3(kWG), 0, s, R, T, u, lam, grad, part,
                       gpart, H, W, th);
  else if (gnorm)
    hipLaunchKernelGGL((k_energy_tiles<S, SW_NONE, true>), grid, dim3(kWG), 0, s, R, T, u, lam, grad, part,
                       gpart, H, W, th);
  else
    hipLaunchKernelGGL((k_energy_tiles<S, SW_NONE, false>), grid, dim3(kWG), 0, s, R, T, u, lam, grad, part,
                       gpart, H, W, th);
}

hipError_t launch_energy_grad(const void* R, const void* T, const void* u, double lam, double* E, void* grad,
                              double* gnorm2, int B, int H, int W, int th, double* part, bool f64,
                              hipStream_t s) {
  if (B == 0) return hipSuccess;
  const int nt = tiles_of(H, W, th);
  double* gpart = part + (size_t)B * nt;
  if (f64)
    energy_dispatch<double>((const double*)R, (const double*)T, (const double*)u, lam, (double*)grad, part,
                            gpart, gnorm2 != nullptr, B, H, W, th, s);
  else
    energy_dispatch<float>((const float*)R, (const float*)T, (const float*)u, lam, (float*)grad, part,
                           gpart, gnorm2 != nullptr, B, H, W, th, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_tiles, dim3(B), dim3(kWave), 0, s, part, gpart, nt, E, gnorm2);
  return hipGetLastError();
}

hipError_t launch_energy_backward_level(const void* Ia, const void* u, const void* Ib, double lam,
                                        const double* gE, void* dIa, void* du, void* dIb, const void* du_c,
                                        bool carry, int B, int h, int w, bool f64, hipStream_t s) {
  const size_t n = (size_t)B * h * w;
  if (n == 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_energy_backward<double>, adjoint_grid(B, h, w, kBackRows), dim3(kEW), 0, s, (const double*)Ia,
                       (const double*)u, (const double*)Ib, lam, gE, (double*)dIa, (double*)du, (double*)dIb,
                       (const double*)du_c, carry, B, h, w);
  else
    hipLaunchKernelGGL(k_energy_backward<float>, adjoint_grid(B, h, w, kBackRows), dim3(kEW), 0, s, (const float*)Ia,
                       (const float*)u, (const float*)Ib, lam, gE, (float*)dIa, (float*)du,
                       (float*)dIb, (const float*)du_c, carry, B, h, w);
  return hipGetLastError();
}

hipError_t launch_synth_frames(float* out, int F, int H, int W, hipStream_t s) {
  const size_t n = (size_t)F * H * W;
  hipLaunchKernelGGL(k_synth_frames, dim3(ew_blocks(n)), dim3(kEW), 0, s, out, F, H, W);
  return hipGetLastError();
}

hipError_t launch_add_energy(const double* Ein, double* Eacc, int B, int first, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_energy, dim3((B + 255) / 256), dim3(256), 0, s, Ein, Eacc, B, first);
  return hipGetLastError();
}

}  // namespace rs
