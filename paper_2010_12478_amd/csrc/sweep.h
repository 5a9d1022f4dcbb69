// The fused gradient-descent sweep over one tile of a pyramid level.
//
// For every pixel x of the tile (registration functional, Section 2.3.1, in
// its dense-displacement form):
//   S, dS/dp  = bilinear sample of T at x + u(x) and its position derivative
//   r         = S - R(x)
//   e(x)      = r^2 + lambda * sum_c [(u_c(x+e1) - u_c(x))^2 + (u_c(x+e2) - u_c(x))^2]
//               (pairs inside the grid only)
//   g_c(x)    = 2 r dS/dp_c + 2 lambda sum_{n in N4(x) inside the grid} (u_c(x) - u_c(n))
//   u'(x)     = u(x) - tau g(x)                     (update mode)
// and the tile energy sum_x e(x) accumulated in double in a fixed order.
// All arithmetic is double; values are stored as float, so the update is the
// double result rounded once.
//
// Layout: a tile is 64 columns (one wavefront, lane = column) by `th` rows;
// the 4 wavefronts of the workgroup take th/4 consecutive rows each and walk
// down their column keeping the rows above / below in registers, so every u
// value is loaded once per sweep (through SharedBuf: other workgroups of a
// persistent launch write these fields).  Horizontal neighbours come from the
// adjacent lanes (cross-lane shuffles); lanes 0 and 63 read the one column
// outside the tile.  R and u are read and u' written fully coalesced; the 4
// taps of T are gathered through the vector L1/L2 (the displacement field is
// smooth, so a wavefront's taps fall on a few adjacent cache lines).
#pragma once

#include <type_traits>

#include "device_common.h"

namespace rs {

enum SweepWrite { SW_NONE = 0, SW_UPDATE = 1, SW_GRAD = 2 };

// One pyramid level of one registration.  R and T point at pixel (0, 0) of
// rows `pitch` elements apart.  In the solver's padded pyramid (PAD) every
// level carries a one-pixel replicate border: rows -1 .. h and columns
// -1 .. w are readable and hold the value of the nearest pixel, so a
// bilinear cell clamped to [-1, h-1] x [-1, w-1] reads exactly the values the
// edge-clamped taps would.
template <typename S>
struct LevelView {
  const S* R;   // [h][pitch]
  const S* T;   // [h][pitch]
  const S* u;   // [2][h][w]
  S* out;       // [2][h][w]: u' (SW_UPDATE) or dE/du (SW_GRAD)
  int h, w, pitch;
  double tau, lam;
};

__host__ __device__ inline int tiles_x(int w) { return (w + kTileW - 1) / kTileW; }
__host__ __device__ inline int tiles_of(int h, int w, int th) { return tiles_x(w) * ((h + th - 1) / th); }

// Tile height of pyramid level l for a finest-level tile height th0: a
// quarter per level (both sides halve), at least 4 rows, so that every level
// of a square image has about as many tiles as the finest one.
__host__ __device__ inline int level_tile_rows(int th0, int l) {
  const int t = th0 >> (2 * l);
  return t < 4 ? 4 : t;
}

// Tile height of a level the solver streams.  A level that some launch
// could run register-resident (64-column tiles, a power-of-two height of at
// most 64 rows that divides the level, at most max_group tiles) streams in
// the same tiles, so that both forms sum its energy alike; any other level
// is tiled at least 4 * kRBStream rows high, so that each wavefront's share
// of a tile (a quarter) holds a whole batch of kRBStream rows (a shorter
// share loads the halo rows and gathers of a full batch for fewer rows).
__host__ __device__ inline int stream_tile_rows(int th, int h, int w, int max_group) {
  const bool may_be_resident = w % kTileW == 0 && h % th == 0 && th <= 4 * kMaxRPT && (th & (th - 1)) == 0 &&
                               tiles_of(h, w, th) <= max_group;
  return may_be_resident || th >= 4 * kRBStream ? th : 4 * kRBStream;
}

// One pixel of the fused sweep, everything in double: bilinear sample S of T
// from the taps i00 (x0, y0), i01 (x0 + 1, y0), i10 (x0, y0 + 1), i11 at the
// in-cell fractions (fx, fy), with its position derivatives; residual
// r = S - R; the differences of the pixel's displacement c to its neighbours
// (l/r/u/d = left/right/up/down; a neighbour outside the grid is the pixel
// itself, difference +0):
//   S     = (1 - fy) ((1 - fx) i00 + fx i01) + fy ((1 - fx) i10 + fx i11)
//   dS/dx = (1 - fy) (i01 - i00) + fy (i11 - i10)
//   dS/dy = (1 - fx) (i10 - i00) + fx (i11 - i01)
//   g     = (2 r) dS/dp + (2 lam) ((((c - l) + (c - r)) + (c - u)) + (c - d))
// The gradient (and with it every stored iterate) is evaluated without
// contraction: each product and sum is one rounded float64 operation, in the
// order written above, so any implementation of these formulas in that
// order produces the same bits.  The energy terms r^2 and
// (r - c)^2 + (d - c)^2 of both components (the forward differences inside
// the grid) go to the accumulators accR and accG, with fused operations: the
// energy only feeds the stopping test.  Every execution path evaluates a
// pixel through this function, so they agree bitwise.
__device__ __forceinline__ void pixel_eval_d(double fx, double fy, double i00, double i01, double i10, double i11,
                                             double R, double lxd, double rxd, double uxd, double dxd, double lyd,
                                             double ryd, double uyd, double dyd, double lam, double& accR,
                                             double& accG, double& gx, double& gy) {
#pragma clang fp contract(off)
  const double ox = 1.0 - fx, oy = 1.0 - fy;
  const double s = oy * (ox * i00 + fx * i01) + fy * (ox * i10 + fx * i11);
  const double sx = oy * (i01 - i00) + fy * (i11 - i10);
  const double sy = ox * (i10 - i00) + fx * (i11 - i01);
  const double res = s - R;
  const double nbx = ((lxd + rxd) + uxd) + dxd;
  const double nby = ((lyd + ryd) + uyd) + dyd;
  const double r2 = 2.0 * res, l2 = 2.0 * lam;
  gx = r2 * sx + l2 * nbx;
  gy = r2 * sy + l2 * nby;
  accR = fma(res, res, accR);
  accG = fma(rxd, rxd, fma(dxd, dxd, fma(ryd, ryd, fma(dyd, dyd, accG))));
}

// A lane's energy over its rows of a tile from its two accumulators.
__device__ __forceinline__ double lane_energy(double accR, double accG, double lam) {
  return fma(lam, accG, accR);
}

// Gradient-descent update of one component, c - tau g (one rounded product,
// one rounded difference), rounded once to the stored type.
template <typename S>
__device__ __forceinline__ S gd_update(double c, double g, double tau) {
#pragma clang fp contract(off)
  return (S)(c - tau * g);
}

// Registers of one unit of work of a wavefront: rows [yb, ye) (at most RB)
// of one tile, lane = column.  k, x0, yb, ye and last are wave-uniform.
template <typename S, int RB>
struct Unit {
  int k;                        // the tile's index in the workgroup's share (by rows of 4: the row's)
  int x0, yb, ye;               // first column of the tile; rows
  bool last;                    // the quarter's last unit
  S ax[RB + 2], ay[RB + 2];   // u at rows yb-1 .. yb+RB of this lane's column (rows clamped)
  S rr[RB];                     // R at rows yb .. yb+RB-1
  S hx[RB], hy[RB];            // lane 0: u at column x-1, lane 63: u at column x+1
};

// LDS doubles a sweep_tiles caller provides as `red` for RT tile sums per
// flush.
template <bool GNORM>
__host__ __device__ constexpr int sweep_red_doubles(int RT) {
  return RT * (kWG / kWave) * (GNORM ? 2 : 1);
}

// Sweeps the workgroup's share of the tiles of level L: the tiles first,
// first + stride, ... or, with ROWS4 and a level whose width in tiles is a
// multiple of 4, the rows of 4 side-by-side tiles first, first +
// stride, ... (in the same order as tiles, ntx / 4 such rows per row of
// tiles).  For every tile the energy (and with GNORM the squared gradient
// norm) is summed in a fixed order: per lane over the rows of a quarter of
// the tile (th / 4 rows) in order, wave_sum over the wavefront, then the 4
// quarters in order (from 0.0, as block_sum); the result goes to part[tile]
// (gpart[tile]).  The quarter sums of up to RT tiles wait in `red`
// (sweep_red_doubles<GNORM>(RT) doubles of LDS) and are combined and stored
// together, so the workgroup synchronises twice per RT tiles rather than
// twice per tile.  Must be called by all kWG threads.
//
// Each wavefront walks a sequence of units of at most RB rows: by tiles,
// wavefront i takes quarter i of each tile of the share; by rows of 4, it
// takes tile i of each row whole, quarter after quarter, so the 4 tiles a
// workgroup sweeps at a time sit side by side and the border columns one
// wavefront reads are the lines its neighbours load at the same time (the
// same sums either way: a quarter is summed by one wavefront).  The loop is
// software-pipelined: the gathers of T for unit i are issued before the u, R
// and halo loads of unit i + 1, and unit i is computed while those are in
// flight, so each unit exposes one memory round trip instead of two; it is
// unrolled twice so that the two units in flight swap roles instead of
// being copied.  Loads and stores share one counter on this GPU, and the
// compiler's wait for a load holds on every path into it: so every unit
// issues the same loads (no per-lane branch around them; a unit continuing
// its tile only skips the two u rows it takes from the previous unit) and
// the last unit is peeled off the loop, or the arithmetic's wait for its
// taps would also drain the next unit's loads.  Every row of a unit is the same
// for the whole wavefront, so row offsets are wave-uniform: loads and stores
// take them as the scalar offset of a buffer instruction and the lane's
// column offset once per unit (no per-row vector address arithmetic), and
// each row of u is converted to double once per unit for its three uses
// (centre, row above, row below).
// Arithmetic is double; the stored type S is float (or double).
template <typename S, int WRITE, bool GNORM, bool PAD, int RB = kRB, int RT = 1, bool ROWS4 = false>
__device__ void sweep_tiles(const LevelView<S>& L, int first_, int stride_, int th_, double* red, double* part,
                            double* gpart) {
  static_assert(RT >= 1 && RT <= kWG, "tile sums per flush");
  static_assert(!ROWS4 || RT % 4 == 0, "rows of 4 tiles are flushed whole");
  constexpr int NW = kWG / kWave;
  // every quantity but the lane is the same across the wavefront: held in
  // scalar registers, so everything derived from it is too
  const int first = __builtin_amdgcn_readfirstlane(first_);
  const int stride = __builtin_amdgcn_readfirstlane(stride_);
  const int th = __builtin_amdgcn_readfirstlane(th_);
  const int h = __builtin_amdgcn_readfirstlane(L.h), w = __builtin_amdgcn_readfirstlane(L.w);
  const int pitch = __builtin_amdgcn_readfirstlane(L.pitch);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int ntx = tiles_x(w);
  const int nt = tiles_of(h, w, th);
  const int rpw = th >> 2;                        // rows of a quarter of a tile
  const int upt = (rpw + RB - 1) / RB;            // units per quarter
  // by rows of 4 tiles: every wavefront has the same number of units, so the
  // flushes below stay block-uniform
  const bool rows4 = ROWS4 && ntx % 4 == 0;
  const int nsx = ntx >> 2;
  const int n_items = rows4 ? nt >> 2 : nt;
  const int my_tiles = first < n_items ? (n_items - first + stride - 1) / stride : 0;   // rows4: rows of 4
  const int n_units = my_tiles * upt * (rows4 ? 4 : 1);
  const int ihw = h * w;
  const SharedBuf ub(L.u);                          // plane 0 at 0, plane 1 at h * w
  // padded: T addressed from its (-1, -1) element, so every offset is >= 0
  const ReadBuf rb(L.R), tb(PAD ? L.T - pitch - 1 : L.T);
  const ReadBuf ob(WRITE != SW_NONE ? (const void*)L.out : (const void*)L.R);   // stores only
  const double lam = L.lam, tau = L.tau;

  // position of the next unit: index k in the share (tile, or row of 4
  // tiles), the tile's column and row in the tile grid, the quarter nq
  // (rows4) and the unit's batch b within the quarter
  int nk = 0, nq = 0, nb = 0, nty, ntxc;
  auto place = [&](int item) {   // one division per tile (row of tiles)
    if (rows4) {
      nty = item / nsx;
      ntxc = (item - nty * nsx) * 4 + wave;
    } else {
      nty = item / ntx;
      ntxc = item - nty * ntx;
    }
  };
  place(first);
  auto setup = [&](Unit<S, RB>& U) {
    U.k = nk;
    U.x0 = ntxc * kTileW;
    const int ys = nty * th + (rows4 ? nq : wave) * rpw;
    const int yend = min(ys + rpw, h);
    U.yb = ys + nb * RB;
    U.ye = min(U.yb + RB, yend);
    U.last = nb == upt - 1;
    if (++nb == upt) {
      nb = 0;
      if (!rows4 || ++nq == 4) {
        nq = 0;
        ++nk;
        place(first + nk * stride);
      }
    }
  };
  // The same loads for every lane (no lane branch), so that the compiler's
  // count of outstanding loads is the same on every path into the arithmetic
  // and its wait for the taps does not also drain the next unit's loads:
  // rows clamped to the image (a unit with no rows loads the last row), and
  // each lane loads one border column (lane 0 the one left of the tile, lane
  // 63 the one right of it, the others their own column, unused).
  // P: the unit before U in this wavefront's sequence.  When U continues
  // P's tile, its first two rows of u (the row above it and its first row)
  // are P's last two, taken from P's registers instead of loaded again.
  // That wave-uniform branch is the one difference between paths: the wait
  // for the taps then counts the shorter sequence, so the first unit of a
  // tile waits for its taps four loads earlier than it needs to.
  auto load = [&](Unit<S, RB>& U, const Unit<S, RB>& P) {
    const int x = U.x0 + lane;
    const int xc = min(x, w - 1);
    const int xn = lane == 0 ? max(x - 1, 0) : (lane == kWave - 1 ? min(x + 1, w - 1) : xc);
    const bool cont = U.k == P.k && U.yb == P.yb + RB;   // the same tile, the next rows
    if (cont) {
      U.ax[0] = P.ax[RB];
      U.ax[1] = P.ax[RB + 1];
      U.ay[0] = P.ay[RB];
      U.ay[1] = P.ay[RB + 1];
    }
#pragma unroll
    for (int r = 0; r < RB + 2; ++r) {
      if (r < 2 && cont) continue;
      // rows clamped to the image: at the top / bottom edge the missing
      // neighbour row is the pixel's own row
      const int row = clampi(U.yb - 1 + r, 0, h - 1) * w;
      U.ax[r] = ub.template load<S>(xc, row);
      U.ay[r] = ub.template load<S>(xc, ihw + row);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) U.rr[r] = rb.template load<S>(xc, min(U.yb + r, h - 1) * pitch);
    // the column outside the tile, clamped to the image: at the image edge
    // it is the pixel's own column, so the missing difference is exactly 0
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int row = min(U.yb + r, h - 1) * w;
      U.hx[r] = ub.template load<S>(xn, row);
      U.hy[r] = ub.template load<S>(xn, ihw + row);
    }
  };

  double accR = 0.0, accG = 0.0, accN = 0.0;
  int lq = 0;   // rows4: the quarter the next last unit ends
  // unit i in C (loaded), unit i + 1 into D
  auto step = [&](Unit<S, RB>& C, Unit<S, RB>& D, auto next) {
    const int x = C.x0 + lane;
    const bool vx = x < w;
    const int xc = vx ? x : w - 1;
    // gathers of T for this unit (also for a unit with no rows, whose taps
    // are unused: every tap address is clamped into the level, whatever u)
    S taps[RB][4];
    // u in double (each row for its three uses), and the cells from its floors
    double axd[RB + 2], ayd[RB + 2];
#pragma unroll
    for (int r = 0; r < RB + 2; ++r) {
      axd[r] = (double)C.ax[r];
      ayd[r] = (double)C.ay[r];
    }
    double flx[RB], fly[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int ix, iy;
      flx[r] = floor_cell_d(axd[r + 1], ix);
      fly[r] = floor_cell_d(ayd[r + 1], iy);
      const int x0 = xc + ix, y0 = min(C.yb + r, h - 1) + iy;
      if constexpr (PAD) {
        // the cell clamped to [-1, w-1] x [-1, h-1], offset by the border
        const int o = __mul24(clamp0(y0 + 1, h), pitch) + clamp0(x0 + 1, w);
        tb.template load2<S>(o, 0, taps[r][0], taps[r][1]);
        tb.template load2<S>(o, pitch, taps[r][2], taps[r][3]);
      } else {
        const int xa = clamp0(x0, w - 1), xb = clamp0(x0 + 1, w - 1);
        const int ya = __mul24(clamp0(y0, h - 1), w), yb = __mul24(clamp0(y0 + 1, h - 1), w);
        taps[r][0] = tb.template load<S>(ya + xa, 0);
        taps[r][1] = tb.template load<S>(ya + xb, 0);
        taps[r][2] = tb.template load<S>(yb + xa, 0);
        taps[r][3] = tb.template load<S>(yb + xb, 0);
      }
    }
    // loads of the next unit, in flight during this unit's arithmetic
    if constexpr (decltype(next)::value) {
      setup(D);
      load(D, C);
    }
    if (C.yb < C.ye) {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int y = C.yb + r;
        if (y >= C.ye) break;
        const S cxs = C.ax[r + 1], cys = C.ay[r + 1];
        // neighbours: lanes past the right edge hold column w - 1, so every
        // missing neighbour equals the pixel's own value (difference +0.0,
        // the same as leaving the term out); lane 0 holds the column left of
        // the tile in hx/hy, lane 63 the one right of it
        const S lxs = wave_from_left(cxs, C.hx[r]), lys = wave_from_left(cys, C.hy[r]);
        const S rxs = wave_from_right(cxs, C.hx[r]), rys = wave_from_right(cys, C.hy[r]);
        const double cx = axd[r + 1], cy = ayd[r + 1];
        double nR = accR, nG = accG, gx, gy;   // accumulated only for pixels inside the grid
        pixel_eval_d(cx - flx[r], cy - fly[r], taps[r][0], taps[r][1], taps[r][2], taps[r][3],
                     C.rr[r], cx - (double)lxs, cx - (double)rxs, cx - axd[r], cx - axd[r + 2],
                     cy - (double)lys, cy - (double)rys, cy - ayd[r], cy - ayd[r + 2], lam, nR, nG, gx, gy);
        if (vx) {
          accR = nR;
          accG = nG;
          const int so = y * w;
          if (WRITE == SW_UPDATE) {
            ob.template store<S>(x, so, gd_update<S>(cx, gx, tau));
            ob.template store<S>(x, ihw + so, gd_update<S>(cy, gy, tau));
          } else if (WRITE == SW_GRAD) {
            ob.template store<S>(x, so, (S)gx);
            ob.template store<S>(x, ihw + so, (S)gy);
          }
          if (GNORM) accN += gx * gx + gy * gy;
        }
      }
    }
    if (C.last) {   // last unit of a quarter of a tile: its wavefront sums
      const int k = C.k;
      const int cq = rows4 ? lq : wave;   // the quarter this unit ends
      lq = (lq + 1) & 3;
      const int slot = (rows4 ? 4 * k + wave : k) % RT;   // the tile's place in the flush
      const double e = wave_sum(lane_energy(accR, accG, lam));
      if (lane == 0) red[slot * NW + cq] = e;
      accR = 0.0;
      accG = 0.0;
      if (GNORM) {
        const double gs = wave_sum(accN);
        if (lane == 0) red[(RT + slot) * NW + cq] = gs;
        accN = 0.0;
      }
      // items (tiles, or rows of 4 tiles) per flush; the same unit of every
      // wavefront, so block-uniform
      const int per = rows4 ? RT / 4 : RT;
      const int q = k % per;
      if ((!rows4 || cq == NW - 1) && (q == per - 1 || k == my_tiles - 1)) {   // combine in order and store
        __syncthreads();
        if ((int)threadIdx.x < (rows4 ? 4 * (q + 1) : q + 1)) {
          const int i = (k - q) * (rows4 ? 4 : 1) + (int)threadIdx.x;   // tile index in the share
          int tile;
          if (rows4) {
            const int item = first + (i >> 2) * stride;
            const int ty = item / nsx;
            tile = ty * ntx + (item - ty * nsx) * 4 + (i & 3);
          } else {
            tile = first + i * stride;
          }
          double t = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) t += red[threadIdx.x * NW + w];
          part[tile] = t;
          if (GNORM) {
            double tg = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) tg += red[(RT + threadIdx.x) * NW + w];
            gpart[tile] = tg;
          }
        }
        __syncthreads();
      }
    }
  };

  Unit<S, RB> A, B;
  using more = std::true_type;
  using last = std::false_type;
  if (n_units > 0) {
    setup(A);
    B.k = -1;   // no unit before the first
    load(A, B);
  }
  // the last unit is peeled off the loop: inside it every step loads the next unit
  int i = 0;
  for (; i + 2 < n_units; i += 2) {
    step(A, B, more{});
    step(B, A, more{});
  }
  if (n_units - i == 2) {
    step(A, B, more{});
    step(B, A, last{});
  } else if (n_units - i == 1) {
    step(A, B, last{});
  }
}

// Initial guess at fine pixel (x, y), in double.  kind 1: the composition
// ua(x) + ub(x + ua(x)); kind 2: the field ua.
template <typename S>
__device__ __forceinline__ void init_fine(int kind, const S* __restrict__ ua, const S* __restrict__ ub, int H,
                                          int W, int x, int y, double& vx, double& vy) {
#pragma clang fp contract(off)
  const size_t HW = (size_t)H * W;
  const S ax = ua[y * W + x], ay = ua[HW + y * W + x];
  if (kind == 1) {
    int ix, iy;
    double fx, fy;
    cell_of(ax, ix, fx);
    cell_of(ay, iy, fy);
    vx = (double)ax + bilin_value(ub, H, W, x + ix, y + iy, fx, fy);
    vy = (double)ay + bilin_value(ub + HW, H, W, x + ix, y + iy, fx, fy);
  } else {
    vx = (double)ax;
    vy = (double)ay;
  }
}

// The fine-level guess restricted D times by half the 2x2 block mean, at
// pixel (X, Y) of the level D coarser, in double throughout.  Every level is
// 0.5 * (0.25 * (((v00 + v01) + v10) + v11)) of the four values below it
// (v00 at (2X, 2Y), v01 at (2X + 1, 2Y), v10 at (2X, 2Y + 1)), each one
// rounded float64 operation, without contraction: the definition's order.
template <int D, typename S>
__device__ void init_restricted(int kind, const S* __restrict__ ua, const S* __restrict__ ub, int H, int W,
                                int X, int Y, double& vx, double& vy) {
#pragma clang fp contract(off)
  if constexpr (D == 0) {
    init_fine<S>(kind, ua, ub, H, W, X, Y, vx, vy);
  } else {
    double sx = 0.0, sy = 0.0;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      double tx, ty;
      init_restricted<D - 1, S>(kind, ua, ub, H, W, 2 * X + (q & 1), 2 * Y + (q >> 1), tx, ty);
      sx = q == 0 ? tx : sx + tx;
      sy = q == 0 ? ty : sy + ty;
    }
    vx = 0.5 * (0.25 * sx);
    vy = 0.5 * (0.25 * sy);
  }
}

// Initial guess of a registration on its coarsest level (pixel (X, Y)):
// the fine-level guess restricted L-1 times by half the 2x2 block mean.
// kind 0: zero; kind 1: the composition ua(x) + ub(x + ua(x)); kind 2: the
// field ua.
template <typename S>
__device__ __forceinline__ void init_pixel(int kind, const S* __restrict__ ua, const S* __restrict__ ub,
                                           int H, int W, int levels, int X, int Y, double& vx, double& vy) {
  switch (kind == 0 ? -1 : levels - 1) {
    case 0: init_restricted<0, S>(kind, ua, ub, H, W, X, Y, vx, vy); return;
    case 1: init_restricted<1, S>(kind, ua, ub, H, W, X, Y, vx, vy); return;
    case 2: init_restricted<2, S>(kind, ua, ub, H, W, X, Y, vx, vy); return;
    case 3: init_restricted<3, S>(kind, ua, ub, H, W, X, Y, vx, vy); return;
    case 4: init_restricted<4, S>(kind, ua, ub, H, W, X, Y, vx, vy); return;
    case 5: init_restricted<5, S>(kind, ua, ub, H, W, X, Y, vx, vy); return;
    case 6: init_restricted<6, S>(kind, ua, ub, H, W, X, Y, vx, vy); return;
    case 7: init_restricted<7, S>(kind, ua, ub, H, W, X, Y, vx, vy); return;
    default: vx = 0.0; vy = 0.0; return;
  }
}

// Prolongation of a coarse displacement [2][hc][wc] to fine pixel (x, y):
// 2 * uc((x - 1/2)/2, (y - 1/2)/2), bilinear with clamped taps.  SHARED: uc
// is written by other workgroups of the launch and is wave-uniform (loads
// through SharedBuf); otherwise plain loads.
template <bool SHARED>
__device__ __forceinline__ void prolong_pixel(const float* __restrict__ uc, int hc, int wc, int x, int y,
                                              double& vx, double& vy) {
  const int x0 = (x - 1) >> 1, y0 = (y - 1) >> 1;      // floor((x - 1/2) / 2)
  const double wx = (x & 1) ? 0.25 : 0.75;
  const double wy = (y & 1) ? 0.25 : 0.75;
  if (SHARED) {
    const SharedBuf bx(uc), by(uc + (size_t)hc * wc);
    vx = 2.0 * bilin_value_shared(bx, hc, wc, x0, y0, wx, wy);
    vy = 2.0 * bilin_value_shared(by, hc, wc, x0, y0, wx, wy);
  } else {
    vx = 2.0 * bilin_value(uc, hc, wc, x0, y0, wx, wy);
    vy = 2.0 * bilin_value(uc + (size_t)hc * wc, hc, wc, x0, y0, wx, wy);
  }
}

}  // namespace rs
