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

#include "device_common.h"

namespace rs {

enum SweepWrite { SW_NONE = 0, SW_UPDATE = 1, SW_GRAD = 2 };

template <typename S>
struct LevelView {
  const S* R;   // [h][w]
  const S* T;   // [h][w]
  const S* u;   // [2][h][w]
  S* out;       // [2][h][w]: u' (SW_UPDATE) or dE/du (SW_GRAD)
  int h, w;
  double tau, lam;
};

__host__ __device__ inline int tiles_x(int w) { return (w + kTileW - 1) / kTileW; }
__host__ __device__ inline int tiles_of(int h, int w, int th) { return tiles_x(w) * ((h + th - 1) / th); }

// Returns the tile energy in thread 0 (other threads: unspecified).  With
// GNORM, *gn (thread 0) receives sum_x |g(x)|^2 of the tile.  `red` is
// __shared__ double[kWG / kWave].  Must be called by all kWG threads.
// Arithmetic is double; the stored type S is float (or double).
template <typename S, int WRITE, bool GNORM>
__device__ double sweep_tile(const LevelView<S>& L, int tile, int th, double* red, double* gn) {
  const int h = L.h, w = L.w;
  const int ntx = tiles_x(w);
  const int tx = tile % ntx, ty = tile / ntx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rpw = th >> 2;
  const int x = tx * kTileW + lane;
  const bool vx = x < w;
  const int xc = vx ? x : w - 1;
  const int y0 = ty * th + wave * rpw;
  const int y1 = min(y0 + rpw, h);
  const size_t hw = (size_t)h * w;
  const SharedBuf ub(L.u);           // plane 0 at 0, plane 1 at hw
  const int ihw = (int)hw;
  const S* __restrict__ Rr = L.R;
  const double lam = L.lam, tau = L.tau;
  double acc = 0.0, gacc = 0.0;

  if (y0 < y1) {
    S ax[kRB + 2], ay[kRB + 2];   // column values of rows yb-1 .. yb+kRB
    const int ym = y0 > 0 ? y0 - 1 : 0;
    ax[0] = ub.load<S>(ym * w + xc);
    ay[0] = ub.load<S>(ihw + ym * w + xc);
    ax[1] = ub.load<S>(y0 * w + xc);
    ay[1] = ub.load<S>(ihw + y0 * w + xc);
    for (int yb = y0; yb < y1; yb += kRB) {
      S rr[kRB];
#pragma unroll
      for (int r = 0; r < kRB; ++r) {
        const int yn = min(yb + 1 + r, h - 1);
        ax[r + 2] = ub.load<S>(yn * w + xc);
        ay[r + 2] = ub.load<S>(ihw + yn * w + xc);
        rr[r] = Rr[min(yb + r, h - 1) * w + xc];
      }
#pragma unroll
      for (int r = 0; r < kRB; ++r) {
        const int y = yb + r;
        if (y >= y1) break;
        const S cxs = ax[r + 1], cys = ay[r + 1];
        S lxs = __shfl_up(cxs, 1, kWave), lys = __shfl_up(cys, 1, kWave);
        S rxs = __shfl_down(cxs, 1, kWave), rys = __shfl_down(cys, 1, kWave);
        if (lane == 0 && x > 0) {
          lxs = ub.load<S>(y * w + x - 1);
          lys = ub.load<S>(ihw + y * w + x - 1);
        }
        if (lane == kWave - 1 && x + 1 < w) {
          rxs = ub.load<S>(y * w + x + 1);
          rys = ub.load<S>(ihw + y * w + x + 1);
        }
        const bool hl = x > 0, hr = x + 1 < w, hu = y > 0, hd = y + 1 < h;
        int ix, iy;
        double fx, fy;
        cell_of(cxs, ix, fx);
        cell_of(cys, iy, fy);
        double s, dsx, dsy;
        bilin(L.T, h, w, xc + ix, y + iy, fx, fy, s, dsx, dsy);
        const double cx = cxs, cy = cys;
        const double lx = lxs, ly = lys, rx = rxs, ry = rys;
        const double upx = ax[r], upy = ay[r], dnx = ax[r + 2], dny = ay[r + 2];
        const double res = s - (double)rr[r];
        const double drx = hr ? rx - cx : 0.0, dry = hr ? ry - cy : 0.0;
        const double ddx = hd ? dnx - cx : 0.0, ddy = hd ? dny - cy : 0.0;
        const double e = res * res + lam * ((drx * drx + ddx * ddx) + (dry * dry + ddy * ddy));
        const double nbx = ((hl ? cx - lx : 0.0) + (hr ? cx - rx : 0.0)) +
                           ((hu ? cx - upx : 0.0) + (hd ? cx - dnx : 0.0));
        const double nby = ((hl ? cy - ly : 0.0) + (hr ? cy - ry : 0.0)) +
                           ((hu ? cy - upy : 0.0) + (hd ? cy - dny : 0.0));
        const double gx = 2.0 * res * dsx + 2.0 * lam * nbx;
        const double gy = 2.0 * res * dsy + 2.0 * lam * nby;
        if (vx) {
          acc += e;
          if (WRITE == SW_UPDATE) {
            L.out[y * w + x] = (S)(cx - tau * gx);
            L.out[hw + y * w + x] = (S)(cy - tau * gy);
          } else if (WRITE == SW_GRAD) {
            L.out[y * w + x] = (S)gx;
            L.out[hw + y * w + x] = (S)gy;
          }
          if (GNORM) gacc += gx * gx + gy * gy;
        }
      }
      ax[0] = ax[kRB];
      ay[0] = ay[kRB];
      ax[1] = ax[kRB + 1];
      ay[1] = ay[kRB + 1];
    }
  }
  const double E = block_sum(acc, red);
  if (GNORM) {
    const double G = block_sum(gacc, red);
    if (threadIdx.x == 0) *gn = G;
  }
  return E;
}

// Initial guess of a registration on its coarsest level (pixel (X, Y)):
// the fine-level guess restricted L-1 times by half the 2x2 block mean, i.e.
// 2^-(L-1) times the mean over the 2^(L-1) x 2^(L-1) block.  kind 0: zero;
// kind 1: the composition ua(x) + ub(x + ua(x)); kind 2: the field ua.
template <typename S>
__device__ __forceinline__ void init_pixel(int kind, const S* __restrict__ ua, const S* __restrict__ ub,
                                           int H, int W, int levels, int X, int Y, double& vx, double& vy) {
  if (kind == 0) {
    vx = 0.0;
    vy = 0.0;
    return;
  }
  const int F = 1 << (levels - 1);
  const size_t HW = (size_t)H * W;
  double sx = 0.0, sy = 0.0;
  for (int dy = 0; dy < F; ++dy) {
    const int y = Y * F + dy;
    for (int dx = 0; dx < F; ++dx) {
      const int x = X * F + dx;
      const S ax = ua[y * W + x], ay = ua[HW + y * W + x];
      if (kind == 1) {
        int ix, iy;
        double fx, fy;
        cell_of(ax, ix, fx);
        cell_of(ay, iy, fy);
        sx += (double)ax + bilin_value(ub, H, W, x + ix, y + iy, fx, fy);
        sy += (double)ay + bilin_value(ub + HW, H, W, x + ix, y + iy, fx, fy);
      } else {
        sx += (double)ax;
        sy += (double)ay;
      }
    }
  }
  const double scale = 1.0 / ((double)F * F * F);
  vx = sx * scale;
  vy = sy * scale;
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
