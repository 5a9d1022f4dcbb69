// Register-resident gradient descent on one pyramid level.
//
// A level is cut into tiles of 64 columns by th = 4 * RPT rows; the group's
// member m owns tile m for the whole level.  Lane = column, wavefront w of the
// workgroup holds rows y0 .. y0 + RPT - 1 of the tile (y0 = tile row + w*RPT)
// of the displacement field in registers, so an iteration reads from memory
// only R and the four taps of T per pixel (through L1/L2) and the halo of its
// tile, and writes only the tile's halo-facing values:
//   - rows: every wavefront stores its first and last row, and loads the row
//     above its first and below its last (rows clamped to the grid: at the
//     border the neighbour is the pixel itself, so the difference is 0);
//   - columns: lanes 0 and 63 store their column into a small exchange
//     buffer (contiguous per tile, side and wavefront), and one wave-wide
//     load fetches the columns left and right of the tile for the
//     wavefront's rows; a cross-lane permute puts each row's pair into lanes
//     0 / 63.
// The field is updated in place, row by row (the old value of the row above
// is kept aside for the next row).  The state an iteration starts from is
// copied to LDS first: when the energy of that iteration stops the level, it
// is the result.  The halo values of iteration t are read from U[t % 2] and
// those of its result written to U[(t + 1) % 2] (full-size fields of which
// only halo rows are written; the columns likewise alternate between two
// exchange buffers), so a reader in iteration t reads what its neighbours
// wrote before the barrier that ended iteration t - 1, and the writers of
// iteration t write the other buffer.
//
// Per pixel and iteration the arithmetic is pixel_eval and gd_update, the tile
// energy is summed in the order of the streaming sweep with the same tile
// height (per lane over its rows, wave_sum, the 4 wavefronts), so both
// paths produce bitwise identical fields, energies and iteration counts.
#pragma once

#include "sweep.h"

namespace rs {

// Whole-wavefront lane shifts by one (DPP wave_shr:1 / wave_shl:1): lane i
// receives src from lane i - 1 (from_left) or i + 1 (from_right); the lane
// without a source (0, respectively 63) keeps `edge`.
__device__ __forceinline__ float from_left(float src, float edge) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                               __builtin_bit_cast(int, src), 0x138, 0xf, 0xf,
                                                               false));
}
__device__ __forceinline__ float from_right(float src, float edge) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                               __builtin_bit_cast(int, src), 0x130, 0xf, 0xf,
                                                               false));
}

// Value of `v` in lane `src_lane` (per lane), through the LDS crossbar.
__device__ __forceinline__ float lane_pull(float v, int src_lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src_lane << 2, __builtin_bit_cast(int, v)));
}

struct ResidentTile {
  int h, w, hw;
  int pitch;         // row pitch of R and T (padded pyramid: one-pixel replicate border)
  int xt, y0;        // the tile's first column, the wavefront's first row
  int tile, tx, ntx, wave;
  int lane;
  double tau, lam;
};

// Column-halo exchange buffer (one parity): for every tile, side (0: its
// first column, 1: its last), wavefront and component the wavefront's RPT
// rows, contiguous, so a wavefront reads each neighbouring column it needs
// from one 2 RPT-float run.
template <int RPT>
__device__ __forceinline__ int colx_index(int tile, int side, int wave, int comp, int r) {
  return (((tile * 2 + side) * 4 + wave) * 2 + comp) * RPT + r;
}

// Lanes 0 and 63 store the tile's first and last columns of (sx, sy).
template <int RPT>
__device__ __forceinline__ void store_columns(const ResidentTile& P, const float (&sx)[RPT], const float (&sy)[RPT],
                                              const ReadBuf& cx, int lane) {
  if (lane == 0 || lane == kWave - 1) {
    const int side = lane == 0 ? 0 : 1;
    const int b = colx_index<RPT>(P.tile, side, P.wave, 0, 0);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      cx.st32(b + r, 0, sx[r]);
      cx.st32(b + RPT + r, 0, sy[r]);
    }
  }
}

// One iteration on the state (sx, sy), updated in place (R read through rb
// from pixel (0, 0), T through tb from its border element (-1, -1)): returns
// this lane's energy over its rows (accumulated in row order).  `ucur` holds the halo of the state; the halo-facing values of the
// new state are stored through `unext`; the old state is saved to `roll`
// (RPT float2 per thread, LDS).
template <int RPT>
__device__ __forceinline__ double resident_step(const ResidentTile& P, float (&sx)[RPT], float (&sy)[RPT],
                                                const SharedBuf& ucur, const ReadBuf& unext, const SharedBuf& ccur,
                                                const ReadBuf& cnext, const ReadBuf& tb, const ReadBuf& rb,
                                                float2* roll) {
  // P.h, P.w, P.xt, P.y0 are wave-uniform: row offsets go to the scalar
  // offset of the buffer instructions, the per-lane offset is the lane.
  // y0 and pitch are made opaque per iteration so that the per-row offsets
  // are recomputed (a few scalar instructions) instead of being hoisted out
  // of the level loop, where they outnumber the scalar registers and were
  // spilled to vector-register lanes and read back row by row.
  const int h = P.h, w = P.w, hw = P.hw, xt = P.xt;
  int y0 = P.y0, pitch = P.pitch;
  asm volatile("" : "+s"(y0), "+s"(pitch));
  // per-lane values derived afresh every iteration rather than held in
  // registers across the level (the empty asm hides their invariance)
  int lane = P.lane;
  asm volatile("" : "+v"(lane));
  const int x = xt + lane;
  // halo loads
  const int ru = __mul24(max(y0 - 1, 0), w) + xt, rd = __mul24(min(y0 + RPT, h - 1), w) + xt;
  const float hux = ucur.f32(lane, ru), huy = ucur.f32(lane, hw + ru);
  const float hdx = ucur.f32(lane, rd), hdy = ucur.f32(lane, hw + rd);
  // lane k < 4 RPT: halo side k / (2 RPT) (0 left, 1 right), component
  // (k / RPT) & 1, row k % RPT; the left halo is the last column of the tile
  // to the left (at the grid's edge: this tile's own first column), the
  // right halo the first column of the tile to the right
  const int k = lane & (4 * RPT - 1);
  const int side = k / (2 * RPT), comp = (k / RPT) & 1, rk = k & (RPT - 1);
  int src = P.tile, src_side = side;
  if (side == 0 && P.tx > 0) src = P.tile - 1, src_side = 1;
  if (side == 1 && P.tx < P.ntx - 1) src = P.tile + 1, src_side = 0;
  const float hcol = ccur.f32(colx_index<RPT>(src, src_side, P.wave, comp, rk));
  const int sel = lane == kWave - 1 ? 2 * RPT : 0;   // lane 63 pulls the right column, the others the left

  // the state this iteration starts from
#pragma unroll
  for (int r = 0; r < RPT; ++r) roll[r * kWG] = make_float2(sx[r], sy[r]);

  // Rows are computed in order; R and the four taps of T for row r + kAhead
  // are loaded while row r is computed (scheduling barriers keep each row's
  // work in its own block, which bounds the registers in flight).
  constexpr int kAhead = RPT < 2 ? RPT : 2;
  float taps[RPT][4];
  float flx[RPT], fly[RPT], rr[RPT];   // float32 floors of the state (the cells)
  auto gather = [&](int r) {
    rr[r] = rb.f32(lane, __mul24(y0 + r, pitch) + xt);
    int ix, iy;
    flx[r] = floor_cell(sx[r], ix);
    fly[r] = floor_cell(sy[r], iy);
    // the cell clamped to [-1, w-1] x [-1, h-1], offset by the border: the
    // four taps are o, o + 1, o + pitch, o + pitch + 1
    const int o = __mul24(clamp0(y0 + r + iy + 1, h), pitch) + clamp0(x + ix + 1, w);
    taps[r][0] = tb.f32(o, 0);
    taps[r][1] = tb.f32(o, 1);
    taps[r][2] = tb.f32(o, pitch);
    taps[r][3] = tb.f32(o, pitch + 1);
  };
#pragma unroll
  for (int r = 0; r < kAhead; ++r) gather(r);
  __builtin_amdgcn_sched_barrier(0);

  double accR = 0.0, accG = 0.0;
  // c - u of a row is -(c - d) of the row above (both from the old state;
  // IEEE subtraction is antisymmetric, so the negation is exact)
  double nux = 0.0, nuy = 0.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (r + kAhead < RPT) gather(r + kAhead);
    const float ex = lane_pull(hcol, sel + r), ey = lane_pull(hcol, sel + RPT + r);
    const float lx = from_left(sx[r], ex), ly = from_left(sy[r], ey);
    const float rx = from_right(sx[r], ex), ry = from_right(sy[r], ey);
    const float dx = r == RPT - 1 ? hdx : sx[r + 1], dy = r == RPT - 1 ? hdy : sy[r + 1];
    const double cx = sx[r], cy = sy[r];
    const double uxd = r == 0 ? cx - (double)hux : -nux, uyd = r == 0 ? cy - (double)huy : -nuy;
    const double dxd = cx - (double)dx, dyd = cy - (double)dy;
    double gx, gy;
    pixel_eval_d(cx - (double)flx[r], cy - (double)fly[r], taps[r][0], taps[r][1], taps[r][2], taps[r][3], rr[r],
                 cx - (double)lx, cx - (double)rx, uxd, dxd, cy - (double)ly, cy - (double)ry, uyd, dyd, P.lam,
                 accR, accG, gx, gy);
    nux = dxd;
    nuy = dyd;
    sx[r] = gd_update<float>(cx, gx, P.tau);
    sy[r] = gd_update<float>(cy, gy, P.tau);
    // pin the row's results here: without this the compiler sinks the
    // energy and update arithmetic of all rows to the end of the iteration,
    // keeping every row's intermediates live at once
    asm volatile("" : "+v"(accR), "+v"(accG), "+v"(sx[r]), "+v"(sy[r]));
    __builtin_amdgcn_sched_barrier(0);
  }

  // halo-facing values of the new state: the first and last rows, and (lanes
  // 0 and 63) the tile's first and last columns
  {
    const int o = __mul24(y0, w) + xt;
    unext.st32(lane, o, sx[0]);
    unext.st32(lane, hw + o, sy[0]);
    if (RPT > 1) {
      const int q = __mul24(y0 + RPT - 1, w) + xt;
      unext.st32(lane, q, sx[RPT - 1]);
      unext.st32(lane, hw + q, sy[RPT - 1]);
    }
    store_columns<RPT>(P, sx, sy, cnext, lane);
  }
  return lane_energy(accR, accG, P.lam);
}

}  // namespace rs
