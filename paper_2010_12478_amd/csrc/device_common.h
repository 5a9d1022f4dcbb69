// Device helpers shared by the registration kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr int kWG = 256;        // threads of every tile workgroup (4 wavefronts)
constexpr int kWave = 64;
constexpr int kTileW = 64;      // a tile row is one wavefront wide
constexpr int kMaxLevels = 8;
constexpr int kRB = 2;          // rows per register batch in the sweep (solver instantiations with resident levels)
constexpr int kRBStream = 4;    // the same in the streaming-only solver instantiation and the plain sweep
constexpr int kSweepTiles = 64; // tile sums per workgroup synchronisation in the solver's sweep
constexpr int kMaxRPT = 16;     // rows per thread of a register-resident tile at most (tile height 64)

__host__ __device__ inline int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }
// clampi(v, 0, hi) as one v_med3_i32 (the compiler forms it only for
// immediate bounds); hi is wave-uniform.
__device__ __forceinline__ int clamp0(int v, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(v), "s"(hi));
  return r;
}

// clampi(v, -1, hi) as one v_med3_i32; hi is wave-uniform.
__device__ __forceinline__ int clampm1(int v, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, -1, %2" : "=v"(r) : "v"(v), "s"(hi));
  return r;
}

// XCD-aware order of a launch's blocks.  The hardware hands block L (in
// launch order) to XCD L % 8.  In every run of 8 * chunk consecutive work
// items, XCD x is given the chunk items [x * chunk, (x + 1) * chunk), so
// that neighbouring items (tiles sharing halo and gather cache lines) are
// worked on behind one L2 while the launch as a whole still sweeps the items
// in order; the items after the last full run keep their place.  A
// bijection of [0, total).
__device__ __forceinline__ int xcd_item(int L, int total, int chunk) {
  const int run = 8 * chunk;
  if (L >= total / run * run) return L;
  const int base = L / run * run, l = L - base;
  return base + (l & 7) * chunk + (l >> 3);
}

// Stopping rule of a level (relative energy decrease), shared by the device
// solver and the host loop of the plain path so both decide identically.
__host__ __device__ inline bool level_stops(double e_prev, double e, double rel_tol) {
  return (e_prev - e) <= rel_tol * e_prev;
}

// Cell of a displacement component: its float32 floor fl (exact), and the
// integer cell used to index taps, clamped to +-2^20 (NaN -> -2^20: the taps
// clamp to the image and the value stays NaN).  The in-cell fraction is
// u - fl formed in double, which is exact for every float32 u with
// |u| >= 2^-29; formed in float32 it is not (u + 1 rounds for most u in
// (-1, 0)).  All arithmetic of the kernels is double; stored data are float
// (or double in the float64 instantiations).
__device__ __forceinline__ float floor_cell(float u, int& c) {
  const float fl = floorf(u);
  c = (int)fminf(fmaxf(fl, -1048576.f), 1048576.f);
  return fl;
}
// floor_cell of a float32 value held in double: the same floor (exact in
// either precision) and the same cell for every finite u (the conversion
// saturates before the clamp; a NaN u gives cell 0 here, -2^20 there, and
// NaN arithmetic either way).
__device__ __forceinline__ double floor_cell_d(double u, int& c) {
  const double fl = floor(u);
  c = min(max((int)fl, -1048576), 1048576);
  return fl;
}
__device__ __forceinline__ void cell_of(float u, int& c, double& f) {
  const float fl = floor_cell(u, c);
  f = (double)u - (double)fl;
}
__device__ __forceinline__ void cell_of(double u, int& c, double& f) {
  const float fl = floor_cell((float)u, c);
  f = u - (double)fl;
}

// Bilinear sample of img [H][W] at (x0 + wx, y0 + wy) with edge-clamped taps,
// and its derivatives with respect to the sample position:
//   s = (1 - wy) ((1 - wx) i00 + wx i01) + wy ((1 - wx) i10 + wx i11),
// each product and sum one rounded float64 operation in that order (no
// contraction), here and in the value-only forms below.
template <typename S>
__device__ __forceinline__ void bilin(const S* __restrict__ img, int H, int W, int x0, int y0,
                                      double wx, double wy, double& s, double& dsx, double& dsy) {
#pragma clang fp contract(off)
  const int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
  const int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
  const double i00 = img[ya * W + xa], i01 = img[ya * W + xb];
  const double i10 = img[yb * W + xa], i11 = img[yb * W + xb];
  const double ox = 1.0 - wx, oy = 1.0 - wy;
  s = oy * (ox * i00 + wx * i01) + wy * (ox * i10 + wx * i11);
  dsx = oy * (i01 - i00) + wy * (i11 - i10);
  dsy = ox * (i10 - i00) + wx * (i11 - i01);
}

// Bilinear value from the four taps (the order of bilin_value).
__device__ __forceinline__ double bilin_taps(double i00, double i01, double i10, double i11, double wx, double wy) {
#pragma clang fp contract(off)
  const double ox = 1.0 - wx, oy = 1.0 - wy;
  return oy * (ox * i00 + wx * i01) + wy * (ox * i10 + wx * i11);
}

template <typename S>
__device__ __forceinline__ double bilin_value(const S* __restrict__ img, int H, int W, int x0, int y0,
                                              double wx, double wy) {
#pragma clang fp contract(off)
  const int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
  const int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
  const double ox = 1.0 - wx, oy = 1.0 - wy;
  return oy * (ox * (double)img[ya * W + xa] + wx * (double)img[ya * W + xb]) +
         wy * (ox * (double)img[yb * W + xa] + wx * (double)img[yb * W + xb]);
}

// Loads of data that other workgroups of the same launch write (displacement
// fields, per-tile energies) go through a buffer descriptor with the
// device-scope policy (sc1): they miss the CU's L1 but allocate in and hit the
// XCD's L2, so no stale L1 line is returned once the writer's stores have
// reached that L2 (measured on gfx950: loads with the default or workgroup
// policy return stale lines; sc1 or nontemporal loads do not, and
// nontemporal ones also stop the line from staying in L2).  The base pointer
// must be uniform across the wavefront: it is moved to scalar registers from
// lane 0.
constexpr int kAuxSC1 = 16;

// A pointer every lane of the wavefront holds, moved to scalar registers.
__device__ __forceinline__ void* uniform_ptr(const void* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (void*)(((uint64_t)hi << 32) | lo);
}

// A double every lane of the wavefront holds, moved to scalar registers.
__device__ __forceinline__ double uniform_f64(double x) {
  const uint64_t v = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Buffer descriptor over a wave-uniform base: 32-bit element offsets keep the
// per-lane address arithmetic in one register.  AUX is the cache policy
// (0: default, kAuxSC1: miss the L1, see above).
template <int AUX>
struct BufView {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ explicit BufView(const void* base)
      : r(__builtin_amdgcn_make_buffer_rsrc(uniform_ptr(base), 0, -1, 0x00020000)) {}
  __device__ __forceinline__ float f32(int i) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, AUX));
  }
  __device__ __forceinline__ double f64(int i) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8, 0, AUX));
  }
  template <typename S>
  __device__ __forceinline__ S load(int i) const {
    if constexpr (sizeof(S) == 4) return f32(i); else return f64(i);
  }
  // element v (per lane) + s (wave-uniform, added in the scalar offset)
  __device__ __forceinline__ float f32(int v, int s) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v * 4, s * 4, AUX));
  }
  __device__ __forceinline__ double f64(int v, int s) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v * 8, s * 8, AUX));
  }
  template <typename S>
  __device__ __forceinline__ S load(int v, int s) const {
    if constexpr (sizeof(S) == 4) return f32(v, s); else return f64(v, s);
  }
  // elements v and v + 1 (per lane) + s (wave-uniform) in one load
  template <typename S>
  __device__ __forceinline__ void load2(int v, int s, S& a, S& b) const {
    if constexpr (sizeof(S) == 4) {
      const auto p = __builtin_bit_cast(unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(r, v * 4, s * 4, AUX));
      a = __builtin_bit_cast(float, (unsigned)p);
      b = __builtin_bit_cast(float, (unsigned)(p >> 32));
    } else {
      struct D2 {
        double a, b;
      };
      const D2 p = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(r, v * 8, s * 8, AUX));
      a = p.a;
      b = p.b;
    }
  }
  __device__ __forceinline__ void st32(int v, int s, float x) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, x), r, v * 4, s * 4, 0);
  }
  template <typename S>
  __device__ __forceinline__ void store(int v, int s, S x) const {
    if constexpr (sizeof(S) == 4) {
      st32(v, s, x);
    } else {
      typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v * 8, s * 8, 0);
    }
  }
};
using SharedBuf = BufView<kAuxSC1>;   // data written by other workgroups of the launch
using ReadBuf = BufView<0>;           // data no one writes during the launch

// Bilinear value of a shared field (see SharedBuf) with clamped taps.
__device__ __forceinline__ double bilin_value_shared(const SharedBuf& img, int H, int W, int x0, int y0,
                                                     double wx, double wy) {
#pragma clang fp contract(off)
  const int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
  const int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
  const double ox = 1.0 - wx, oy = 1.0 - wy;
  return oy * (ox * (double)img.f32(ya * W + xa) + wx * (double)img.f32(ya * W + xb)) +
         wy * (ox * (double)img.f32(yb * W + xa) + wx * (double)img.f32(yb * W + xb));
}

// Whole-wavefront shift by one lane (DPP wave_shr:1 / wave_shl:1): lane i
// receives v from lane i - 1 (from_left) or i + 1 (from_right); the lane
// without a source (0, respectively 63) keeps its own `edge`.
template <int CTRL>
__device__ __forceinline__ float wave_shift(float v, float edge) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                               __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ int wave_shift(int v, int edge) {
  return __builtin_amdgcn_update_dpp(edge, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v, double edge) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned long long e = __builtin_bit_cast(unsigned long long, edge);
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)e, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(e >> 32), (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf,
                                             false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <typename S>
__device__ __forceinline__ S wave_from_left(S v, S edge) { return wave_shift<0x138>(v, edge); }
template <typename S>
__device__ __forceinline__ S wave_from_right(S v, S edge) { return wave_shift<0x130>(v, edge); }

// A double moved across lanes by one DPP pattern (both halves); lanes with
// no source, or outside the row / bank masks, receive 0.
template <int CTRL, int ROW, int BANK>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW, BANK, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW, BANK, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Order-fixed sum over the 64 lanes of a wavefront, returned to every lane:
// a prefix tree inside each 16-lane row (row_shr 1, 2, 4, 8), then the rows
// through row_bcast 15 and 31, the total ending in lane 63.  DPP moves stay
// in the VALU (no LDS round trip per step).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0x111, 0xf, 0xf>(v);   // row_shr:1
  v += dpp_f64<0x112, 0xf, 0xf>(v);   // row_shr:2
  v += dpp_f64<0x114, 0xf, 0xe>(v);   // row_shr:4, banks 1-3
  v += dpp_f64<0x118, 0xf, 0xc>(v);   // row_shr:8, banks 2-3
  v += dpp_f64<0x142, 0xa, 0xf>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc, 0xf>(v);   // row_bcast:31 into rows 2 and 3
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, 63);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Canonical order-fixed sum of n doubles by one wavefront: lane l adds
// p[l], p[l+64], ... in sequence, then wave_sum.  Used for every
// per-tile energy total so that all execution paths agree bitwise.
__device__ __forceinline__ double wave_sum_array(const double* p, int n, int lane) {
  const SharedBuf buf(p);
  double acc = 0.0;
  for (int i = lane; i < n; i += kWave) acc += buf.f64(i);
  return wave_sum(acc);
}

// Block-wide order-fixed sum of one double per thread (kWG threads); the
// result is valid in thread 0.  `red` is __shared__ double[kWG / kWave].
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kWG / kWave; ++w) t += red[w];
  }
  __syncthreads();
  return t;
}

}  // namespace rs
