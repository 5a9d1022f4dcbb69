// Batched registration solver: a persistent kernel fed by a device atomic work
// queue, and the kernels of the plain one-launch-per-iteration path.
//
// Dataflow mode runs a whole series in one launch: a group's leader draws
// the next slot of a device ready queue; a finished task publishes its output
// (agent-scope release) and releases each consumer whose last missing input
// it was.  Groups that finish early draw the next ready registration, wherever
// it sits in the scan: imbalance between registrations is absorbed across the
// whole plan, not only within a level.
//
// Persistent kernel.  The grid is sized to be fully resident.  Workgroups form
// groups of g (same blockIdx % 8, so a group shares one XCD and its L2); a
// group takes registrations from an atomic ticket counter one at a time and
// runs each through all pyramid levels: initial guess on the coarsest level,
// then per level the gradient-descent sweeps, each followed by a group
// barrier, an order-fixed sum of the per-tile energies and the stopping
// decision, which every member takes identically.  A level's tiles are dealt
// round-robin to the g members.  Groups that finish early take the next
// ticket: the on-chip counterpart of the paper's work stealing (Section 4.3),
// absorbing the uneven iteration counts of the registrations.
//
// Every energy is a per-tile double sum (fixed order inside the tile) followed
// by the canonical wave sum over tiles, so the plain path, the persistent
// kernel at any group size, and repeated runs agree bitwise.
#include "internal.h"
#include "resident.h"
#include "sweep.h"

namespace rs {

namespace {

__device__ __forceinline__ int ld_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Group {
  int g, member, id;
  int* arrive;   // [g] epoch each member has reached (one word per member)
  int* task;     // [2] ticket broadcast
  int* xcc;      // [g] XCC id of every member
  int epoch;
  bool local;    // every member runs on the same XCD (verified at launch)
};

__device__ __forceinline__ int xcc_id() {
  return __builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11));   // HW_REG_XCC_ID[3:0]
}

// Barrier over the g workgroups of a group.  Returns false if the run has been
// aborted (by this or another workgroup's watchdog); all workgroups then leave.
//
// When all members share one XCD (G.local) they also share its L2, and since
// the vector L1 is write-through, a member's stores are visible to the others
// once they have completed (vmcnt 0), provided every read of such data misses
// the reader's L1 (SharedBuf): neither the L2 write-back of an agent-scope
// release nor the L1/L2 invalidation of an agent-scope acquire is needed, so
// the XCD's L2 keeps the frames and fields between iterations.  (Measured on
// gfx950: the workgroup-scope invalidate, buffer_inv sc0, leaves another CU's
// stale L1 lines in place; sc1 loads do not return them.)  Otherwise
// the agent-scope release and acquire make the data coherent across XCDs.
__device__ bool group_sync(Group& G, int* abort_flag, unsigned spin_limit, int* s_flag) {
  if (G.g == 1) {
    __syncthreads();
    return true;
  }
  if (G.local)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  else
    __threadfence();
  __syncthreads();
  G.epoch += 1;
  if (threadIdx.x < kWave) {   // wavefront 0 announces arrival and polls every member's word
    const int lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_store(&G.arrive[G.member], G.epoch, G.local ? __ATOMIC_RELAXED : __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      const int v0 = lane < G.g ? ld_relaxed(&G.arrive[lane]) : G.epoch;
      const int v1 = lane + kWave < G.g ? ld_relaxed(&G.arrive[lane + kWave]) : G.epoch;
      const int abort = ld_relaxed(abort_flag);   // in the same round trip
      if (__all(min(v0, v1) >= G.epoch)) break;
      if (abort) {
        ok = 0;
        break;
      }
      if (++spins > spin_limit) {
        if (lane == 0) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) *s_flag = ok;
  }
  __syncthreads();
  if (!G.local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *s_flag != 0;
}

// Barrier of the resident loop that also carries the energies.  Member m
// publishes its tile energy (0 for idle members) in slot m of the
// iteration's buffer, once the stores of all its wavefronts to shared data
// are complete; its wavefront 0 waits until all g slots are filled and forms
// the level energy in the canonical order (the tiles 0 .. nt-1 summed as in
// wave_sum_array), which it passes to the other wavefronts through LDS.
//
// The slots rotate over three buffers.  At the start of iteration t a member
// empties its slot of buffer (t + 1) % 3, last filled in t - 2 and read by
// every member before it published in t - 1 (which this member has seen);
// that store completes before the member publishes in t, so no member polling
// in t + 1 can mistake the value of t - 2 for a new one.
constexpr unsigned long long kSlotEmpty = ~0ull;   // a NaN no arithmetic produces

// Called by all threads with this thread's energy sum `acc`; returns false
// if the run was aborted, otherwise E is the level energy.
__device__ bool energy_barrier(const Group& G, unsigned long long* cur, double acc, bool active, int nt,
                               int* abort_flag, unsigned spin_limit, double* red, double* s_E, int* s_flag,
                               double& E) {
  const int lane = threadIdx.x & (kWave - 1);
  const double wp = wave_sum(acc);
  if (G.local)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  else
    __threadfence();
  if (lane == 0) red[threadIdx.x >> 6] = wp;
  __syncthreads();
  if (threadIdx.x < kWave) {
    if (lane == 0) {
      double t = 0.0;   // the order of block_sum
#pragma unroll
      for (int w = 0; w < kWG / kWave; ++w) t += red[w];
      __hip_atomic_store(cur + G.member, __builtin_bit_cast(unsigned long long, active ? t : 0.0),
                         G.local ? __ATOMIC_RELAXED : __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    const bool t0 = lane < G.g, t1 = lane + kWave < G.g;
    unsigned long long v0, v1;
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      v0 = t0 ? __hip_atomic_load(cur + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
      v1 = t1 ? __hip_atomic_load(cur + lane + kWave, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
      const int abort = ld_relaxed(abort_flag);   // in the same round trip
      if (__all(v0 != kSlotEmpty && v1 != kSlotEmpty)) break;
      if (abort) {
        ok = 0;
        break;
      }
      if (++spins > spin_limit) {
        if (lane == 0) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    double sum = 0.0;
    if (lane < nt) sum += __builtin_bit_cast(double, v0);
    if (lane + kWave < nt) sum += __builtin_bit_cast(double, v1);
    sum = wave_sum(sum);
    if (lane == 0) {
      *s_E = sum;
      *s_flag = ok;
    }
  }
  __syncthreads();
  if (!G.local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  E = *s_E;
  return *s_flag != 0;
}

// One pyramid level with the field resident in registers (see resident.h):
// member m owns tile m (members beyond the tile count only take part in the
// barriers).  U0 holds the level's initial field and receives its result
// (whole); U1 is the second halo buffer; roll is the LDS copy of the state an
// iteration starts from (kWG * RPT float2).  Returns false on abort;
// otherwise `iters` is the number of updates kept and `nonfinite` tells
// whether an energy was not finite (then U0 is left as it is).
template <int RPT>
__device__ bool level_resident(const SolveArgs& a, const LevelView<float>& V, float* U0, float* U1, float* slot, Group& G,
                               double* part, int& par, double* red, double* s_E, int* s_flag, float2* roll,
                               int& iters, bool& nonfinite) {
  int* abort_flag = a.ctrl + 1;
  constexpr int th = 4 * RPT;
  const int h = V.h, w = V.w;
  const int ntx = w / kTileW;
  const int nt = ntx * (h / th);
  const bool active = G.member < nt;
  const int tile = active ? G.member : 0;
  ResidentTile P;
  P.h = h;
  P.w = w;
  P.hw = h * w;
  P.lane = threadIdx.x & (kWave - 1);
  P.xt = (tile % ntx) * kTileW;
  P.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  P.y0 = (tile / ntx) * th + P.wave * RPT;
  P.tile = tile;
  P.tx = tile % ntx;
  P.ntx = ntx;
  P.tau = V.tau;
  P.lam = V.lam;
  P.pitch = V.pitch;
  const ReadBuf tb(V.T - V.pitch - 1), rb(V.R);   // T from its border element (-1, -1)
  float sx[RPT], sy[RPT];
  float* colx0 = slot + a.colx_off;
  float* colx1 = colx0 + a.colx_stride;
  {
    const SharedBuf u0(U0);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int o = __mul24(P.y0 + r, w) + P.xt + P.lane;
      sx[r] = active ? u0.f32(o) : 0.f;
      sy[r] = active ? u0.f32(P.hw + o) : 0.f;
    }
    // the initial field's tile columns for the first iteration (made
    // visible by the barrier below)
    if (active) store_columns<RPT>(P, sx, sy, ReadBuf(colx0), P.lane);
  }
  roll += threadIdx.x;
  // energy slots: three buffers of a.max_tiles (>= g) words, this member's
  // emptied before the first iteration
  unsigned long long* slots = (unsigned long long*)part;
  const size_t sbuf = (size_t)a.max_tiles;
  if (threadIdx.x < 3) slots[threadIdx.x * sbuf + G.member] = kSlotEmpty;
  if (!group_sync(G, abort_flag, a.spin_limit, s_flag)) return false;
  double e_prev = 0.0;
  int it = 0, eslot = 0;
  bool rollback = false;
  nonfinite = false;
  for (; it < a.max_iter; ++it) {
    const int nslot = eslot == 2 ? 0 : eslot + 1;
    if (threadIdx.x == 0)
      __hip_atomic_store(slots + nslot * sbuf + G.member, kSlotEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool odd = it & 1;
    const SharedBuf ucur(odd ? U1 : U0), ccur(odd ? colx1 : colx0);
    const ReadBuf unext(odd ? U0 : U1), cnext(odd ? colx0 : colx1);
    const double acc = active ? resident_step<RPT>(P, sx, sy, ucur, unext, ccur, cnext, tb, rb, roll) : 0.0;
    double E;
    if (!energy_barrier(G, slots + eslot * sbuf, acc, active, nt, abort_flag, a.spin_limit, red, s_E, s_flag, E))
      return false;
    eslot = nslot;
    if (!isfinite(E)) {
      nonfinite = true;
      break;
    }
    if (!a.fixed_iter && it > 0 && level_stops(e_prev, E, a.rel_tol)) {
      rollback = true;
      break;
    }
    e_prev = E;
  }
  iters = it;
  if (!nonfinite && active) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if (rollback) {
        const float2 v = roll[r * kWG];
        sx[r] = v.x;
        sy[r] = v.y;
      }
      const int o = __mul24(P.y0 + r, w) + P.xt + P.lane;
      U0[o] = sx[r];
      U0[P.hw + o] = sy[r];
    }
  }
  return true;
}

__device__ __forceinline__ float* start_buffer(const SolveArgs& a, const TaskDesc& d, float* slot, int l) {
  return l == 0 ? d.out : slot + a.lvl_off[l];
}

// Runs one registration with the calling group.  Returns false on abort.
// RES: levels that fit the group may run register-resident (otherwise every
// level streams, and the resident code is not compiled in).
template <bool RES>
__device__ __forceinline__ bool run_task(const SolveArgs& a, const TaskDesc& d, Group& G, float* slot, double* part, int& par,
                         double* red, double* s_E, int* s_flag, float2* roll) {
  int* abort_flag = a.ctrl + 1;
  const int L = a.levels;
  const int stride = G.g * kWG;
  const int first = G.member * kWG + threadIdx.x;

  {  // initial guess on the coarsest level
    const int hc = a.H >> (L - 1), wc = a.W >> (L - 1);
    float* dst = start_buffer(a, d, slot, L - 1);
    const int n = hc * wc;
    for (int p = first; p < n; p += stride) {
      const int Y = p / wc, X = p - Y * wc;
      double vx, vy;
      init_pixel<float>(d.kind, d.ua, d.ub, a.H, a.W, L, X, Y, vx, vy);
      dst[p] = (float)vx;
      dst[(size_t)n + p] = (float)vy;
    }
  }
  if (!group_sync(G, abort_flag, a.spin_limit, s_flag)) return false;

  float* bufB = slot + a.bufB_off;
  float* cur = start_buffer(a, d, slot, L - 1);
  int status = 0;
  int iters[kMaxLevels];
  bool dead = false;
  for (int l = L - 1; l >= 0; --l) {
    iters[l] = 0;
    if (dead) continue;
    const int h = a.H >> l, w = a.W >> l;
    const int n = h * w;
    if (l < L - 1) {
      float* dst = start_buffer(a, d, slot, l);
      for (int p = first; p < n; p += stride) {
        const int y = p / w, x = p - y * w;
        double vx, vy;
        prolong_pixel<true>(cur, h >> 1, w >> 1, x, y, vx, vy);
        dst[p] = (float)vx;
        dst[(size_t)n + p] = (float)vy;
      }
      if (!group_sync(G, abort_flag, a.spin_limit, s_flag)) return false;
      cur = dst;
    }
    LevelView<float> V;
    V.R = a.pyr[l] + (size_t)d.ref * a.fstride[l];
    V.T = a.pyr[l] + (size_t)d.tmpl * a.fstride[l];
    V.h = h;
    V.w = w;
    V.pitch = a.pitch[l];
    V.tau = a.tau;
    V.lam = a.lam;
    const int th = a.thl[l];
    const int nt = tiles_of(h, w, th);
    if (RES && a.resident && w % kTileW == 0 && h % th == 0 && nt <= G.g && th <= 4 * kMaxRPT &&
        (th & (th - 1)) == 0) {
      int it = 0;
      bool nf = false, ok = true;
      if (th == 4) ok = level_resident<1>(a, V, cur, bufB, slot, G, part, par, red, s_E, s_flag, roll, it, nf);
      else if (th == 8) ok = level_resident<2>(a, V, cur, bufB, slot, G, part, par, red, s_E, s_flag, roll, it, nf);
      else if (th == 16) ok = level_resident<4>(a, V, cur, bufB, slot, G, part, par, red, s_E, s_flag, roll, it, nf);
      else if (th == 32) ok = level_resident<8>(a, V, cur, bufB, slot, G, part, par, red, s_E, s_flag, roll, it, nf);
      else ok = level_resident<16>(a, V, cur, bufB, slot, G, part, par, red, s_E, s_flag, roll, it, nf);
      if (!ok) return false;
      iters[l] = it;
      if (nf) {
        status |= 2;   // REG_S_NONFINITE
        dead = true;
      } else if (!group_sync(G, abort_flag, a.spin_limit, s_flag)) {   // the result is read whole next
        return false;
      }
      if (it == a.max_iter && !a.fixed_iter) status |= 1;   // REG_S_MAXITER
      continue;
    }
    const int ths = stream_tile_rows(th, h, w, kMaxGroup);
    const int nts = tiles_of(h, w, ths);   // <= nt: the energy slots suffice
    float* other = bufB;
    double e_prev = 0.0;
    int it = 0;
    for (; it < a.max_iter; ++it) {
      V.u = cur;
      V.out = other;
      double* pp = part + (size_t)par * a.max_tiles;
      sweep_tiles<float, SW_UPDATE, false, true, RES ? kRB : kRBStream, kSweepTiles, !RES>(V, G.member, G.g, ths,
                                                                                           red, pp, nullptr);
      if (!group_sync(G, abort_flag, a.spin_limit, s_flag)) return false;
      if (threadIdx.x < kWave) {
        const double E = wave_sum_array(pp, nts, threadIdx.x);
        if (threadIdx.x == 0) *s_E = E;
      }
      __syncthreads();
      const double E = *s_E;
      par ^= 1;
      if (!isfinite(E)) {
        status |= 2;   // REG_S_NONFINITE
        dead = true;
        break;
      }
      if (!a.fixed_iter && it > 0 && level_stops(e_prev, E, a.rel_tol)) break;
      e_prev = E;
      float* t = cur;
      cur = other;
      other = t;
    }
    iters[l] = it;
    if (it == a.max_iter && !a.fixed_iter) status |= 1;   // REG_S_MAXITER
  }

  const size_t nf = (size_t)2 * a.H * a.W;
  if (dead) {
    for (size_t p = first; p < nf; p += stride) d.out[p] = __builtin_nanf("");
  } else if (cur != d.out) {
    const SharedBuf src(cur);
    for (size_t p = first; p < nf; p += stride) d.out[p] = src.f32((int)p);
  }
  if (G.member == 0 && threadIdx.x == 0) {
    if (d.iters)
      for (int l = 0; l < L; ++l) d.iters[l] = iters[l];
    if (d.status) *d.status = status;
  }
  return true;
}

// Next task for the calling group's leader.  Batched: the next ticket of the
// work queue (>= n_tasks: none left).  Dataflow: the next ready-queue slot,
// waiting until a finished task has filled it (n_tasks once all are drawn).
__device__ int next_task(const SolveArgs& a, int* queue, int* abort_flag) {
  if (!a.dataflow) return atomicAdd(queue, 1);
  const int pos = __hip_atomic_fetch_add(&a.ctrl[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (pos >= a.n_tasks) return a.n_tasks;
  unsigned spins = 0;
  for (;;) {
    const int t = ld_relaxed(&a.ready[pos]);
    if (t >= 0) return t;
    if (ld_relaxed(abort_flag)) return a.n_tasks;
    if (++spins > a.spin_limit) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return a.n_tasks;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

static_assert(sizeof(TaskDesc) == 56, "TaskDesc is broadcast as 7 words");

// Phase 1 with flexible segment boundaries (Algorithm 1, Section 4.3) for
// group w = worker w.  The leader (member 0, thread 0) keeps the worker's
// state: the segment [pl, pr] it has absorbed and where its running result
// lies.  Worker 0 starts at element 0 and only moves right (its partial
// results are the prefixes, written to phi0); the last worker starts at the
// last element and only moves left; the others start in the middle of their
// static segment.  After one step to the right a worker extends toward the
// neighbour whose time per registration is larger (ties: right), or toward
// the only side with unclaimed elements; it claims the element next to its
// segment from the gap (one 64-bit word (lo, hi) per pair of neighbours,
// compare-and-swap) and the group runs B(res, x_e) or B(x_e, res).  The leader
// broadcasts each registration's descriptor through agent-scope atomics; the
// members read it after the group barrier and invalidate their L1 before
// reading fields another step of the group wrote.
__device__ int flex_claim(unsigned long long* gaps, int gi, bool from_left) {
  unsigned long long g = __hip_atomic_load(gaps + gi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const int lo = (int)(g & 0xffffffffu), hi = (int)(g >> 32);
    if (lo > hi) return -1;
    const unsigned long long nw = from_left ? (unsigned long long)(unsigned)(lo + 1) | ((unsigned long long)(unsigned)hi << 32)
                                            : (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)(hi - 1) << 32);
    if (__hip_atomic_compare_exchange_strong(gaps + gi, &g, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return from_left ? lo : hi;
  }
}

__device__ __forceinline__ int flex_gap_size(const unsigned long long* gaps, int gi) {
  const unsigned long long g =
      __hip_atomic_load((unsigned long long*)gaps + gi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (int)(g >> 32) - (int)(g & 0xffffffffu) + 1;
}

// State a flexible-segment worker's leader keeps between registrations.
struct FlexState {
  int pl, pr, ops;
  unsigned long long t0;
};

// The next registration of worker w = G.id (see flex_claim): the leader picks
// the direction, claims the element and publishes the descriptor and a
// command word; after the group barrier every thread reads them back.
// Returns 1 with *d filled, 0 when the worker's gaps are empty, -1 on abort.
__device__ int flex_next(const SolveArgs& a, Group& G, FlexState& F, TaskDesc& d, int* s_flag,
                         unsigned long long* s_desc) {
  int* abort_flag = a.ctrl + 1;
  const int w = G.id, P = a.flex_workers;
  const size_t nf = (size_t)2 * a.H * a.W;
  unsigned long long* desc = a.flex_desc + (size_t)w * 8;
  if (G.member == 0 && threadIdx.x == 0) {
    int e = -1;
    bool right = true;
    for (;;) {
      const int sL = w > 0 ? flex_gap_size(a.gaps, w - 1) : 0;
      const int sR = w < P - 1 ? flex_gap_size(a.gaps, w) : 0;
      if (sL <= 0 && sR <= 0) break;
      if (F.ops == 0 && sR > 0) right = true;
      else if (sL > 0 && sR > 0)
        right = !(__hip_atomic_load(a.rates + w - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >
                  __hip_atomic_load(a.rates + w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      else right = sL <= 0;
      e = right ? flex_claim(a.gaps, w, true) : flex_claim(a.gaps, w - 1, false);
      if (e >= 0) break;
    }
    unsigned long long cmd = 0;
    if (e >= 0) {
      cmd = 1;
      const float* res = F.ops == 0 ? a.elem + (size_t)a.starts[w] * nf
                         : w == 0   ? a.phi0 + (size_t)F.pr * nf
                                    : a.flex_buf + ((size_t)w * 2 + ((F.ops - 1) & 1)) * nf;
      const float* el = a.elem + (size_t)e * nf;
      float* out = w == 0 ? a.phi0 + (size_t)e * nf : a.flex_buf + ((size_t)w * 2 + (F.ops & 1)) * nf;
      const int ref = right ? F.pl : e, tmpl = right ? e + 1 : F.pr + 1;
      const unsigned long long words[7] = {
          (unsigned long long)(unsigned)ref | ((unsigned long long)(unsigned)tmpl << 32),
          1ull,   // kind 1: composition of ua and ub
          (unsigned long long)(right ? res : el),
          (unsigned long long)(right ? el : res),
          (unsigned long long)out,
          (unsigned long long)(a.elem_iters + (size_t)e * a.levels),
          (unsigned long long)(a.elem_status + e)};
#pragma unroll
      for (int q = 0; q < 7; ++q) __hip_atomic_store(desc + q, words[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a.elem_step[e] = F.ops + 1;
      if (right) F.pr = e;
      else F.pl = e;
    }
    __hip_atomic_store(desc + 7, cmd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!group_sync(G, abort_flag, a.spin_limit, s_flag)) return -1;
  if (threadIdx.x < 8) s_desc[threadIdx.x] = __hip_atomic_load(desc + threadIdx.x, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (s_desc[7] == 0) return 0;
  d.ref = (int)(s_desc[0] & 0xffffffffu);
  d.tmpl = (int)(s_desc[0] >> 32);
  d.kind = 1;
  d.pad = 0;
  d.ua = (const float*)s_desc[2];
  d.ub = (const float*)s_desc[3];
  d.out = (float*)s_desc[4];
  d.iters = (int32_t*)s_desc[5];
  d.status = (int32_t*)s_desc[6];
  __syncthreads();
  // the running result was written by this group's previous registration
  // through other CUs' L1s: drop stale lines before reading it
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return 1;
}

// FLEX: the flexible-segment phase 1 (a separate instantiation, so that the
// other modes carry none of its state).  RES: with the register-resident
// levels; without them (a launch none of whose levels can run resident) the
// kernel needs no rollback copy in LDS and runs kStreamWaves waves per SIMD,
// whose registers its sweep's 4-row batches take without spilling.
template <bool FLEX, bool RES>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(RES ? 4 : kStreamWaves)))
k_persistent(SolveArgs a) {
  __shared__ double red[sweep_red_doubles<false>(kSweepTiles)];
  __shared__ double s_E;
  __shared__ int s_flag;
  __shared__ int s_task;
  __shared__ float2 roll[RES ? kWG * kMaxRPT : 1];
  const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3;
  Group G;
  G.g = a.g;
  G.member = lb % a.g;
  G.id = (lb / a.g) * 8 + xcd;
  int* gctl = a.ctrl + kCtrlHead + kCtrlGroup * G.id;
  G.arrive = gctl;
  G.task = gctl + kMaxGroup;
  G.xcc = gctl + 2 * kMaxGroup;
  G.epoch = 0;
  G.local = false;
  int* queue = a.ctrl;
  int* abort_flag = a.ctrl + 1;
  double* part = a.part + (size_t)G.id * 3 * a.max_tiles;
  float* slot = a.ws + (size_t)G.id * a.slot_floats;
  int par = 0, tpar = 0;

  // Control words are written and read with agent-scope atomics only, so they
  // are coherent whatever the barrier flavour (the data buffers are not).
  if (threadIdx.x == 0) __hip_atomic_store(&G.xcc[G.member], xcc_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (G.member == 0 && threadIdx.x == 0)
    __hip_atomic_store(&G.task[0], next_task(a, queue, abort_flag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!group_sync(G, abort_flag, a.spin_limit, &s_flag)) return;   // agent scope: always coherent
  if (G.g > 1) {
    if (threadIdx.x == 0) {
      int same = 1;
      const int mine = __hip_atomic_load(&G.xcc[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int m = 1; m < G.g; ++m)
        same &= __hip_atomic_load(&G.xcc[m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == mine;
      s_task = same;
    }
    __syncthreads();
    G.local = s_task != 0;
    __syncthreads();
  }
  FlexState F{0, 0, 0, 0};
  __shared__ unsigned long long s_desc[8];
  if constexpr (FLEX) {
    if (G.id >= a.flex_workers) return;   // groups come in multiples of 8: the surplus has no segment
    F.pl = F.pr = a.starts[G.id];
    if (G.member == 0 && threadIdx.x == 0) F.t0 = wall_clock64();
  }
  for (;;) {
    TaskDesc d;
    int t = 0;
    if constexpr (FLEX) {
      const int r = flex_next(a, G, F, d, &s_flag, s_desc);
      if (r < 0) return;
      if (r == 0) break;
    } else {
      if (threadIdx.x == 0) s_task = ld_relaxed(&G.task[tpar]);
      __syncthreads();
      t = s_task;
      if (t >= a.n_tasks) break;
      // dataflow: the inputs were written by other groups, possibly on other
      // XCDs, and published with an agent-scope release
      if (a.dataflow) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      d = a.tasks[t];
    }
    if (!run_task<RES>(a, d, G, slot, part, par, red, &s_E, &s_flag, roll)) return;
    if constexpr (FLEX) {
      if (!group_sync(G, abort_flag, a.spin_limit, &s_flag)) return;
      if (G.member == 0 && threadIdx.x == 0) {
        ++F.ops;
        const float r = (float)((double)(wall_clock64() - F.t0) / F.ops);
        __hip_atomic_store(a.rates + G.id, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      continue;
    }
    tpar ^= 1;
    if (a.dataflow) {
      // publish this task's output device-wide, then (leader) release its
      // consumers whose last input it was
      __threadfence();
      if (!group_sync(G, abort_flag, a.spin_limit, &s_flag)) return;
      if (G.member == 0 && threadIdx.x == 0) {
        for (int q = a.cons_off[t]; q < a.cons_off[t + 1]; ++q) {
          const int c = a.cons[q];
          if (__hip_atomic_fetch_add(&a.deps[c], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1) {
            const int pos = __hip_atomic_fetch_add(&a.ctrl[3], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.ready[pos], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
    }
    if (G.member == 0 && threadIdx.x == 0)
      __hip_atomic_store(&G.task[tpar], next_task(a, queue, abort_flag), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    if (!group_sync(G, abort_flag, a.spin_limit, &s_flag)) return;
  }
  if (FLEX && G.member == 0 && threadIdx.x == 0) {
    a.flex_seg[G.id * 4 + 0] = F.pl;
    a.flex_seg[G.id * 4 + 1] = F.pr;
    a.flex_seg[G.id * 4 + 2] = F.ops;
    a.flex_seg[G.id * 4 + 3] = 0;
  }
}

// ------------------------------------------------------- rigid operator

// theta of phi_jk o phi_ij about the common centre: angles add,
// G = Rot(alpha_jk) G_ij + G_jk.
__device__ __forceinline__ void rigid_compose(const double* t1, const double* t2, double* out) {
#pragma clang fp contract(off)
  const double c = cos(t2[0]), s = sin(t2[0]);
  out[0] = t1[0] + t2[0];
  out[1] = c * t1[1] - s * t1[2] + t2[1];
  out[2] = s * t1[1] + c * t1[2] + t2[2];
}

// Pixels of a rigid-operator pass.  The sample position phi(x) from the
// column terms (ca dx, sa dx) and the row's dy: p_x = (t1 + c_x) + G_x and
// p_y = (t2 + c_y) + G_y with t1 = ca dx - sa dy, t2 = sa dx + ca dy and
// dp/dalpha = (-t2, t1); at alpha = 0 the positions are formed exactly as the
// definition reads, so integer translations land on the same cells on every
// evaluation.  A pixel is taken in two steps so that a thread can have the
// loads of several pixels in flight: fetch (position, in-cell fraction, the
// two tap pairs of T and the value of R) and accumulate (the bilinear value
// and its derivatives from the shared tap differences -- b0, b1: the value
// interpolated along x on the cell's upper and lower row, dT/dy = b1 - b0 --,
// the angle derivative grad T . dphi/dalpha, and the 14 moment sums).
// Multiply-adds are fused (results agree with the definition-order
// evaluation to rounding).
struct RigidCol {
  double cadx, sadx, ca, sa, cx, cy, gx, gy;
  int x, w1, h1, pitch;
};
struct RigidSample {
  float i00, i01, i10, i11, av;
  double fx, fy;
};

// Row dy = y - c_y of the column; R at element ro (per lane) + so (uniform).
__device__ __forceinline__ void rigid_fetch(const ReadBuf& rb, const ReadBuf& tb, const RigidCol& c, double dy,
                                            int ro, int so, RigidSample& s) {
  const double t1 = c.cadx - c.sa * dy;
  const double t2 = c.sadx + c.ca * dy;
  const double px = (t1 + c.cx) + c.gx;
  const double py = (t2 + c.cy) + c.gy;
  const double fx0 = floor(px), fy0 = floor(py);
  s.fx = px - fx0;
  s.fy = py - fy0;
  // the cell clamped to [-1, w-1] x [-1, h-1], offset by the border (the
  // conversion saturates, so clamping the integer equals clamping the
  // double for every finite position; a NaN position gives NaN sums either way)
  const int cxi = clampm1((int)fx0, c.w1) + 1;
  const int cyi = clampm1((int)fy0, c.h1) + 1;
  const int o = __umul24((unsigned)cyi, (unsigned)c.pitch) + cxi;
  tb.load2<float>(o, 0, s.i00, s.i01);
  tb.load2<float>(o, c.pitch, s.i10, s.i11);
  s.av = rb.f32(ro, so);
}

// t1 and t2 are formed again rather than kept from the fetch: the registers
// of the batch in flight are worth more than the two multiply-adds.
__device__ __forceinline__ void rigid_accumulate(const RigidCol& c, double dy, const RigidSample& s, double* acc) {
  const double t1 = c.cadx - c.sa * dy;
  const double t2 = c.sadx + c.ca * dy;
  const double i00 = s.i00, i01 = s.i01, i10 = s.i10, i11 = s.i11, av = s.av;
  const double fx = s.fx, fy = s.fy;
  const double d0 = i01 - i00, d1 = i11 - i10;
  const double b0 = i00 + fx * d0, b1 = i10 + fx * d1;
  const double by = b1 - b0;
  const double b = b0 + fy * by;
  const double bx = d0 + fy * (d1 - d0);
  const double ga = by * t1 - bx * t2;
  acc[0] += av;
  acc[1] += b;
  acc[2] += av * av;
  acc[3] += b * b;
  acc[4] += av * b;
  acc[5] += ga;
  acc[6] += bx;
  acc[7] += by;
  acc[8] += av * ga;
  acc[9] += av * bx;
  acc[10] += av * by;
  acc[11] += b * ga;
  acc[12] += b * bx;
  acc[13] += b * by;
}

// One column's rows y0, y0 + rpi, ... < y1 in row order, in batches of
// kRigidBatch rows whose loads are issued while the previous batch is
// accumulated (the same loads on every path into a batch's accumulation, so
// the wait for its taps leaves the next batch's loads in flight; the last
// batch is peeled), then the rows left over one at a time.  Within a batch
// the rows differ by multiples of rpi: dy by exact additions, R's offset in
// the load's scalar offset.
constexpr int kRigidBatch = 2;   // two batches in flight fit 4 waves per SIMD without spills

__device__ __forceinline__ void rigid_column(const ReadBuf& rb, const ReadBuf& tb, const RigidCol& c, int y0,
                                             int y1, int rpi, double* acc) {
  constexpr int P = kRigidBatch;
  const int n = y0 < y1 ? (y1 - 1 - y0) / rpi + 1 : 0;
  const int nb = n / P, step = P * rpi;
  const int rstride = rpi * c.pitch;
  RigidSample A[P], B[P];
  auto fetch = [&](RigidSample* S, int y) {
    const double dy = y - c.cy;
    const int ro = __umul24((unsigned)y, (unsigned)c.pitch) + c.x;
#pragma unroll
    for (int j = 0; j < P; ++j) rigid_fetch(rb, tb, c, dy + (double)(j * rpi), ro, j * rstride, S[j]);
  };
  auto accumulate = [&](const RigidSample* S, int y) {
    const double dy = y - c.cy;
#pragma unroll
    for (int j = 0; j < P; ++j) rigid_accumulate(c, dy + (double)(j * rpi), S[j], acc);
  };
  int y = y0;
  if (nb > 0) {
    fetch(A, y);
    int b = 0;
    for (; b + 2 < nb; b += 2, y += 2 * step) {
      fetch(B, y + step);
      accumulate(A, y);
      fetch(A, y + 2 * step);
      accumulate(B, y + step);
    }
    if (b + 1 < nb) {
      fetch(B, y + step);
      accumulate(A, y);
      accumulate(B, y + step);
      y += 2 * step;
    } else {
      accumulate(A, y);
      y += step;
    }
  }
  for (; y < y1; y += rpi) {
    RigidSample s;
    const double dy = y - c.cy;
    rigid_fetch(rb, tb, c, dy, __umul24((unsigned)y, (unsigned)c.pitch) + c.x, 0, s);
    rigid_accumulate(c, dy, s, acc);
  }
}

// sin and cos of the angle, not inlined: inlined, the compiler hoists the
// polynomials' constants out of the iteration loop and then spills them
// (the pixel loop holds the registers), and every pass waited on their reloads.
__device__ __attribute__((noinline)) void rigid_sincos(double a, double* s, double* c) { sincos(a, s, c); }

// Next registration for the calling group's leader: the next ticket, or in
// dataflow mode the next ready-queue slot once a finished registration has
// filled it (n_tasks when none is left or the run was aborted).
__device__ int rigid_next(const RigidArgs& a, int* abort_flag) {
  if (!a.dataflow) return atomicAdd(a.ctrl, 1);
  const int pos = __hip_atomic_fetch_add(&a.ctrl[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (pos >= a.n_tasks) return a.n_tasks;
  unsigned spins = 0;
  for (;;) {
    const int t = ld_relaxed(&a.ready[pos]);
    if (t >= 0) return t;
    if (ld_relaxed(abort_flag)) return a.n_tasks;
    if (++spins > a.spin_limit) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return a.n_tasks;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Barrier of a rigid-operator pass that also carries the moment sums: member
// m stores its 14 sums in its slots of the pass's buffer ([member][16] u64,
// kSlotEmpty when not yet written), and wavefront 0 polls every member's
// slots until all are filled, then adds them in member order into s_sum.  The
// buffers rotate over three passes as in energy_barrier: at the start of pass
// t a member empties its slots of the buffer of pass t + 1, last filled in
// pass t - 2 and read by every member before it published in t - 1; that
// store lands before the member's pass-t sums do.  Called by all threads once
// the sums are stored; returns false if the run was aborted.
__device__ bool rigid_barrier(const Group& G, const unsigned long long* cur, int* abort_flag, unsigned spin_limit,
                              double* s_sum, int* s_flag) {
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    const bool mine = lane < kRigidSums;
    unsigned long long v[kRigidMaxGroup];
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      bool full = true;
      if (mine) {
#pragma unroll
        for (int m = 0; m < kRigidMaxGroup; ++m) {   // slots of members >= g exist and stay empty
          v[m] = __hip_atomic_load(cur + m * 16 + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          full &= (m >= G.g) | (v[m] != kSlotEmpty);
        }
      }
      const int abort = ld_relaxed(abort_flag);   // in the same round trip
      if (__all(full)) break;
      if (abort) {
        ok = 0;
        break;
      }
      if (++spins > spin_limit) {
        if (lane == 0) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (mine) {
      double sum = 0.0;
#pragma unroll
      for (int m = 0; m < kRigidMaxGroup; ++m)
        if (m < G.g) sum += __builtin_bit_cast(double, v[m]);
      s_sum[lane] = sum;
    }
    if (lane == 0) *s_flag = ok;
  }
  __syncthreads();
  if (!G.local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *s_flag != 0;
}

// Rigid registration with normalized cross-correlation (the paper's operator,
// Definition "Image registration problem", Section 2.3.1): phi(x) =
// Rot(alpha)(x - c) + c + G about the image centre c, E = 1 - NCC(R, T o phi),
// gradient flow in the metric diag(r^2, 1, 1) (r^2: mean squared pixel
// distance from c) on the padded pyramid, G halved per coarser level.  A
// group of g workgroups takes registrations from the ticket queue (or, in
// dataflow mode, from the ready queue that finished registrations fill); per
// iteration every member streams its rows once, accumulating in double the 14
// sums that give NCC and its gradient (sum a, b, a^2, b^2, ab and per
// parameter sum g_p, a g_p, b g_p, with g_p = grad T(phi(x)) . dphi/dtheta_p),
// publishes them, and after the group barrier every thread adds the members'
// sums in member order and takes the same step.  Threads own columns (a
// thread's column terms are computed once per iteration) and walk their rows
// in batches (rigid_column), so that a lone wavefront keeps loads in flight.
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4))) k_rigid(RigidArgs a) {
  __shared__ double tacc[kRigidSums][kWG + 16];   // row padding: 2-way bank use on the strided reads
  __shared__ double s_sum[16];
  __shared__ int s_flag, s_task;
  const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3;
  Group G;
  G.g = a.g;
  G.member = lb % a.g;
  G.id = (lb / a.g) * 8 + xcd;
  int* gctl = a.ctrl + kCtrlHead + kCtrlGroup * G.id;
  G.arrive = gctl;
  G.task = gctl + kMaxGroup;
  G.xcc = gctl + 2 * kMaxGroup;
  G.epoch = 0;
  G.local = false;
  int* abort_flag = a.ctrl + 1;
  unsigned long long* slots = (unsigned long long*)a.part + (size_t)G.id * 3 * kRigidSlotBuf;
  int tpar = 0, slot = 0;
  if (threadIdx.x == 0) __hip_atomic_store(&G.xcc[G.member], xcc_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (G.member == 0 && threadIdx.x == 0)
    __hip_atomic_store(&G.task[0], rigid_next(a, abort_flag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!group_sync(G, abort_flag, a.spin_limit, &s_flag)) return;   // agent scope: always coherent
  if (G.g > 1) {   // members on one XCD share its L2: the light barrier (see group_sync)
    if (threadIdx.x == 0) {
      int same = 1;
      const int mine = __hip_atomic_load(&G.xcc[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int m = 1; m < G.g; ++m)
        same &= __hip_atomic_load(&G.xcc[m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == mine;
      s_task = same;
    }
    __syncthreads();
    G.local = s_task != 0;
    __syncthreads();
  }
  for (;;) {
    if (threadIdx.x == 0) s_task = ld_relaxed(&G.task[tpar]);
    __syncthreads();
    // the registration's state is the same in every thread: kept in scalar
    // registers, so that the pixel loop has the vector registers
    const int t = __builtin_amdgcn_readfirstlane(s_task);
    if (t >= a.n_tasks) break;
    // dataflow: the inputs were written by other groups, possibly on other
    // XCDs, and published with an agent-scope release
    if (a.dataflow) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const RigidTask d = a.tasks[t];
    const int ref = __builtin_amdgcn_readfirstlane(d.ref), tmpl = __builtin_amdgcn_readfirstlane(d.tmpl);
    int32_t* const d_iters = (int32_t*)uniform_ptr(d.iters);
    const bool leader = G.member == 0 && threadIdx.x == 0;
    double th[3] = {0.0, 0.0, 0.0};
    if (d.kind == 1) rigid_compose(d.ta, d.tb, th);
    else if (d.kind == 2) th[0] = d.ta[0], th[1] = d.ta[1], th[2] = d.ta[2];
    const double down = (double)(1 << (a.levels - 1));
    th[0] = uniform_f64(th[0]);
    th[1] = uniform_f64(th[1] / down);
    th[2] = uniform_f64(th[2] / down);
    int status = 0;
    bool dead = false;
    for (int l = a.levels - 1; l >= 0; --l) {
      if (dead) {
        if (leader && d_iters) d_iters[l] = 0;
        continue;
      }
      if (l < a.levels - 1) {
        th[1] = 2.0 * th[1];
        th[2] = 2.0 * th[2];
      }
      const int h = a.H >> l, w = a.W >> l, pitch = a.pitch[l];
      const float* Rp = a.pyr[l] + (size_t)ref * a.fstride[l];
      const float* Tp = a.pyr[l] + (size_t)tmpl * a.fstride[l];
      const ReadBuf rb(Rp), tb(Tp - pitch - 1);   // T from its border element (-1, -1)
      const double r2 = uniform_f64(((double)w * w - 1.0 + ((double)h * h - 1.0)) / 12.0);
      const double cx = uniform_f64((w - 1) / 2.0), cy = uniform_f64((h - 1) / 2.0);
      const double n = uniform_f64((double)h * w);
      const int row0 = (int)((long long)G.member * h / a.g), row1 = (int)((long long)(G.member + 1) * h / a.g);
      // thread -> (column tx + k tw, rows ty, ty + rpi, ...) of the member's band
      const int tw = w < kWG ? w : kWG, rpi = kWG / tw;
      const int tx = threadIdx.x % tw, ty = threadIdx.x / tw;
      const int y_first = ty < rpi ? row0 + ty : row1;
      double e_prev = 0.0;
      int it = 0;
      for (; it < a.max_iter; ++it) {
        // empty this member's slots of the buffer after this pass's (see rigid_barrier)
        const int nslot = slot == 2 ? 0 : slot + 1;
        if (G.g > 1 && threadIdx.x < kRigidSums * 16 && (threadIdx.x & 15) == 15)
          __hip_atomic_store(slots + nslot * kRigidSlotBuf + G.member * 16 + (threadIdx.x >> 4), kSlotEmpty,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        double acc[kRigidSums];
#pragma unroll
        for (int j = 0; j < kRigidSums; ++j) acc[j] = 0.0;
        {
          double sa, ca;
          rigid_sincos(th[0], &sa, &ca);
          sa = uniform_f64(sa);
          ca = uniform_f64(ca);
          RigidCol c;
          c.ca = ca;
          c.sa = sa;
          c.cx = cx;
          c.cy = cy;
          c.gx = th[1];
          c.gy = th[2];
          c.w1 = w - 1;
          c.h1 = h - 1;
          c.pitch = pitch;
          for (int x = tx; x < w; x += tw) {
            const double dx = x - cx;
            c.x = x;
            c.cadx = ca * dx;
            c.sadx = sa * dx;
            rigid_column(rb, tb, c, y_first, row1, rpi, acc);
          }
        }
        // member partial sums through LDS: every thread's 14 sums, then the
        // 16 lanes of one DPP row per sum add 16 threads' values each (stride
        // 16) and the row's 16 partials (row_shr 1, 2, 4, 8: lane 15 holds
        // the member's sum)
#pragma unroll
        for (int j = 0; j < kRigidSums; ++j) tacc[j][threadIdx.x] = acc[j];
        __syncthreads();
        unsigned long long* cur = slots + slot * kRigidSlotBuf;
        if (threadIdx.x < kRigidSums * 16) {   // whole 16-lane rows
          const int j = threadIdx.x >> 4, q = threadIdx.x & 15;
          double v = 0.0;
#pragma unroll
          for (int k = 0; k < kWG / 16; ++k) v += tacc[j][q + 16 * k];
          v += dpp_f64<0x111, 0xf, 0xf>(v);
          v += dpp_f64<0x112, 0xf, 0xf>(v);
          v += dpp_f64<0x114, 0xf, 0xe>(v);
          v += dpp_f64<0x118, 0xf, 0xc>(v);
          if (q == 15) {
            if (G.g == 1) {
              s_sum[j] = 0.0 + v;   // the members' sum of a group of one
            } else {
              // the slot is this moment's arrival: the empty marker stored at
              // the start of the pass lands first
              if (G.local) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
              __hip_atomic_store(cur + G.member * 16 + j, __builtin_bit_cast(unsigned long long, v),
                                 G.local ? __ATOMIC_RELAXED : __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
        }
        if (G.g == 1) {
          __syncthreads();
        } else if (!rigid_barrier(G, cur, abort_flag, a.spin_limit, s_sum, &s_flag)) {
          return;
        }
        slot = nslot;
        double E, g0, g1, g2;
        {
#pragma clang fp contract(off)
          const double abar = s_sum[0] / n, bbar = s_sum[1] / n;
          const double saa = s_sum[2] - n * abar * abar, sbb = s_sum[3] - n * bbar * bbar;
          const double sab = s_sum[4] - n * abar * bbar;
          if (!(saa * sbb > 0.0)) {
            E = 1.0;
            g0 = g1 = g2 = 0.0;
          } else {
            // one reciprocal each for the two denominators (a division is a
            // long dependent sequence, and every iteration waits for these)
            const double den = sqrt(saa * sbb), ncc = sab / den;
            const double rden = 1.0 / den, q = ncc / sbb;
            E = 1.0 - ncc;
            g0 = -((s_sum[8] - abar * s_sum[5]) * rden - (s_sum[11] - bbar * s_sum[5]) * q);
            g1 = -((s_sum[9] - abar * s_sum[6]) * rden - (s_sum[12] - bbar * s_sum[6]) * q);
            g2 = -((s_sum[10] - abar * s_sum[7]) * rden - (s_sum[13] - bbar * s_sum[7]) * q);
          }
        }
        if (!isfinite(E)) {
          status |= 2;   // REG_S_NONFINITE
          dead = true;
          break;
        }
        if (!a.fixed_iter && it > 0 && level_stops(e_prev, E, a.rel_tol)) break;
        e_prev = E;
        {
#pragma clang fp contract(off)
          th[0] = uniform_f64(th[0] - a.tau * g0 / r2);
          th[1] = uniform_f64(th[1] - a.tau * g1);
          th[2] = uniform_f64(th[2] - a.tau * g2);
        }
      }
      if (leader && d_iters) d_iters[l] = it;
      if (it == a.max_iter && !a.fixed_iter) status |= 1;   // REG_S_MAXITER
    }
    if (leader) {
      const double nan = __builtin_nan("");
      d.out[0] = dead ? nan : th[0];
      d.out[1] = dead ? nan : th[1];
      d.out[2] = dead ? nan : th[2];
      if (d.status) *d.status = status;
      if (a.dataflow) {
        // publish the parameters device-wide, then release the consumers whose
        // last input they were
        __threadfence();
        for (int q = a.cons_off[t]; q < a.cons_off[t + 1]; ++q) {
          const int c = a.cons[q];
          if (__hip_atomic_fetch_add(&a.deps[c], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1) {
            const int pos = __hip_atomic_fetch_add(&a.ctrl[3], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.ready[pos], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      __hip_atomic_store(&G.task[tpar ^ 1], rigid_next(a, abort_flag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    tpar ^= 1;
    if (!group_sync(G, abort_flag, a.spin_limit, &s_flag)) return;
  }
}

// Clears the queue / barrier words and marks every task aborted until it
// completes (a task the watchdog never let finish keeps that status).
__global__ void k_reset(int* ctrl, int n_ints, const TaskDesc* tasks, int n_tasks) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_ints; i += gridDim.x * blockDim.x) ctrl[i] = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_tasks; i += gridDim.x * blockDim.x)
    if (tasks[i].status) *tasks[i].status = 4;   // REG_S_ABORTED
}

__global__ void k_reset_rigid(int* ctrl, int n_ints, const RigidTask* tasks, int n_tasks, unsigned long long* slots,
                              int n_slots) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_ints; i += gridDim.x * blockDim.x) ctrl[i] = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_slots; i += gridDim.x * blockDim.x) slots[i] = kSlotEmpty;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_tasks; i += gridDim.x * blockDim.x)
    if (tasks[i].status) *tasks[i].status = 4;   // REG_S_ABORTED
}

__global__ void k_reset_dataflow(int* deps, const int* deps0, int* ready, const int* ready0, int n, int* ctrl,
                                 int n_ready0) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    deps[i] = deps0[i];
    ready[i] = ready0[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl[2] = 0;          // head
    ctrl[3] = n_ready0;   // tail
  }
}

// ---------------------------------------------------------------- plain path

__global__ void __launch_bounds__(kWG) k_plain_init(const TaskDesc* d, SolveArgs a, float* dst) {
  const int L = a.levels;
  const int hc = a.H >> (L - 1), wc = a.W >> (L - 1);
  const int n = hc * wc;
  for (int p = blockIdx.x * kWG + threadIdx.x; p < n; p += gridDim.x * kWG) {
    const int Y = p / wc, X = p - Y * wc;
    double vx, vy;
    init_pixel<float>(d->kind, d->ua, d->ub, a.H, a.W, L, X, Y, vx, vy);
    dst[p] = (float)vx;
    dst[(size_t)n + p] = (float)vy;
  }
}

__global__ void __launch_bounds__(kWG) k_plain_prolong(const float* uc, float* uf, int h, int w) {
  const int n = h * w;
  for (int p = blockIdx.x * kWG + threadIdx.x; p < n; p += gridDim.x * kWG) {
    const int y = p / w, x = p - y * w;
    double vx, vy;
    prolong_pixel<true>(uc, h >> 1, w >> 1, x, y, vx, vy);
    uf[p] = (float)vx;
    uf[(size_t)n + p] = (float)vy;
  }
}

__global__ void __launch_bounds__(kWG) k_plain_sweep(LevelView<float> V, int th, double* part) {
  __shared__ double red[kWG / kWave];
  sweep_tiles<float, SW_UPDATE, false, true, kRBStream>(V, blockIdx.x, gridDim.x, th, red, part, nullptr);
}

__global__ void __launch_bounds__(kWave) k_plain_reduce(const double* part, int n, double* E) {
  const double e = wave_sum_array(part, n, threadIdx.x);
  if (threadIdx.x == 0) *E = e;
}

__global__ void __launch_bounds__(256) k_copy(const float* src, float* dst, size_t n) {
  for (size_t p = blockIdx.x * (size_t)256 + threadIdx.x; p < n; p += (size_t)gridDim.x * 256)
    dst[p] = src ? src[p] : __builtin_nanf("");
}

inline int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b < 8192 ? (b ? b : 1) : 8192);
}

}  // namespace

const void* persistent_kernel(bool resident) {
  return resident ? (const void*)k_persistent<false, true> : (const void*)k_persistent<false, false>;
}

hipError_t launch_persistent(const SolveArgs& a, int grid, hipStream_t s) {
  if (a.flex)
    hipLaunchKernelGGL((k_persistent<true, true>), dim3(grid), dim3(kWG), 0, s, a);
  else if (a.resident)
    hipLaunchKernelGGL((k_persistent<false, true>), dim3(grid), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL((k_persistent<false, false>), dim3(grid), dim3(kWG), 0, s, a);
  return hipGetLastError();
}

const void* rigid_kernel() { return (const void*)k_rigid; }

hipError_t launch_rigid(const RigidArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_rigid, dim3(grid), dim3(kWG), 0, s, a);
  return hipGetLastError();
}

// *sticky |= the abort word of a finished persistent launch (clear: *sticky = 0)
__global__ void k_note_abort(const int* ctrl, int* sticky, int clear) {
  if (threadIdx.x == 0) *sticky = clear ? 0 : (*sticky | (ctrl[1] != 0));
}

hipError_t launch_note_abort(const int* ctrl, int* sticky, bool clear, hipStream_t s) {
  hipLaunchKernelGGL(k_note_abort, dim3(1), dim3(64), 0, s, ctrl, sticky, clear ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_reset_ctrl(int* ctrl, int n_ints, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(grid_for((size_t)n_ints)), dim3(256), 0, s, ctrl, n_ints,
                     (const TaskDesc*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_reset_tasks(int* ctrl, int n_ints, const TaskDesc* tasks, int n_tasks, hipStream_t s) {
  const size_t n = (size_t)(n_ints > n_tasks ? n_ints : n_tasks);
  hipLaunchKernelGGL(k_reset, dim3(grid_for(n)), dim3(256), 0, s, ctrl, n_ints, tasks, n_tasks);
  return hipGetLastError();
}

hipError_t launch_reset_rigid(int* ctrl, int n_ints, const RigidTask* tasks, int n_tasks, unsigned long long* slots,
                              int n_slots, hipStream_t s) {
  const size_t n = (size_t)std::max(std::max(n_ints, n_tasks), n_slots);
  hipLaunchKernelGGL(k_reset_rigid, dim3(grid_for(n)), dim3(256), 0, s, ctrl, n_ints, tasks, n_tasks, slots, n_slots);
  return hipGetLastError();
}

hipError_t launch_reset_dataflow(int* deps, const int* deps0, int* ready, const int* ready0, int n_tasks,
                                 int* ctrl, int n_ready0, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_dataflow, dim3(grid_for((size_t)n_tasks)), dim3(256), 0, s, deps, deps0, ready, ready0,
                     n_tasks, ctrl, n_ready0);
  return hipGetLastError();
}

hipError_t launch_plain_init(const TaskDesc* d_task, const SolveArgs& a, float* dst, hipStream_t s) {
  const int L = a.levels;
  const size_t n = (size_t)(a.H >> (L - 1)) * (a.W >> (L - 1));
  hipLaunchKernelGGL(k_plain_init, dim3(grid_for(n)), dim3(kWG), 0, s, d_task, a, dst);
  return hipGetLastError();
}

hipError_t launch_plain_prolong(const float* uc, float* uf, int h, int w, hipStream_t s) {
  hipLaunchKernelGGL(k_plain_prolong, dim3(grid_for((size_t)h * w)), dim3(kWG), 0, s, uc, uf, h, w);
  return hipGetLastError();
}

hipError_t launch_plain_sweep(const float* R, const float* T, int pitch, const float* u, float* un, int h, int w,
                              double tau, double lam, int th, double* part, hipStream_t s) {
  LevelView<float> V;
  V.R = R;
  V.T = T;
  V.u = u;
  V.out = un;
  V.h = h;
  V.w = w;
  V.pitch = pitch;
  V.tau = tau;
  V.lam = lam;
  hipLaunchKernelGGL(k_plain_sweep, dim3(tiles_of(h, w, th)), dim3(kWG), 0, s, V, th, part);
  return hipGetLastError();
}

hipError_t launch_plain_reduce(const double* part, int n, double* E, hipStream_t s) {
  hipLaunchKernelGGL(k_plain_reduce, dim3(1), dim3(kWave), 0, s, part, n, E);
  return hipGetLastError();
}

hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace rs
