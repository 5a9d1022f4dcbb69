// C interface of the registration library: argument validation, workspace,
// batch / scan orchestration and the plain and batched execution paths.
#include "regscan.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "plan.h"
#include "sweep.h"

using namespace rs;

namespace {

thread_local std::string g_err;
std::recursive_mutex g_mu;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(REG_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)          \
  do {                     \
    int r_ = (expr);       \
    if (r_ != REG_OK) return r_; \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

struct State {
  bool init = false;
  int device = -1;
  int n_cu = 0;
  int blocks_per_cu = 0;          // persistent solver with resident levels (and the flex phase 1)
  int blocks_per_cu_stream = 0;   // the instantiation without them
  int tile_rows = 64;
  int max_group = 64;
  bool resident = true;
  unsigned spin_limit = 1u << 22;   // ~seconds of polling before the watchdog aborts a run
  DevBuf pyr, slots, part, ctrl, tasks, nodes, upair, iters, status, misc, lvl, flow, mock;
  DevBuf flexw, flexn, flext, flexf;   // flexible-segment scan: worker state, pool, tasks, flow
  DevBuf rnodes, rtasks, rpart, rctrl, rflow;   // rigid operator: parameters, descriptors, sums, queue, DAG
  int rigid_blocks_per_cu = 0;
  double* h_E = nullptr;   // pinned host scalar for the plain path
  int* h_abort = nullptr;  // pinned host copy of the sticky watchdog word
  DevBuf abortw;           // sticky: a persistent launch of this call was aborted
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used = 0;
  struct Graph {
    std::string key;
    unsigned generation;
    hipGraphExec_t exec;
    DevBuf tasks, flow;   // descriptors owned by the graph
  };
  std::vector<Graph> graphs;
  std::map<long long, std::pair<int, int>> tuned;   // autotune results by shape
  unsigned generation = 0;   // bumps whenever a workspace buffer moves
};

State g;

int ensure_device() {
  if (g.init) return REG_OK;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return fail(REG_E_NODEVICE, "no HIP device available");
  HIPCHK(hipGetDevice(&g.device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, g.device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(REG_E_NODEVICE, "device %s is not gfx950 (this library is built for gfx950 only)",
                prop.gcnArchName);
  g.n_cu = prop.multiProcessorCount;
  int nb = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persistent_kernel(true), kWG, 0));
  if (nb < 1) return fail(REG_E_HIP, "persistent kernel cannot be resident");
  g.blocks_per_cu = nb;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persistent_kernel(false), kWG, 0));
  if (nb < 1) return fail(REG_E_HIP, "persistent kernel cannot be resident");
  g.blocks_per_cu_stream = nb;
  HIPCHK(hipHostMalloc((void**)&g.h_E, sizeof(double), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&g.h_abort, sizeof(int), hipHostMallocDefault));
  if (hipMalloc(&g.abortw.p, 256) != hipSuccess) return fail(REG_E_NOMEM, "watchdog word");
  g.abortw.n = 256;
  g.init = true;
  return REG_OK;
}

int ensure(DevBuf& b, size_t bytes) {
  if (b.n >= bytes) return REG_OK;
  if (b.p) {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipFree(b.p));
    b.p = nullptr;
    b.n = 0;
  }
  size_t want = std::max(bytes, (size_t)256);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(REG_E_NOMEM, "workspace allocation of %zu bytes failed", want);
  }
  b.n = want;
  g.generation++;
  return REG_OK;
}

int check_dims(int B, int H, int W) {
  if (B < 0) return fail(REG_E_INVALID, "batch size %d < 0", B);
  if (H < 1 || W < 1) return fail(REG_E_INVALID, "image size %dx%d must be positive", H, W);
  if (H > 16384 || W > 16384 || (long long)H * W > (1LL << 26))
    return fail(REG_E_INVALID, "image size %dx%d exceeds 16384 per side or 2^26 pixels", H, W);
  return REG_OK;
}

int check_params(const reg_params_t* p, int H, int W) {
  if (!p) return fail(REG_E_INVALID, "params is NULL");
  if (p->levels < 1 || p->levels > kMaxLevels) return fail(REG_E_INVALID, "levels %d not in [1, %d]", p->levels, kMaxLevels);
  if (p->max_iter < 1) return fail(REG_E_INVALID, "max_iter %d < 1", p->max_iter);
  if (!(p->tau > 0.0) || !std::isfinite(p->tau)) return fail(REG_E_INVALID, "tau must be positive and finite");
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return fail(REG_E_INVALID, "lambda must be >= 0 and finite");
  if (!(p->rel_tol >= 0.0) || !std::isfinite(p->rel_tol)) return fail(REG_E_INVALID, "rel_tol must be >= 0 and finite");
  const int F = 1 << (p->levels - 1);
  if (H % F || W % F) return fail(REG_E_INVALID, "%dx%d is not divisible by 2^(levels-1) = %d", H, W, F);
  if (H / F < 8 || W / F < 8) return fail(REG_E_INVALID, "coarsest level %dx%d is below 8 px", H / F, W / F);
  return REG_OK;
}

hipEvent_t* next_events() {
  if (g.events_used == g.events.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return nullptr;
    g.events.push_back({a, b});
  }
  return &g.events[g.events_used++].first;
}

// ------------------------------------------------------------------ pyramid

// The solver's padded pyramid of all N frames (levels 0..L-1, see SolveArgs)
// in g.pyr.
struct Pyr {
  const float* lv[kMaxLevels];   // pixel (0, 0) of frame 0 of level l
  int pitch[kMaxLevels];
  size_t fstride[kMaxLevels];
};

int level_pitch(int w) { return (kPadLeft + w + 1 + 31) / 32 * 32; }

int build_pyramid(const float* frames, int N, int H, int W, int L, Pyr& P, hipStream_t s) {
  std::memset(&P, 0, sizeof P);
  size_t total = 0;
  for (int l = 0; l < L; ++l) {
    P.pitch[l] = level_pitch(W >> l);
    P.fstride[l] = (size_t)((H >> l) + 2) * P.pitch[l];
    total += (size_t)N * P.fstride[l];
  }
  TRY(ensure(g.pyr, total * sizeof(float)));
  float* p = (float*)g.pyr.p;
  for (int l = 0; l < L; ++l) {
    if (l == 0)
      HIPCHK(launch_pad_level(frames, W, (size_t)H * W, true, p, P.pitch[0], N, H, W, s));
    else
      HIPCHK(launch_pad_level(P.lv[l - 1], P.pitch[l - 1], P.fstride[l - 1], false, p, P.pitch[l], N, H >> l,
                              W >> l, s));
    P.lv[l] = p + P.pitch[l] + kPadLeft;
    p += (size_t)N * P.fstride[l];
  }
  return REG_OK;
}

SolveArgs base_args(const Pyr& P, int H, int W, const reg_params_t* p) {
  SolveArgs a;
  std::memset(&a, 0, sizeof a);
  for (int l = 0; l < kMaxLevels; ++l) {
    a.pyr[l] = l < p->levels ? P.lv[l] : nullptr;
    a.pitch[l] = P.pitch[l];
    a.fstride[l] = P.fstride[l];
  }
  a.H = H;
  a.W = W;
  a.levels = p->levels;
  a.max_iter = p->max_iter;
  a.fixed_iter = p->fixed_iter ? 1 : 0;
  a.tau = p->tau;
  a.lam = p->lambda;
  a.rel_tol = p->rel_tol;
  a.max_tiles = 0;
  for (int l = 0; l < p->levels; ++l) {
    a.thl[l] = level_tile_rows(g.tile_rows, l);
    a.max_tiles = std::max(a.max_tiles, tiles_of(H >> l, W >> l, a.thl[l]));
  }
  a.resident = g.resident ? 1 : 0;
  a.slot_floats = slot_floats_for(H, W, p->levels, a.lvl_off, &a.bufB_off);
  a.colx_off = a.slot_floats;
  a.colx_stride = (size_t)16 * kMaxRPT * a.max_tiles;
  a.slot_floats += 2 * a.colx_stride;
  a.spin_limit = g.spin_limit;
  return a;
}

// ------------------------------------------------------------ batched path

struct Launch {
  int g, groups, grid;
};

// Workgroups per registration.  When the finest level can run
// register-resident (64-column tiles, tile height a power of two <= 64 that
// divides the height) and its tile count fits the cap, the group gets one
// workgroup per tile.  Otherwise the largest power of two within the cap and
// the tile count.  The cap is max_group; batched runs stop doubling once
// fewer groups than tasks would remain, dataflow runs once fewer than
// min(kDataflowGroups, tasks) groups would be resident: a dataflow scan of a
// long series has thousands of ready registrations, and more, smaller groups
// pay fewer members per iteration barrier (measured on the 256x256, 512x512
// and 1024x1024 series: 16 workgroups per registration, 64 resident groups,
// beat 32 and 64 by 7-22%; the tile assignment does not change results).
constexpr int kDataflowGroups = 64;

int group_size(int n_tasks, int H, int W, bool dataflow) {
  const int slots = g.blocks_per_cu * g.n_cu;
  const int th = g.tile_rows;
  const int tiles = tiles_of(H, W, th);
  int cap = g.max_group;
  if (dataflow) cap = std::min(cap, std::max(1, slots / std::max(1, std::min(kDataflowGroups, n_tasks))));
  if (g.resident && W % kTileW == 0 && H % th == 0 && th <= 4 * kMaxRPT && (th & (th - 1)) == 0 &&
      tiles <= cap && tiles <= kMaxGroup && 8 * tiles <= slots)
    return tiles;
  int gs = 1;
  while (gs * 2 <= cap && gs * 2 <= tiles && 8 * gs * 2 <= slots &&
         (dataflow || (long long)n_tasks * gs * 2 <= slots))
    gs *= 2;
  return gs;
}

// Whether some pyramid level of a registration runs register-resident in
// groups of gs workgroups (the condition of run_task); if none does, the
// launch uses the solver instantiation without resident levels.
bool any_resident(const SolveArgs& a, int gs) {
  if (!a.resident) return false;
  for (int l = 0; l < a.levels; ++l) {
    const int h = a.H >> l, w = a.W >> l, th = a.thl[l];
    if (w % kTileW == 0 && h % th == 0 && tiles_of(h, w, th) <= gs && th <= 4 * kMaxRPT && (th & (th - 1)) == 0)
      return true;
  }
  return false;
}

// Workgroups that can be resident at once for the chosen instantiation.
int solver_slots(bool resident) { return (resident ? g.blocks_per_cu : g.blocks_per_cu_stream) * g.n_cu; }

// A group of gs workgroups halved until 8 groups (one per XCD, the fewest a
// launch has) of the instantiation it selects are resident at once: every
// member of a group must be running for its barriers to complete, and the
// streaming-only instantiation fits fewer workgroups per CU than the one
// group_size counts with.
int fit_group(const SolveArgs& a, int gs) {
  while (gs > 1 && 8 * gs > solver_slots(any_resident(a, gs))) gs >>= 1;
  return gs;
}

Launch plan_launch(int n_tasks, const SolveArgs& a) {
  const int gs = fit_group(a, group_size(n_tasks, a.H, a.W, false));
  const int slots = solver_slots(any_resident(a, gs));
  int groups = std::min(slots / gs, ((n_tasks + 7) / 8) * 8);
  groups = std::max(8, (groups / 8) * 8);
  return {gs, groups, groups * gs};
}

// Runs n tasks (device descriptors) with one persistent launch.
int run_batched(SolveArgs a, const TaskDesc* d_tasks, int n, hipStream_t s, bool timed) {
  if (n == 0) return REG_OK;
  const Launch L = plan_launch(n, a);
  a.resident = any_resident(a, L.g) ? 1 : 0;
  const int ctrl_ints = kCtrlHead + kCtrlGroup * L.groups;
  TRY(ensure(g.ctrl, (size_t)ctrl_ints * sizeof(int)));
  a.max_tiles = std::max(a.max_tiles, L.g);   // resident levels keep one energy slot per member
  TRY(ensure(g.part, (size_t)L.groups * 3 * a.max_tiles * sizeof(double)));
  TRY(ensure(g.slots, (size_t)L.groups * a.slot_floats * sizeof(float)));
  a.tasks = d_tasks;
  a.n_tasks = n;
  a.g = L.g;
  a.ctrl = (int*)g.ctrl.p;
  a.part = (double*)g.part.p;
  a.ws = (float*)g.slots.p;
  HIPCHK(launch_reset_tasks(a.ctrl, ctrl_ints, d_tasks, n, s));
  hipEvent_t* ev = timed ? next_events() : nullptr;
  if (ev) HIPCHK(hipEventRecord(ev[0], s));
  HIPCHK(launch_persistent(a, L.grid, s));
  if (ev) HIPCHK(hipEventRecord(ev[1], s));
  HIPCHK(launch_note_abort(a.ctrl, (int*)g.abortw.p, false, s));
  return REG_OK;
}

// Runs a task DAG with one persistent launch.  deps0/ready0/cons_off/cons are
// device arrays (see SolveArgs); deps/ready are their working copies.
int run_dataflow(SolveArgs a, const TaskDesc* d_tasks, int n, int* deps, const int* deps0, int* ready,
                 const int* ready0, int n_ready0, const int* cons_off, const int* cons, hipStream_t s, bool timed) {
  if (n == 0) return REG_OK;
  const int gs = fit_group(a, group_size(n, a.H, a.W, true));
  a.resident = any_resident(a, gs) ? 1 : 0;
  const int groups = std::max(8, (solver_slots(a.resident != 0) / gs / 8) * 8);
  const int ctrl_ints = kCtrlHead + kCtrlGroup * groups;
  TRY(ensure(g.ctrl, (size_t)ctrl_ints * sizeof(int)));
  a.max_tiles = std::max(a.max_tiles, gs);
  TRY(ensure(g.part, (size_t)groups * 3 * a.max_tiles * sizeof(double)));
  TRY(ensure(g.slots, (size_t)groups * a.slot_floats * sizeof(float)));
  a.tasks = d_tasks;
  a.n_tasks = n;
  a.g = gs;
  a.ctrl = (int*)g.ctrl.p;
  a.part = (double*)g.part.p;
  a.ws = (float*)g.slots.p;
  a.dataflow = 1;
  a.deps = deps;
  a.ready = ready;
  a.cons_off = cons_off;
  a.cons = cons;
  HIPCHK(launch_reset_tasks(a.ctrl, ctrl_ints, d_tasks, n, s));
  HIPCHK(launch_reset_dataflow(deps, deps0, ready, ready0, n, a.ctrl, n_ready0, s));
  hipEvent_t* ev = timed ? next_events() : nullptr;
  if (ev) HIPCHK(hipEventRecord(ev[0], s));
  HIPCHK(launch_persistent(a, groups * gs, s));
  if (ev) HIPCHK(hipEventRecord(ev[1], s));
  HIPCHK(launch_note_abort(a.ctrl, (int*)g.abortw.p, false, s));
  return REG_OK;
}

// -------------------------------------------------------------- plain path

int run_plain(SolveArgs a, const std::vector<TaskDesc>& tasks, const TaskDesc* d_tasks, hipStream_t s) {
  TRY(ensure(g.slots, a.slot_floats * sizeof(float)));
  TRY(ensure(g.part, (size_t)(a.max_tiles + 1) * sizeof(double)));
  float* slot = (float*)g.slots.p;
  double* part = (double*)g.part.p;
  double* dE = part + a.max_tiles;
  const int L = a.levels;
  std::vector<int32_t> iters(L);
  for (size_t b = 0; b < tasks.size(); ++b) {
    const TaskDesc& d = tasks[b];
    auto start = [&](int l) -> float* { return l == 0 ? d.out : slot + a.lvl_off[l]; };
    float* cur = start(L - 1);
    HIPCHK(launch_plain_init(d_tasks + b, a, cur, s));
    float* bufB = slot + a.bufB_off;
    int32_t status = 0;
    bool dead = false;
    for (int l = L - 1; l >= 0; --l) {
      iters[l] = 0;
      if (dead) continue;
      const int h = a.H >> l, w = a.W >> l;
      if (l < L - 1) {
        HIPCHK(launch_plain_prolong(cur, start(l), h, w, s));
        cur = start(l);
      }
      float* other = bufB;
      const float* R = a.pyr[l] + (size_t)d.ref * a.fstride[l];
      const float* T = a.pyr[l] + (size_t)d.tmpl * a.fstride[l];
      const int th = stream_tile_rows(a.thl[l], h, w, kMaxGroup);   // the solver's tiles of a streamed level
      const int nt = tiles_of(h, w, th);
      double e_prev = 0.0;
      int it = 0;
      for (; it < a.max_iter; ++it) {
        HIPCHK(launch_plain_sweep(R, T, a.pitch[l], cur, other, h, w, a.tau, a.lam, th, part, s));
        HIPCHK(launch_plain_reduce(part, nt, dE, s));
        HIPCHK(hipMemcpyAsync(g.h_E, dE, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double E = *g.h_E;
        if (!std::isfinite(E)) {
          status |= REG_S_NONFINITE;
          dead = true;
          break;
        }
        if (!a.fixed_iter && it > 0 && level_stops(e_prev, E, a.rel_tol)) break;
        e_prev = E;
        std::swap(cur, other);
      }
      iters[l] = it;
      if (it == a.max_iter && !a.fixed_iter) status |= REG_S_MAXITER;
    }
    const size_t nf = (size_t)2 * a.H * a.W;
    if (dead)
      HIPCHK(launch_copy(nullptr, d.out, nf, s));
    else if (cur != d.out)
      HIPCHK(launch_copy(cur, d.out, nf, s));
    if (d.iters) HIPCHK(hipMemcpyAsync(d.iters, iters.data(), L * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (d.status) HIPCHK(hipMemcpyAsync(d.status, &status, sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));   // host staging of iters/status must outlive the copies
  }
  return REG_OK;
}

// Waits for the stream and reports a watchdog abort of any persistent launch
// since the sticky word was last cleared.
int check_abort(hipStream_t s, const char* what) {
  HIPCHK(hipMemcpyAsync(g.h_abort, g.abortw.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (*g.h_abort) return fail(REG_E_HIP, "%s abandoned by the forward-progress watchdog", what);
  return REG_OK;
}

int upload_tasks(DevBuf& buf, const std::vector<TaskDesc>& t, hipStream_t s) {
  if (t.empty()) return REG_OK;
  TRY(ensure(buf, t.size() * sizeof(TaskDesc)));
  HIPCHK(hipMemcpyAsync(buf.p, t.data(), t.size() * sizeof(TaskDesc), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return REG_OK;
}

void drop_graphs() {
  for (auto& gr : g.graphs) {
    (void)hipGraphExecDestroy(gr.exec);
    if (gr.tasks.p) (void)hipFree(gr.tasks.p);
    if (gr.flow.p) (void)hipFree(gr.flow.p);
  }
  g.graphs.clear();
}

}  // namespace

namespace rs {
size_t slot_floats_for(int H, int W, int levels, size_t* lvl_off, size_t* bufB_off) {
  size_t off = 0;
  for (int l = 0; l < kMaxLevelsHost; ++l) lvl_off[l] = 0;
  for (int l = 1; l < levels; ++l) {
    lvl_off[l] = off;
    off += (size_t)2 * (H >> l) * (W >> l);
  }
  *bufB_off = off;
  off += (size_t)2 * H * W;
  return (off + 63) & ~(size_t)63;
}
}  // namespace rs

// ===================================================================== C ABI

// Dependency lists -> the dataflow arrays of run_dataflow: per task the
// number of inputs produced by other tasks, the initially ready tasks, and the
// consumers of every task.
struct TaskFlow {
  std::vector<int> host;   // deps0 [T], ready0 [T], cons_off [T + 1], cons
  int n_ready0 = 0;
};

TaskFlow task_flow(const std::vector<std::vector<int>>& deps) {
  const int T = (int)deps.size();
  TaskFlow f;
  std::vector<int> deps0(T), ready0(T, -1), cons_off(T + 1, 0), cons;
  for (int t = 0; t < T; ++t) {
    deps0[t] = (int)deps[t].size();
    for (int d : deps[t]) cons_off[d + 1]++;
    if (deps0[t] == 0) ready0[f.n_ready0++] = t;
  }
  for (int t = 0; t < T; ++t) cons_off[t + 1] += cons_off[t];
  cons.assign(cons_off[T], 0);
  std::vector<int> fill(cons_off.begin(), cons_off.end() - 1);
  for (int t = 0; t < T; ++t)
    for (int d : deps[t]) cons[fill[d]++] = t;
  f.host = deps0;
  f.host.insert(f.host.end(), ready0.begin(), ready0.end());
  f.host.insert(f.host.end(), cons_off.begin(), cons_off.end());
  f.host.insert(f.host.end(), cons.begin(), cons.end());
  return f;
}

// ------------------------------------------------------------ mock scan

namespace {

// Host arrays of a dataflow run over a plan: initial dependency counts (inputs
// that are op outputs), the initially ready ops, and the consumers of every
// op output.
struct Flow {
  std::vector<int> deps0, ready0, cons_off, cons;
  int n_ready0 = 0;
};

Flow plan_flow(const std::vector<PlanOp>& plan, int n_base) {
  const int n = (int)plan.size();
  Flow f;
  f.deps0.assign(n, 0);
  f.ready0.assign(n, -1);
  f.cons_off.assign(n + 1, 0);
  for (const PlanOp& q : plan)
    for (int in : {q.a, q.b})
      if (in >= n_base) f.cons_off[in - n_base + 1]++;
  for (int q = 0; q < n; ++q) f.cons_off[q + 1] += f.cons_off[q];
  f.cons.assign(f.cons_off[n], 0);
  std::vector<int> fill(f.cons_off.begin(), f.cons_off.end() - 1);
  for (int q = 0; q < n; ++q) {
    for (int in : {plan[q].a, plan[q].b})
      if (in >= n_base) {
        f.deps0[q]++;
        f.cons[fill[in - n_base]++] = q;
      }
    if (f.deps0[q] == 0) f.ready0[f.n_ready0++] = q;
  }
  return f;
}

// Node holding the prefix (0, e + 1) of element e under `plan`.
std::vector<int> final_nodes(const std::vector<PlanOp>& plan, int n_base) {
  std::vector<int> fin(n_base, -1);
  fin[0] = 0;
  for (const PlanOp& q : plan)
    if (q.i == 0) fin[q.k - 1] = q.out;
  return fin;
}

struct MockBuf {
  char* p;
  template <typename T>
  T* take(size_t n) {
    T* r = (T*)p;
    p += (n * sizeof(T) + 255) / 256 * 256;
    return r;
  }
};

// Workspace of scan_mock_run (every array rounded up to 256 bytes).
size_t mock_bytes(size_t n_nodes, size_t n_ops, size_t n_base, size_t n_levels, size_t workers) {
  return 32 * 256 + n_nodes * 8 + n_ops * 48 + n_base * 4 + (n_levels + 16) * 4 + workers * 40;
}

}  // namespace

extern "C" {

const char* reg_last_error(void) { return g_err.c_str(); }

int reg_version(void) { return 100; }

int reg_pyramid(const float* frames, float* pyr, int N, int H, int W, int levels, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(N, H, W));
  if (levels < 1 || levels > kMaxLevels) return fail(REG_E_INVALID, "levels %d not in [1, %d]", levels, kMaxLevels);
  const int F = 1 << (levels - 1);
  if (H % F || W % F || H / F < 8 || W / F < 8)
    return fail(REG_E_INVALID, "%dx%d cannot hold %d levels (divisible by %d, coarsest >= 8 px)", H, W, levels, F);
  if (N == 0 || levels == 1) return REG_OK;
  if (!frames || !pyr) return fail(REG_E_INVALID, "NULL pointer");
  TRY(ensure_device());
  hipStream_t s = (hipStream_t)stream;
  const float* src = frames;
  float* dst = pyr;
  for (int l = 1; l < levels; ++l) {
    HIPCHK(launch_restrict_frame(src, dst, N, H >> (l - 1), W >> (l - 1), false, s));
    src = dst;
    dst += (size_t)N * (H >> l) * (W >> l);
  }
  return REG_OK;
}

static int warp_common(const void* T, const void* u, void* out, int B, int H, int W, void* stream, bool f64) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(B, H, W));
  if (B == 0) return REG_OK;
  if (!T || !u || !out) return fail(REG_E_INVALID, "NULL pointer");
  if (out == T || out == u) return fail(REG_E_INVALID, "out aliases an input");
  TRY(ensure_device());
  HIPCHK(launch_warp(T, u, out, B, H, W, f64, (hipStream_t)stream));
  return REG_OK;
}

int reg_warp(const float* T, const float* u, float* out, int B, int H, int W, void* stream) {
  return warp_common(T, u, out, B, H, W, stream, false);
}
int reg_warp_f64(const double* T, const double* u, double* out, int B, int H, int W, void* stream) {
  return warp_common(T, u, out, B, H, W, stream, true);
}

static int adjoint_common(const void* gout, const void* u, void* gT, int B, int H, int W, void* stream, bool f64) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(B, H, W));
  if (B == 0) return REG_OK;
  if (!gout || !u || !gT) return fail(REG_E_INVALID, "NULL pointer");
  TRY(ensure_device());
  HIPCHK(launch_warp_adjoint(gout, u, gT, B, H, W, f64, (hipStream_t)stream));
  return REG_OK;
}

int reg_warp_adjoint(const float* gout, const float* u, float* gT, int B, int H, int W, void* stream) {
  return adjoint_common(gout, u, gT, B, H, W, stream, false);
}
int reg_warp_adjoint_f64(const double* gout, const double* u, double* gT, int B, int H, int W, void* stream) {
  return adjoint_common(gout, u, gT, B, H, W, stream, true);
}

static int energy_common(const void* R, const void* T, const void* u, double lam, double* E, void* grad,
                         double* gnorm2, int B, int H, int W, void* stream, bool f64) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(B, H, W));
  if (B == 0) return REG_OK;
  if (!R || !T || !u || !E) return fail(REG_E_INVALID, "NULL pointer");
  if (!(lam >= 0.0) || !std::isfinite(lam)) return fail(REG_E_INVALID, "lambda must be >= 0 and finite");
  TRY(ensure_device());
  const int th = g.tile_rows;
  const size_t nt = (size_t)tiles_of(H, W, th);
  TRY(ensure(g.misc, (size_t)2 * B * nt * sizeof(double)));
  HIPCHK(launch_energy_grad(R, T, u, lam, E, grad, gnorm2, B, H, W, th, (double*)g.misc.p, f64,
                            (hipStream_t)stream));
  return REG_OK;
}

int reg_energy_grad(const float* R, const float* T, const float* u, double lambda, double* E, float* grad,
                    double* gnorm2, int B, int H, int W, void* stream) {
  return energy_common(R, T, u, lambda, E, grad, gnorm2, B, H, W, stream, false);
}

// Scratch of reg_energy_grad_noalloc: the per-tile partial sums (energies,
// then squared gradient norms) that reg_energy_grad keeps in library
// workspace.  Every GPU holds its own copy until the process ends; every
// call on a GPU reuses it (calls that overlap on one GPU race).  The kernels
// write every partial sum before it is read, so nothing needs clearing.
// In host code `scratch` only stands for the symbol: its device address on
// the current GPU comes from hipGetSymbolAddress (noalloc_scratch).
constexpr size_t kNoallocSums = 262144;   // doubles: 2 MiB
static __device__ __align__(256) double scratch[kNoallocSums];

constexpr int kNoallocDevices = 64;
double* g_scratch_addr[kNoallocDevices] = {};   // per device, set on the first call there

// Device address of `scratch` on the current GPU (looked up once per GPU;
// allocates nothing).
static int noalloc_scratch(double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoallocDevices) return fail(REG_E_NODEVICE, "device %d beyond %d", dev, kNoallocDevices);
  if (!g_scratch_addr[dev]) {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(REG_E_NODEVICE, "device %s is not gfx950 (this library is built for gfx950 only)",
                  prop.gcnArchName);
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_addr[dev] = (double*)p;
  }
  *out = g_scratch_addr[dev];
  return REG_OK;
}

int reg_energy_grad_noalloc(const float* R, const float* T, const float* u, double lambda, double* E,
                            float* grad, double* gnorm2, int B, int H, int W, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(B, H, W));
  if (B == 0) return REG_OK;
  if (!R || !T || !u || !E) return fail(REG_E_INVALID, "NULL pointer");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(REG_E_INVALID, "lambda must be >= 0 and finite");
  const int th = g.tile_rows;
  const size_t sums = (size_t)(gnorm2 ? 2 : 1) * B * tiles_of(H, W, th);
  if (sums > kNoallocSums)
    return fail(REG_E_INVALID, "%zu tile sums (B = %d, %d tiles of %dx%d, %s) exceed the %zu of the allocation-free "
                "scratch", sums, B, tiles_of(H, W, th), H, W, gnorm2 ? "energy and gradient norm" : "energy",
                kNoallocSums);
  double* part = nullptr;
  TRY(noalloc_scratch(&part));
  HIPCHK(launch_energy_grad(R, T, u, lambda, E, grad, gnorm2, B, H, W, th, part, false, (hipStream_t)stream));
  return REG_OK;
}
int reg_energy_grad_f64(const double* R, const double* T, const double* u, double lambda, double* E,
                        double* grad, double* gnorm2, int B, int H, int W, void* stream) {
  return energy_common(R, T, u, lambda, E, grad, gnorm2, B, H, W, stream, true);
}

// Coarser levels of (Ia, u, Ib) for the differentiable energy, in g.lvl:
// per level l >= 1: Ia_l, Ib_l [B][h][w], u_l [B][2][h][w], and gradient
// buffers dIa_l, dIb_l, du_l of the same shapes.
struct PyrLevels {
  const void* Ia[kMaxLevels];
  const void* Ib[kMaxLevels];
  const void* u[kMaxLevels];
  void* dIa[kMaxLevels];
  void* dIb[kMaxLevels];
  void* du[kMaxLevels];
};

static int pyramid_levels(const void* Ia, const void* u, const void* Ib, int levels, int B, int H, int W,
                          bool f64, bool grads, PyrLevels& P, hipStream_t s) {
  const size_t es = f64 ? 8 : 4;
  size_t total = 0;
  for (int l = 1; l < levels; ++l) total += (size_t)B * (H >> l) * (W >> l) * (grads ? 8 : 4);
  TRY(ensure(g.lvl, total * es + 256));
  char* p = (char*)g.lvl.p;
  P.Ia[0] = Ia;
  P.Ib[0] = Ib;
  P.u[0] = u;
  for (int l = 1; l < levels; ++l) {
    const size_t n = (size_t)B * (H >> l) * (W >> l);
    void* a = p;
    p += n * es;
    void* b = p;
    p += n * es;
    void* v = p;
    p += 2 * n * es;
    HIPCHK(launch_restrict_frame(P.Ia[l - 1], a, B, H >> (l - 1), W >> (l - 1), f64, s));
    HIPCHK(launch_restrict_frame(P.Ib[l - 1], b, B, H >> (l - 1), W >> (l - 1), f64, s));
    HIPCHK(launch_restrict(P.u[l - 1], v, 0.5, 2 * B, H >> (l - 1), W >> (l - 1), f64, s));
    P.Ia[l] = a;
    P.Ib[l] = b;
    P.u[l] = v;
    if (grads) {
      P.dIa[l] = p;
      p += n * es;
      P.dIb[l] = p;
      p += n * es;
      P.du[l] = p;
      p += 2 * n * es;
    }
  }
  return REG_OK;
}

static int pyr_check(int levels, int B, int H, int W) {
  TRY(check_dims(B, H, W));
  if (levels < 1 || levels > kMaxLevels) return fail(REG_E_INVALID, "levels %d not in [1, %d]", levels, kMaxLevels);
  const int F = 1 << (levels - 1);
  if (H % F || W % F) return fail(REG_E_INVALID, "%dx%d is not divisible by %d", H, W, F);
  return REG_OK;
}

static int pyr_energy_common(const void* Ia, const void* u, const void* Ib, double lam, int levels, double* E,
                             int B, int H, int W, void* stream, bool f64) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(pyr_check(levels, B, H, W));
  if (B == 0) return REG_OK;
  if (!Ia || !u || !Ib || !E) return fail(REG_E_INVALID, "NULL pointer");
  if (!(lam >= 0.0) || !std::isfinite(lam)) return fail(REG_E_INVALID, "lambda must be >= 0 and finite");
  TRY(ensure_device());
  hipStream_t s = (hipStream_t)stream;
  PyrLevels P;
  TRY(pyramid_levels(Ia, u, Ib, levels, B, H, W, f64, false, P, s));
  const int th = g.tile_rows;
  const size_t nt = (size_t)tiles_of(H, W, th);
  TRY(ensure(g.misc, ((size_t)2 * B * nt + B) * sizeof(double)));
  double* part = (double*)g.misc.p;
  double* El = part + 2 * B * nt;
  for (int l = 0; l < levels; ++l) {
    HIPCHK(launch_energy_grad(P.Ib[l], P.Ia[l], P.u[l], lam, El, nullptr, nullptr, B, H >> l, W >> l, th, part,
                              f64, s));
    HIPCHK(launch_add_energy(El, E, B, l == 0, s));
  }
  return REG_OK;
}

int reg_pyramid_energy(const float* Ia, const float* u, const float* Ib, double lambda, int levels, double* E,
                       int B, int H, int W, void* stream) {
  return pyr_energy_common(Ia, u, Ib, lambda, levels, E, B, H, W, stream, false);
}
int reg_pyramid_energy_f64(const double* Ia, const double* u, const double* Ib, double lambda, int levels,
                           double* E, int B, int H, int W, void* stream) {
  return pyr_energy_common(Ia, u, Ib, lambda, levels, E, B, H, W, stream, true);
}

static int pyr_backward_common(const void* Ia, const void* u, const void* Ib, double lam, int levels,
                               const double* gE, void* dIa, void* du, void* dIb, int B, int H, int W,
                               void* stream, bool f64) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(pyr_check(levels, B, H, W));
  if (B == 0) return REG_OK;
  if (!Ia || !u || !Ib || !gE) return fail(REG_E_INVALID, "NULL pointer");
  if (!(lam >= 0.0) || !std::isfinite(lam)) return fail(REG_E_INVALID, "lambda must be >= 0 and finite");
  TRY(ensure_device());
  hipStream_t s = (hipStream_t)stream;
  PyrLevels P;
  TRY(pyramid_levels(Ia, u, Ib, levels, B, H, W, f64, true, P, s));
  const size_t es = f64 ? 8 : 4;
  const size_t n0 = (size_t)B * H * W;
  // level-0 outputs the caller skipped go to scratch
  TRY(ensure(g.misc, 4 * n0 * es));
  char* scratch = (char*)g.misc.p;
  P.dIa[0] = dIa ? dIa : (void*)scratch;
  P.dIb[0] = dIb ? dIb : (void*)(scratch + n0 * es);
  P.du[0] = du ? du : (void*)(scratch + 2 * n0 * es);
  for (int l = levels - 1; l >= 0; --l) {
    const bool top = l == levels - 1;
    // dIa (scattered into) and dIb (added to) start from the transpose of
    // the frame restriction applied to the coarser level's gradients
    HIPCHK(launch_restrict_frame_adjoint(top ? nullptr : P.dIa[l + 1], P.dIa[l], B, H >> l, W >> l, f64, s));
    if (!top) HIPCHK(launch_restrict_frame_adjoint(P.dIb[l + 1], P.dIb[l], B, H >> l, W >> l, f64, s));
    HIPCHK(launch_energy_backward_level(P.Ia[l], P.u[l], P.Ib[l], lam, gE, P.dIa[l], P.du[l], P.dIb[l],
                                        top ? nullptr : P.du[l + 1], !top, B, H >> l, W >> l, f64, s));
  }
  return REG_OK;
}

int reg_pyramid_energy_backward(const float* Ia, const float* u, const float* Ib, double lambda, int levels,
                                const double* gE, float* dIa, float* du, float* dIb, int B, int H, int W,
                                void* stream) {
  return pyr_backward_common(Ia, u, Ib, lambda, levels, gE, dIa, du, dIb, B, H, W, stream, false);
}
int reg_pyramid_energy_backward_f64(const double* Ia, const double* u, const double* Ib, double lambda,
                                    int levels, const double* gE, double* dIa, double* du, double* dIb, int B,
                                    int H, int W, void* stream) {
  return pyr_backward_common(Ia, u, Ib, lambda, levels, gE, dIa, du, dIb, B, H, W, stream, true);
}

int reg_compose(const float* u_ij, const float* u_jk, float* out, int B, int H, int W, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(B, H, W));
  if (B == 0) return REG_OK;
  if (!u_ij || !u_jk || !out) return fail(REG_E_INVALID, "NULL pointer");
  if (out == u_ij || out == u_jk) return fail(REG_E_INVALID, "out aliases an input");
  TRY(ensure_device());
  HIPCHK(launch_compose(u_ij, u_jk, out, B, H, W, (hipStream_t)stream));
  return REG_OK;
}

int reg_restrict(const float* in, float* out, double scale, int B, int H, int W, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(B, H, W));
  if (H % 2 || W % 2) return fail(REG_E_INVALID, "%dx%d is not even", H, W);
  if (B == 0) return REG_OK;
  if (!in || !out) return fail(REG_E_INVALID, "NULL pointer");
  TRY(ensure_device());
  HIPCHK(launch_restrict(in, out, scale, B, H, W, false, (hipStream_t)stream));
  return REG_OK;
}

int reg_prolong(const float* uc, float* uf, int B, int Hf, int Wf, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(B, Hf, Wf));
  if (Hf % 2 || Wf % 2) return fail(REG_E_INVALID, "%dx%d is not even", Hf, Wf);
  if (B == 0) return REG_OK;
  if (!uc || !uf) return fail(REG_E_INVALID, "NULL pointer");
  TRY(ensure_device());
  HIPCHK(launch_prolong(uc, uf, B, Hf, Wf, (hipStream_t)stream));
  return REG_OK;
}

int reg_solve_batch(const float* frames, int N, int H, int W, const int32_t* ref_idx, const int32_t* tmpl_idx,
                    const float* u0, float* u, int32_t* iters, int32_t* status, int B, const reg_params_t* p,
                    int mode, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(B, H, W));
  TRY(check_params(p, H, W));
  if (N < 1) return fail(REG_E_INVALID, "N = %d frames", N);
  if (mode != REG_PLAIN && mode != REG_BATCHED && mode != REG_DATAFLOW)
    return fail(REG_E_INVALID, "unknown mode %d", mode);
  if (B == 0) return REG_OK;
  if (!frames || !ref_idx || !tmpl_idx || !u) return fail(REG_E_INVALID, "NULL pointer");
  if (u0 && u0 == u) return fail(REG_E_INVALID, "u aliases u0");
  for (int b = 0; b < B; ++b)
    if (ref_idx[b] < 0 || ref_idx[b] >= N || tmpl_idx[b] < 0 || tmpl_idx[b] >= N)
      return fail(REG_E_INVALID, "frame index out of range at item %d", b);
  TRY(ensure_device());
  hipStream_t s = (hipStream_t)stream;
  Pyr P;
  TRY(build_pyramid(frames, N, H, W, p->levels, P, s));
  SolveArgs a = base_args(P, H, W, p);
  const size_t nf = (size_t)2 * H * W;
  std::vector<TaskDesc> tasks(B);
  for (int b = 0; b < B; ++b) {
    TaskDesc& d = tasks[b];
    d.ref = ref_idx[b];
    d.tmpl = tmpl_idx[b];
    d.kind = u0 ? 2 : 0;
    d.pad = 0;
    d.ua = u0 ? u0 + b * nf : nullptr;
    d.ub = nullptr;
    d.out = u + b * nf;
    d.iters = iters ? iters + (size_t)b * p->levels : nullptr;
    d.status = status ? status + b : nullptr;
  }
  TRY(upload_tasks(g.tasks, tasks, s));
  g.events_used = 0;
  if (mode == REG_PLAIN) return run_plain(a, tasks, (const TaskDesc*)g.tasks.p, s);
  HIPCHK(launch_note_abort((const int*)g.abortw.p, (int*)g.abortw.p, true, s));
  TRY(run_batched(a, (const TaskDesc*)g.tasks.p, B, s, true));
  return check_abort(s, "the batch");
}

int scan_plan(int M, int algo, int chunk, int global_algo, scan_op_t* ops, int cap, int* n_ops, int* n_levels) {
  std::vector<PlanOp> plan;
  int nl = 0;
  if (n_ops) *n_ops = 0;
  if (n_levels) *n_levels = 0;
  if (M < 1 || M > (1 << 24)) return fail(REG_E_INVALID, "M = %d not in [1, 2^24]", M);
  if (algo < SCAN_SEQ || algo > SCAN_HIER) return fail(REG_E_INVALID, "unknown scan algorithm %d", algo);
  if (algo == SCAN_HIER && (global_algo < SCAN_SEQ || global_algo > SCAN_BRENT_KUNG))
    return fail(REG_E_INVALID, "unknown global algorithm %d", global_algo);
  try {
    if (rs::build_plan(M, algo, chunk, global_algo, plan, nl) != 0) return fail(REG_E_INVALID, "invalid plan arguments");
  } catch (const std::exception& e) {
    return fail(REG_E_INVALID, "plan construction failed: %s", e.what());
  }
  if (n_ops) *n_ops = (int)plan.size();
  if (n_levels) *n_levels = nl;
  if (!ops) return REG_OK;
  if (cap < (int)plan.size()) return fail(REG_E_INVALID, "ops capacity %d < %zu", cap, plan.size());
  for (size_t n = 0; n < plan.size(); ++n) {
    const PlanOp& q = plan[n];
    ops[n] = scan_op_t{q.level, q.out, q.a, q.b, q.i, q.j, q.k};
  }
  return REG_OK;
}

int scan_run(const float* frames, int N, int H, int W, const reg_params_t* p, int algo, int chunk, int global_algo,
             int mode, int flags, float* phi0, float* u_pair, int32_t* op_iters, int32_t* status, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(1, H, W));
  TRY(check_params(p, H, W));
  if (N < 2) return fail(REG_E_INVALID, "a series needs N >= 2 frames (got %d)", N);
  if (mode != REG_PLAIN && mode != REG_BATCHED && mode != REG_DATAFLOW)
    return fail(REG_E_INVALID, "unknown mode %d", mode);
  if (flags & ~SCAN_F_GRAPH) return fail(REG_E_INVALID, "unknown flags 0x%x", flags);
  if (!frames || !phi0) return fail(REG_E_INVALID, "NULL pointer");
  const int M = N - 1;
  std::vector<PlanOp> plan;
  int n_levels = 0;
  if (algo < SCAN_SEQ || algo > SCAN_HIER) return fail(REG_E_INVALID, "unknown scan algorithm %d", algo);
  if (algo == SCAN_HIER && (global_algo < SCAN_SEQ || global_algo > SCAN_BRENT_KUNG))
    return fail(REG_E_INVALID, "unknown global algorithm %d", global_algo);
  try {
    if (rs::build_plan(M, algo, chunk, global_algo, plan, n_levels) != 0)
      return fail(REG_E_INVALID, "invalid plan arguments");
  } catch (const std::exception& e) {
    return fail(REG_E_INVALID, "plan construction failed: %s", e.what());
  }
  TRY(ensure_device());
  hipStream_t s = (hipStream_t)stream;
  const int L = p->levels;
  const size_t nf = (size_t)2 * H * W;
  const size_t n_ops = plan.size();

  // node storage: elements in u_pair, prefixes (0, k) in phi0, the rest in
  // workspace slots reused once their last consumer's level has completed
  std::vector<int> last_use(M + n_ops, 0);
  for (const PlanOp& q : plan) {
    last_use[q.a] = std::max(last_use[q.a], q.level);
    last_use[q.b] = std::max(last_use[q.b], q.level);
  }
  std::vector<int> slot_of(M + n_ops, -1);
  int n_slots = 0;
  {
    std::vector<std::vector<int>> dies(n_levels + 1);
    for (const PlanOp& q : plan)
      if (q.i != 0) dies[std::max(last_use[q.out], q.level)].push_back(q.out);
    std::vector<int> free_slots;
    size_t q = 0;
    for (int lvl = 1; lvl <= n_levels; ++lvl) {
      for (; q < n_ops && plan[q].level == lvl; ++q) {
        if (plan[q].i == 0) continue;
        if (free_slots.empty()) free_slots.push_back(n_slots++);
        slot_of[plan[q].out] = free_slots.back();
        free_slots.pop_back();
      }
      // levels overlap in dataflow mode: no reuse there
      if (mode != REG_DATAFLOW)
        for (int nd : dies[lvl]) free_slots.push_back(slot_of[nd]);
    }
  }
  TRY(ensure(g.nodes, std::max<size_t>(1, (size_t)n_slots) * nf * sizeof(float)));
  float* pair = u_pair;
  if (!pair) {
    TRY(ensure(g.upair, (size_t)M * nf * sizeof(float)));
    pair = (float*)g.upair.p;
  }
  int32_t* it_out = op_iters;
  int32_t* st_out = status;
  if (!it_out || !st_out) {
    TRY(ensure(g.iters, (M + n_ops) * (size_t)(L + 1) * sizeof(int32_t)));
    if (!it_out) it_out = (int32_t*)g.iters.p;
    if (!st_out) st_out = (int32_t*)g.iters.p + (M + n_ops) * (size_t)L;
  }
  auto node_ptr = [&](int nd) -> float* {
    if (nd < M) return pair + (size_t)nd * nf;
    const PlanOp& q = plan[nd - M];
    if (q.i == 0) return phi0 + (size_t)(q.k - 1) * nf;
    return (float*)g.nodes.p + (size_t)slot_of[nd] * nf;
  };

  std::vector<TaskDesc> tasks(M + n_ops);
  for (int k = 1; k <= M; ++k) {
    TaskDesc& d = tasks[k - 1];
    d.ref = k - 1;
    d.tmpl = k;
    d.kind = 0;
    d.pad = 0;
    d.ua = d.ub = nullptr;
    d.out = pair + (size_t)(k - 1) * nf;
    d.iters = it_out + (size_t)(k - 1) * L;
    d.status = st_out + (k - 1);
  }
  for (size_t n = 0; n < n_ops; ++n) {
    const PlanOp& q = plan[n];
    TaskDesc& d = tasks[M + n];
    d.ref = q.i;
    d.tmpl = q.k;
    d.kind = 1;
    d.pad = 0;
    d.ua = node_ptr(q.a);
    d.ub = node_ptr(q.b);
    d.out = node_ptr(q.out);
    d.iters = it_out + (M + n) * (size_t)L;
    d.status = st_out + (M + n);
  }
  const bool use_graph = (flags & SCAN_F_GRAPH) && mode != REG_PLAIN;
  char keybuf[512];
  snprintf(keybuf, sizeof keybuf, "%p %p %p %p %p %d %d %d %d %d %d %.17g %.17g %.17g %d %d %d %d %d %d %d",
           (const void*)frames, (void*)phi0, (void*)pair, (void*)it_out, (void*)st_out, N, H, W, p->levels,
           p->max_iter, p->fixed_iter, p->tau, p->lambda, p->rel_tol, algo, chunk, global_algo, mode,
           g.tile_rows, g.max_group, (int)g.resident);
  const std::string key(keybuf);
  if (use_graph) {
    // graphs whose workspace has moved can never be replayed: free them
    for (size_t q = 0; q < g.graphs.size();) {
      if (g.graphs[q].generation != g.generation) {
        (void)hipGraphExecDestroy(g.graphs[q].exec);
        if (g.graphs[q].tasks.p) (void)hipFree(g.graphs[q].tasks.p);
        if (g.graphs[q].flow.p) (void)hipFree(g.graphs[q].flow.p);
        g.graphs.erase(g.graphs.begin() + q);
      } else {
        ++q;
      }
    }
    for (auto& gr : g.graphs) {
      if (gr.key == key && gr.generation == g.generation) {
        // timing: one event pair around the whole replay (event records
        // captured inside a graph are not re-recorded when it is replayed)
        g.events_used = 0;
        hipEvent_t* ev = next_events();
        if (ev) HIPCHK(hipEventRecord(ev[0], s));
        HIPCHK(hipGraphLaunch(gr.exec, s));
        if (ev) HIPCHK(hipEventRecord(ev[1], s));
        return REG_OK;
      }
    }
  }

  TRY(upload_tasks(g.tasks, tasks, s));
  const size_t T = M + n_ops;
  size_t flow_used = 0;
  if (mode == REG_DATAFLOW) {
    // task index == node id: A task k-1 produces node k-1, op n produces M + n
    std::vector<int> host(3 * T + 1 + 2 * n_ops);
    int* deps0 = host.data();
    int* ready0 = deps0 + T;
    int* cons_off = ready0 + T;
    int* cons = cons_off + T + 1;
    std::vector<int> cnt(T, 0);
    for (size_t t = 0; t < T; ++t) {
      deps0[t] = (int)t < M ? 0 : 2;
      ready0[t] = (int)t < M ? (int)t : -1;
    }
    for (const PlanOp& q : plan) {
      cnt[q.a]++;
      cnt[q.b]++;
    }
    cons_off[0] = 0;
    for (size_t t = 0; t < T; ++t) cons_off[t + 1] = cons_off[t] + cnt[t];
    std::vector<int> fill(cons_off, cons_off + T);
    for (size_t n = 0; n < n_ops; ++n) {
      cons[fill[plan[n].a]++] = (int)(M + n);
      cons[fill[plan[n].b]++] = (int)(M + n);
    }
    flow_used = host.size();   // deps0, ready0, cons_off, cons; then deps, ready
    TRY(ensure(g.flow, (flow_used + 2 * T) * sizeof(int)));
    HIPCHK(hipMemcpyAsync(g.flow.p, host.data(), flow_used * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }

  // every launch of the run; graph capture records exactly these
  auto enqueue = [&](hipStream_t st, const TaskDesc* d_tasks, int* dflow, bool timed) -> int {
    if (mode != REG_PLAIN) HIPCHK(launch_note_abort((const int*)g.abortw.p, (int*)g.abortw.p, true, st));
    Pyr P;
    TRY(build_pyramid(frames, N, H, W, L, P, st));
    SolveArgs a = base_args(P, H, W, p);
    if (mode == REG_DATAFLOW) {
      TRY(run_dataflow(a, d_tasks, (int)T, dflow + flow_used, dflow, dflow + flow_used + T, dflow + T, M,
                       dflow + 2 * T, dflow + 3 * T + 1, st, timed));
      HIPCHK(launch_copy(pair, phi0, nf, st));
    } else if (mode == REG_BATCHED) {
      TRY(run_batched(a, d_tasks, M, st, timed));
      HIPCHK(launch_copy(pair, phi0, nf, st));
      size_t q = 0;
      for (int lvl = 1; lvl <= n_levels; ++lvl) {
        const size_t q0 = q;
        while (q < n_ops && plan[q].level == lvl) ++q;
        TRY(run_batched(a, d_tasks + M + q0, (int)(q - q0), st, timed));
      }
    } else {
      std::vector<TaskDesc> A(tasks.begin(), tasks.begin() + M);
      TRY(run_plain(a, A, d_tasks, st));
      HIPCHK(launch_copy(pair, phi0, nf, st));
      for (size_t n = 0; n < n_ops; ++n) {
        std::vector<TaskDesc> one{tasks[M + n]};
        TRY(run_plain(a, one, d_tasks + M + n, st));
      }
    }
    return REG_OK;
  };

  g.events_used = 0;
  TRY(enqueue(s, (const TaskDesc*)g.tasks.p, (int*)g.flow.p, true));
  if (mode != REG_PLAIN) TRY(check_abort(s, "the scan"));
  if (!use_graph) return REG_OK;

  // capture the same launches into a graph that owns copies of the descriptors
  HIPCHK(hipStreamSynchronize(s));
  const unsigned gen = g.generation;
  State::Graph gr;
  gr.key = key;
  gr.exec = nullptr;
  if (hipMalloc(&gr.tasks.p, T * sizeof(TaskDesc)) != hipSuccess) return fail(REG_E_NOMEM, "graph descriptors");
  gr.tasks.n = T * sizeof(TaskDesc);
  HIPCHK(hipMemcpy(gr.tasks.p, g.tasks.p, gr.tasks.n, hipMemcpyDeviceToDevice));
  if (mode == REG_DATAFLOW) {
    gr.flow.n = (flow_used + 2 * T) * sizeof(int);
    if (hipMalloc(&gr.flow.p, gr.flow.n) != hipSuccess) return fail(REG_E_NOMEM, "graph dataflow arrays");
    HIPCHK(hipMemcpy(gr.flow.p, g.flow.p, gr.flow.n, hipMemcpyDeviceToDevice));
  }
  hipStream_t cs;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  const size_t direct_events = g.events_used;   // the direct run's launches stay the last call's timing
  const int rc = enqueue(cs, (const TaskDesc*)gr.tasks.p, (int*)gr.flow.p, false);
  g.events_used = direct_events;
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (rc != REG_OK) return rc;
  if (ec != hipSuccess) return fail(REG_E_HIP, "graph capture failed: %s", hipGetErrorString(ec));
  if (g.generation != gen) return fail(REG_E_HIP, "workspace moved during graph capture");
  const hipError_t ei = hipGraphInstantiate(&gr.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return fail(REG_E_HIP, "graph instantiation failed: %s", hipGetErrorString(ei));
  gr.generation = gen;
  g.graphs.push_back(gr);
  return REG_OK;
}

int reg_last_solve_launch_ms(double* ms, int cap, int* n) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (cap < 0 || (cap > 0 && !ms)) return fail(REG_E_INVALID, "launch_ms: cap %d with output %p", cap, (void*)ms);
  for (size_t q = 0; q < g.events_used && (int)q < cap; ++q) {
    HIPCHK(hipEventSynchronize(g.events[q].second));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, g.events[q].first, g.events[q].second));
    ms[q] = t;
  }
  if (n) *n = (int)g.events_used;
  return REG_OK;
}

int reg_last_solve_timing(double* total_ms, int* launches) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  double tot = 0.0;
  for (size_t q = 0; q < g.events_used; ++q) {
    HIPCHK(hipEventSynchronize(g.events[q].second));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, g.events[q].first, g.events[q].second));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int)g.events_used;
  return REG_OK;
}

int reg_set_tuning(int tile_rows, int max_group, int resident) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (tile_rows != 0 && (tile_rows < 4 || tile_rows > 64 || tile_rows % 4))
    return fail(REG_E_INVALID, "tile_rows %d must be a multiple of 4 in [4, 64]", tile_rows);
  if (max_group != 0 && (max_group < 1 || max_group > kMaxGroup))
    return fail(REG_E_INVALID, "max_group %d must be in [1, %d]", max_group, kMaxGroup);
  if (resident < -1 || resident > 1) return fail(REG_E_INVALID, "resident %d must be -1, 0 or 1", resident);
  if (tile_rows) g.tile_rows = tile_rows;
  if (max_group) g.max_group = max_group;
  if (resident >= 0) g.resident = resident != 0;
  return REG_OK;
}

int reg_autotune(int H, int W, int levels, int batch, int* tile_rows, int* max_group, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(batch, H, W));
  if (batch < 1) return fail(REG_E_INVALID, "batch %d < 1", batch);
  reg_params_t p{levels, 20, 1, 0.5, 0.1, 1e-5};
  TRY(check_params(&p, H, W));
  TRY(ensure_device());
  hipStream_t s = (hipStream_t)stream;
  const long long key = ((long long)H << 40) ^ ((long long)W << 20) ^ ((long long)levels << 16) ^ batch;
  auto hit = g.tuned.find(key);
  if (hit == g.tuned.end()) {
    // synthetic lattice frames and a batch of pairwise registrations, timed
    // with a fixed iteration count for every candidate
    const int F = batch + 1;
    const size_t nf = (size_t)2 * H * W;
    DevBuf frames, u;
    if (hipMalloc(&frames.p, (size_t)F * H * W * sizeof(float)) != hipSuccess ||
        hipMalloc(&u.p, (size_t)batch * nf * sizeof(float)) != hipSuccess) {
      if (frames.p) (void)hipFree(frames.p);
      return fail(REG_E_NOMEM, "autotune buffers");
    }
    HIPCHK(launch_synth_frames((float*)frames.p, F, H, W, s));
    std::vector<int32_t> ref(batch), tmpl(batch);
    for (int b = 0; b < batch; ++b) {
      ref[b] = b;
      tmpl[b] = b + 1;
    }
    const int saved_th = g.tile_rows, saved_mg = g.max_group;
    double best = 1e300;
    int best_th = saved_th, best_mg = saved_mg;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int rc = REG_OK;
    for (int th : {16, 32, 64}) {
      if (th > H) continue;
      for (int mg : {1, 4, 8, 16, 32, 64, 128}) {
        g.tile_rows = th;
        g.max_group = mg;
        float ms = 0.f;
        for (int rep = 0; rep < 2 && rc == REG_OK; ++rep) {   // first run warms up
          (void)hipEventRecord(e0, s);
          rc = reg_solve_batch((const float*)frames.p, F, H, W, ref.data(), tmpl.data(), nullptr, (float*)u.p,
                               nullptr, nullptr, batch, &p, REG_BATCHED, stream);
          (void)hipEventRecord(e1, s);
          (void)hipEventSynchronize(e1);
          (void)hipEventElapsedTime(&ms, e0, e1);
        }
        if (rc != REG_OK) break;
        if (ms < best) {
          best = ms;
          best_th = th;
          best_mg = mg;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(frames.p);
    (void)hipFree(u.p);
    g.tile_rows = saved_th;
    g.max_group = saved_mg;
    if (rc != REG_OK) return rc;
    hit = g.tuned.emplace(key, std::make_pair(best_th, best_mg)).first;
  }
  g.tile_rows = hit->second.first;
  g.max_group = hit->second.second;
  if (tile_rows) *tile_rows = g.tile_rows;
  if (max_group) *max_group = g.max_group;
  return REG_OK;
}

int scan_run_flex(const float* frames, int N, int H, int W, const reg_params_t* p, int workers, int global_algo,
                  float* phi0, float* u_pair, int32_t* seg_out, int32_t* step_out, int64_t* counts, double* ms,
                  void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(1, H, W));
  TRY(check_params(p, H, W));
  if (N < 3) return fail(REG_E_INVALID, "a flexible-segment scan needs N >= 3 frames (got %d)", N);
  const int M = N - 1;
  if (workers < 2 || workers > M) return fail(REG_E_INVALID, "workers %d not in [2, %d]", workers, M);
  if (global_algo < SCAN_SEQ || global_algo > SCAN_BRENT_KUNG)
    return fail(REG_E_INVALID, "unknown global algorithm %d", global_algo);
  if (!frames || !phi0) return fail(REG_E_INVALID, "NULL pointer");
  TRY(ensure_device());
  hipStream_t s = (hipStream_t)stream;
  const int L = p->levels;
  const size_t nf = (size_t)2 * H * W;
  const int slots = g.blocks_per_cu * g.n_cu;
  const int groups = (workers + 7) / 8 * 8;
  if (groups > slots) return fail(REG_E_INVALID, "%d workers exceed the %d resident workgroups", workers, slots);
  int gs = group_size(workers, H, W, false);
  while (gs > 1 && (long long)groups * gs > slots) gs /= 2;

  float* pair = u_pair;
  if (!pair) {
    TRY(ensure(g.upair, (size_t)M * nf * sizeof(float)));
    pair = (float*)g.upair.p;
  }
  // worker state
  const size_t ws_bytes = 256 * 16 + (size_t)workers * (8 + 4 + 4 + 16) + (size_t)M * (4 + 4 * L + 4) +
                          (size_t)workers * 64 + (size_t)workers * 2 * nf * sizeof(float);
  TRY(ensure(g.flexw, ws_bytes));
  MockBuf mb{(char*)g.flexw.p};
  unsigned long long* gaps = mb.take<unsigned long long>(workers);
  float* rates = mb.take<float>(workers);
  int* starts = mb.take<int>(workers);
  int* seg = mb.take<int>(4 * (size_t)workers);
  int* step = mb.take<int>(M);
  int* eiters = mb.take<int>((size_t)M * L);
  int* estatus = mb.take<int>(M);
  unsigned long long* desc = mb.take<unsigned long long>(8 * (size_t)workers);
  float* fbuf = mb.take<float>((size_t)workers * 2 * nf);

  std::vector<int> hstart(workers);
  for (int w = 0; w < workers; ++w) {
    const int s0 = (int)((long long)w * M / workers), s1 = (int)((long long)(w + 1) * M / workers);
    hstart[w] = w == 0 ? 0 : w == workers - 1 ? M - 1 : (s0 + s1 - 1) / 2;
  }
  std::vector<unsigned long long> hgap(workers, 0);
  for (int w = 0; w + 1 < workers; ++w)
    hgap[w] = (unsigned long long)(unsigned)(hstart[w] + 1) | ((unsigned long long)(unsigned)(hstart[w + 1] - 1) << 32);
  std::vector<float> hrate(workers, 0.f);
  std::vector<int> hzero(M, 0);
  HIPCHK(hipMemcpyAsync(gaps, hgap.data(), workers * sizeof(unsigned long long), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(rates, hrate.data(), workers * sizeof(float), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(starts, hstart.data(), workers * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(step, hzero.data(), M * sizeof(int), hipMemcpyHostToDevice, s));

  hipEvent_t ev[4];
  for (int i = 0; i < 4; ++i) HIPCHK(hipEventCreate(&ev[i]));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};

  // pairwise registrations, one batch
  Pyr P;
  TRY(build_pyramid(frames, N, H, W, L, P, s));
  SolveArgs a = base_args(P, H, W, p);
  std::vector<TaskDesc> tasks(M);
  for (int k = 1; k <= M; ++k) {
    TaskDesc& d = tasks[k - 1];
    d.ref = k - 1;
    d.tmpl = k;
    d.kind = 0;
    d.pad = 0;
    d.ua = d.ub = nullptr;
    d.out = pair + (size_t)(k - 1) * nf;
    d.iters = nullptr;
    d.status = nullptr;
  }
  TRY(upload_tasks(g.tasks, tasks, s));
  HIPCHK(hipEventRecord(ev[0], s));
  TRY(run_batched(a, (const TaskDesc*)g.tasks.p, M, s, false));
  HIPCHK(launch_copy(pair, phi0, nf, s));   // phi_{0,1} = u_{0,1}
  HIPCHK(hipEventRecord(ev[1], s));

  // phase 1: flexible segments, one group per worker
  {
    SolveArgs f = a;
    const int ctrl_ints = kCtrlHead + kCtrlGroup * groups;
    TRY(ensure(g.ctrl, (size_t)ctrl_ints * sizeof(int)));
    f.max_tiles = std::max(f.max_tiles, gs);
    TRY(ensure(g.part, (size_t)groups * 3 * f.max_tiles * sizeof(double)));
    TRY(ensure(g.slots, (size_t)groups * f.slot_floats * sizeof(float)));
    f.tasks = nullptr;
    f.n_tasks = 0;
    f.g = gs;
    f.ctrl = (int*)g.ctrl.p;
    f.part = (double*)g.part.p;
    f.ws = (float*)g.slots.p;
    f.flex = 1;
    f.flex_workers = workers;
    f.flex_M = M;
    f.gaps = gaps;
    f.rates = rates;
    f.starts = starts;
    f.flex_buf = fbuf;
    f.elem = pair;
    f.phi0 = phi0;
    f.flex_seg = seg;
    f.elem_step = step;
    f.elem_iters = eiters;
    f.elem_status = estatus;
    f.flex_desc = desc;
    HIPCHK(launch_reset_ctrl(f.ctrl, ctrl_ints, s));
    HIPCHK(launch_persistent(f, groups * gs, s));
  }
  HIPCHK(hipEventRecord(ev[2], s));
  std::vector<int> hseg(4 * (size_t)workers);
  HIPCHK(hipMemcpyAsync(hseg.data(), seg, hseg.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  std::vector<int> hstep(M);
  HIPCHK(hipMemcpyAsync(hstep.data(), step, M * sizeof(int), hipMemcpyDeviceToHost, s));
  int h_abort = 0;
  HIPCHK(hipMemcpyAsync(&h_abort, (int*)g.ctrl.p + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h_abort) return fail(REG_E_HIP, "phase 1 abandoned by the forward-progress watchdog");
  for (int w = 0; w < workers; ++w) {
    const int pl = hseg[4 * w], pr = hseg[4 * w + 1];
    if (pl > pr || (w == 0 && pl != 0) || (w + 1 == workers && pr != M - 1) ||
        (w > 0 && hseg[4 * (w - 1) + 1] + 1 != pl))
      return fail(REG_E_HIP, "phase 1 left an invalid segment %d: [%d, %d]", w, pl, pr);
  }

  // global scan of the segment totals and the rescans, one dataflow launch
  std::vector<PlanOp> plan;
  int n_levels = 0;
  if (rs::build_plan(workers, global_algo, 0, global_algo, plan, n_levels) != 0)
    return fail(REG_E_INVALID, "invalid global plan");
  const int n2 = (int)plan.size();
  auto pl_of = [&](int w) { return hseg[4 * w]; };
  auto pr_of = [&](int w) { return hseg[4 * w + 1]; };
  std::vector<const float*> node(workers + n2, nullptr);
  for (int w = 0; w < workers; ++w) {
    const int ops = hseg[4 * w + 2];
    if (ops == 0) node[w] = pair + (size_t)hstart[w] * nf;
    else if (w == 0) node[w] = phi0 + (size_t)pr_of(0) * nf;
    else node[w] = fbuf + ((size_t)w * 2 + ((ops - 1) & 1)) * nf;
  }
  int n_pool = 0;
  for (const PlanOp& q : plan)
    if (q.i != 0) ++n_pool;
  TRY(ensure(g.flexn, std::max<size_t>(1, (size_t)n_pool) * nf * sizeof(float)));
  std::vector<TaskDesc> t2;
  std::vector<std::vector<int>> dep;
  std::vector<int> prefix_task(workers, -1);   // task producing phi0[pr_w] (prefix over segments 0..w)
  int pool = 0;
  for (int n = 0; n < n2; ++n) {
    const PlanOp& q = plan[n];
    TaskDesc d;
    d.ref = pl_of(q.i);
    d.tmpl = pr_of(q.k - 1) + 1;
    d.kind = 1;
    d.pad = 0;
    d.ua = node[q.a];
    d.ub = node[q.b];
    float* out = q.i == 0 ? phi0 + (size_t)pr_of(q.k - 1) * nf : (float*)g.flexn.p + (size_t)pool++ * nf;
    d.out = out;
    d.iters = nullptr;
    d.status = nullptr;
    node[q.out] = out;
    if (q.i == 0) prefix_task[q.k - 1] = n;
    std::vector<int> dl;
    for (int in : {q.a, q.b})
      if (in >= workers) dl.push_back(in - workers);
    t2.push_back(d);
    dep.push_back(dl);
  }
  int n3 = 0;
  for (int w = 1; w < workers; ++w) {
    int prev = prefix_task[w - 1];   // -1: phi0[pl_w - 1] exists already (worker 0)
    for (int e = pl_of(w); e < pr_of(w); ++e) {
      TaskDesc d;
      d.ref = 0;
      d.tmpl = e + 1;
      d.kind = 1;
      d.pad = 0;
      d.ua = phi0 + (size_t)(e - 1) * nf;
      d.ub = pair + (size_t)e * nf;
      d.out = phi0 + (size_t)e * nf;
      d.iters = nullptr;
      d.status = nullptr;
      std::vector<int> dl;
      if (prev >= 0) dl.push_back(prev);
      prev = (int)t2.size();
      t2.push_back(d);
      dep.push_back(dl);
      ++n3;
    }
  }
  const int T = (int)t2.size();
  if (T > 0) {
    const TaskFlow tf = task_flow(dep);
    TRY(upload_tasks(g.flext, t2, s));
    TRY(ensure(g.flexf, (tf.host.size() + 2 * (size_t)T) * sizeof(int)));
    HIPCHK(hipMemcpyAsync(g.flexf.p, tf.host.data(), tf.host.size() * sizeof(int), hipMemcpyHostToDevice, s));
    int* fl = (int*)g.flexf.p;
    int* deps = fl + tf.host.size();
    TRY(run_dataflow(a, (const TaskDesc*)g.flext.p, T, deps, fl, deps + T, fl + T, tf.n_ready0, fl + 2 * T,
                     fl + 3 * T + 1, s, false));
  }
  HIPCHK(hipEventRecord(ev[3], s));
  HIPCHK(hipStreamSynchronize(s));
  int h_abort2 = 0;
  HIPCHK(hipMemcpy(&h_abort2, (int*)g.ctrl.p + 1, sizeof(int), hipMemcpyDeviceToHost));
  if (h_abort2) return fail(REG_E_HIP, "global phase abandoned by the forward-progress watchdog");
  if (seg_out)
    for (size_t i = 0; i < hseg.size(); ++i) seg_out[i] = hseg[i];
  if (step_out)
    for (int e = 0; e < M; ++e) step_out[e] = hstep[e];
  if (counts) {
    counts[0] = M - workers;
    counts[1] = n2;
    counts[2] = n3;
    counts[3] = M + (M - workers) + n2 + n3;
  }
  if (ms) {
    float t01 = 0, t12 = 0, t23 = 0;
    HIPCHK(hipEventElapsedTime(&t01, ev[0], ev[1]));
    HIPCHK(hipEventElapsedTime(&t12, ev[1], ev[2]));
    HIPCHK(hipEventElapsedTime(&t23, ev[2], ev[3]));
    ms[0] = t01;
    ms[1] = t12;
    ms[2] = t23;
    ms[3] = (double)t01 + t12 + t23;
  }
  return REG_OK;
}

}  // extern "C"

// ------------------------------------------------------------ rigid operator

namespace {

// Device arrays of a dataflow run (see SolveArgs): initial dependency counts
// and ready queue, the consumers of every task, and the working copies.
struct RigidFlow {
  int* deps;
  const int* deps0;
  int* ready;
  const int* ready0;
  const int* cons_off;
  const int* cons;
  int n_ready0;
};

// Runs n rigid registrations (device descriptors) with one persistent launch:
// groups of g workgroups on one XCD.  Level-synchronous: g the largest power
// of two <= 16 that keeps a group per task (rounded up to 8) resident.
// Dataflow: the number of ready registrations varies over the run and the
// slowest ones set its end, so g is sized for the registration instead:
// about 32 fine-level pixels per thread and pass (at 256x256, g = 8 measured
// as fast as g = 4 and a third faster than g = 16), all slots filled.
constexpr int kRigidPixelsPerThread = 32;

int run_rigid(RigidArgs a, const RigidTask* d_tasks, int n, const RigidFlow* f, hipStream_t s) {
  if (n == 0) return REG_OK;
  if (!g.rigid_blocks_per_cu) {
    int nb = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, rigid_kernel(), kWG, 0));
    if (nb < 1) return fail(REG_E_HIP, "rigid kernel cannot be resident");
    g.rigid_blocks_per_cu = nb;
  }
  const int slots = g.rigid_blocks_per_cu * g.n_cu;
  const int want = (n + 7) / 8 * 8;
  int gs = 1;
  if (f)
    while (gs * 2 <= kRigidMaxGroup && (long long)a.H * a.W >= (long long)gs * 2 * kWG * kRigidPixelsPerThread &&
           8 * gs * 2 <= slots)
      gs *= 2;
  else
    while (gs * 2 <= kRigidMaxGroup && (long long)want * gs * 2 <= slots) gs *= 2;
  int groups = std::max(8, slots / gs / 8 * 8);
  if (!f) groups = std::min(want, groups);
  const int ctrl_ints = kCtrlHead + kCtrlGroup * groups;
  TRY(ensure(g.rctrl, (size_t)ctrl_ints * sizeof(int)));
  const int n_slots = groups * 3 * kRigidSlotBuf;
  TRY(ensure(g.rpart, (size_t)n_slots * sizeof(double)));
  a.tasks = d_tasks;
  a.n_tasks = n;
  a.g = gs;
  a.ctrl = (int*)g.rctrl.p;
  a.part = (double*)g.rpart.p;
  a.spin_limit = g.spin_limit;
  HIPCHK(launch_reset_rigid(a.ctrl, ctrl_ints, d_tasks, n, (unsigned long long*)a.part, n_slots, s));
  if (f) {
    a.dataflow = 1;
    a.deps = f->deps;
    a.ready = f->ready;
    a.cons_off = f->cons_off;
    a.cons = f->cons;
    HIPCHK(launch_reset_dataflow(f->deps, f->deps0, f->ready, f->ready0, n, a.ctrl, f->n_ready0, s));
  }
  hipEvent_t* ev = next_events();
  if (ev) HIPCHK(hipEventRecord(ev[0], s));
  HIPCHK(launch_rigid(a, groups * gs, s));
  if (ev) HIPCHK(hipEventRecord(ev[1], s));
  return REG_OK;
}

RigidArgs rigid_args(const Pyr& P, int H, int W, const reg_params_t* p) {
  RigidArgs a;
  std::memset(&a, 0, sizeof a);
  for (int l = 0; l < p->levels; ++l) {
    a.pyr[l] = P.lv[l];
    a.fstride[l] = P.fstride[l];
    a.pitch[l] = P.pitch[l];
  }
  a.H = H;
  a.W = W;
  a.levels = p->levels;
  a.max_iter = p->max_iter;
  a.fixed_iter = p->fixed_iter ? 1 : 0;
  a.tau = p->tau;
  a.rel_tol = p->rel_tol;
  return a;
}

int upload_rigid(const std::vector<RigidTask>& t, hipStream_t s) {
  TRY(ensure(g.rtasks, t.size() * sizeof(RigidTask)));
  HIPCHK(hipMemcpyAsync(g.rtasks.p, t.data(), t.size() * sizeof(RigidTask), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));   // the host vector may go out of scope
  return REG_OK;
}

}  // namespace

extern "C" {

int reg_rigid_solve_batch(const float* frames, int N, int H, int W, const int32_t* ref_idx, const int32_t* tmpl_idx,
                          const double* theta0, double* theta, int32_t* iters, int32_t* status, int B,
                          const reg_params_t* p, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(B, H, W));
  TRY(check_params(p, H, W));
  if (N < 1) return fail(REG_E_INVALID, "N = %d frames", N);
  if (B == 0) return REG_OK;
  if (!frames || !ref_idx || !tmpl_idx || !theta) return fail(REG_E_INVALID, "NULL pointer");
  if (theta0 && theta0 == theta) return fail(REG_E_INVALID, "theta aliases theta0");
  for (int b = 0; b < B; ++b)
    if (ref_idx[b] < 0 || ref_idx[b] >= N || tmpl_idx[b] < 0 || tmpl_idx[b] >= N)
      return fail(REG_E_INVALID, "frame index out of range at item %d", b);
  TRY(ensure_device());
  hipStream_t s = (hipStream_t)stream;
  Pyr P;
  TRY(build_pyramid(frames, N, H, W, p->levels, P, s));
  std::vector<RigidTask> tasks(B);
  for (int b = 0; b < B; ++b) {
    RigidTask& d = tasks[b];
    d.ref = ref_idx[b];
    d.tmpl = tmpl_idx[b];
    d.kind = theta0 ? 2 : 0;
    d.pad = 0;
    d.ta = theta0 ? theta0 + 3 * b : nullptr;
    d.tb = nullptr;
    d.out = theta + 3 * b;
    d.iters = iters ? iters + (size_t)b * p->levels : nullptr;
    d.status = status ? status + b : nullptr;
  }
  TRY(upload_rigid(tasks, s));
  g.events_used = 0;
  return run_rigid(rigid_args(P, H, W, p), (const RigidTask*)g.rtasks.p, B, nullptr, s);
}

int scan_run_rigid(const float* frames, int N, int H, int W, const reg_params_t* p, int algo, int chunk,
                   int global_algo, int mode, double* phi0, double* pairs, int32_t* op_iters, int32_t* status,
                   void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  TRY(check_dims(1, H, W));
  TRY(check_params(p, H, W));
  if (N < 2) return fail(REG_E_INVALID, "a series needs N >= 2 frames (got %d)", N);
  if (!frames || !phi0) return fail(REG_E_INVALID, "NULL pointer");
  if (mode != REG_BATCHED && mode != REG_DATAFLOW) return fail(REG_E_INVALID, "mode %d: REG_BATCHED or REG_DATAFLOW", mode);
  if (algo < SCAN_SEQ || algo > SCAN_HIER) return fail(REG_E_INVALID, "unknown scan algorithm %d", algo);
  if (algo == SCAN_HIER && (global_algo < SCAN_SEQ || global_algo > SCAN_BRENT_KUNG))
    return fail(REG_E_INVALID, "unknown global algorithm %d", global_algo);
  const int M = N - 1;
  std::vector<PlanOp> plan;
  int n_levels = 0;
  try {
    if (rs::build_plan(M, algo, chunk, global_algo, plan, n_levels) != 0)
      return fail(REG_E_INVALID, "invalid plan arguments");
  } catch (const std::exception& e) {
    return fail(REG_E_INVALID, "plan construction failed: %s", e.what());
  }
  TRY(ensure_device());
  hipStream_t s = (hipStream_t)stream;
  const int L = p->levels;
  const size_t n_ops = plan.size();
  // node parameters: elements in `pairs` (or workspace), every op output in
  // workspace, except that an op yielding a prefix (0, k) writes phi0[k - 1]
  const std::vector<int> fin = final_nodes(plan, M);
  for (int k = 1; k < M; ++k)
    if (fin[k] < M) return fail(REG_E_INVALID, "plan yields no prefix (0, %d)", k + 1);
  TRY(ensure(g.rnodes, (size_t)(M + n_ops) * 3 * sizeof(double)));
  double* ws = (double*)g.rnodes.p;
  std::vector<double*> node(M + n_ops);
  for (int m = 0; m < M; ++m) node[m] = (pairs ? pairs : ws) + 3 * m;
  for (size_t q = 0; q < n_ops; ++q) node[M + q] = ws + 3 * (M + q);
  for (int k = 1; k < M; ++k) node[fin[k]] = phi0 + 3 * k;
  Pyr P;
  TRY(build_pyramid(frames, N, H, W, L, P, s));
  std::vector<RigidTask> tasks(M + n_ops);
  std::vector<int> level_of(M + n_ops, 0);
  for (int m = 0; m < M; ++m) {
    RigidTask& d = tasks[m];
    d = RigidTask{m, m + 1, 0, 0, nullptr, nullptr, node[m], nullptr, nullptr};
  }
  for (size_t q = 0; q < n_ops; ++q) {
    const PlanOp& o = plan[q];
    RigidTask& d = tasks[M + q];
    d = RigidTask{o.i, o.k, 1, 0, node[o.a], node[o.b], node[o.out], nullptr, nullptr};
    level_of[M + q] = o.level;
  }
  for (size_t t = 0; t < tasks.size(); ++t) {
    tasks[t].iters = op_iters ? op_iters + t * L : nullptr;
    tasks[t].status = status ? status + t : nullptr;
  }
  const RigidArgs a = rigid_args(P, H, W, p);
  g.events_used = 0;
  if (mode == REG_DATAFLOW) {
    // one launch over the whole DAG: task id = node id (pairwise tasks are the
    // elements, op q yields node M + q)
    std::vector<std::vector<int>> dep(tasks.size());
    for (size_t q = 0; q < n_ops; ++q) dep[M + q] = {plan[q].a, plan[q].b};
    const TaskFlow tf = task_flow(dep);
    const size_t T = tasks.size();
    TRY(upload_rigid(tasks, s));
    TRY(ensure(g.rflow, (tf.host.size() + 2 * T) * sizeof(int)));
    HIPCHK(hipMemcpyAsync(g.rflow.p, tf.host.data(), tf.host.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));   // tf is host memory of this scope
    const int* fl = (const int*)g.rflow.p;
    int* work = (int*)g.rflow.p + tf.host.size();
    const RigidFlow f{work, fl, work + T, fl + T, fl + 2 * T, fl + 3 * T + 1, tf.n_ready0};
    TRY(run_rigid(a, (const RigidTask*)g.rtasks.p, (int)T, &f, s));
  } else {
    // device descriptors grouped by level (stable), one launch per level
    std::vector<int> order(tasks.size());
    for (size_t t = 0; t < order.size(); ++t) order[t] = (int)t;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return level_of[x] < level_of[y]; });
    std::vector<RigidTask> sorted(tasks.size());
    for (size_t t = 0; t < order.size(); ++t) sorted[t] = tasks[order[t]];
    TRY(upload_rigid(sorted, s));
    size_t first = 0;
    while (first < sorted.size()) {
      size_t last = first;
      while (last < sorted.size() && level_of[order[last]] == level_of[order[first]]) ++last;
      TRY(run_rigid(a, (const RigidTask*)g.rtasks.p + first, (int)(last - first), nullptr, s));
      first = last;
    }
  }
  HIPCHK(hipMemcpyAsync(phi0, node[0], 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  return REG_OK;
}

}  // extern "C"

extern "C" {

int scan_mock_run(int M, int algo, int chunk, int global_algo, int mode, int workers, const mock_params_t* p,
                  int32_t* prefix, int32_t* seg_out, int64_t* counts, double* ms, void* stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (M < 1) return fail(REG_E_INVALID, "M = %d < 1", M);
  if (!p) return fail(REG_E_INVALID, "params is NULL");
  if (!(p->mean_us >= 0.0) || !(p->mean_us <= 1e6)) return fail(REG_E_INVALID, "mean_us must be in [0, 1e6]");
  if (p->dist != MOCK_STATIC_TIME && p->dist != MOCK_EXP_TIME && p->dist != MOCK_FRAME_TIME)
    return fail(REG_E_INVALID, "unknown dist %d", p->dist);
  if (mode < MOCK_LEVEL_STATIC || mode > MOCK_FLEX) return fail(REG_E_INVALID, "unknown mode %d", mode);
  if (!prefix) return fail(REG_E_INVALID, "prefix is NULL");
  if (workers < 1) return fail(REG_E_INVALID, "workers = %d < 1", workers);
  const bool segs = mode == MOCK_SEGMENTS || mode == MOCK_FLEX;
  if (segs && workers > M) return fail(REG_E_INVALID, "%d workers for %d elements", workers, M);
  if (mode == MOCK_FLEX && workers < 2) return fail(REG_E_INVALID, "work stealing needs >= 2 workers");
  if (segs && (global_algo < SCAN_SEQ || global_algo > SCAN_BRENT_KUNG))
    return fail(REG_E_INVALID, "unknown global algorithm %d", global_algo);
  TRY(ensure_device());
  int per_cu = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mock_worker_kernel(), 64, 0));
  const int capacity = per_cu * g.n_cu;
  if (workers > capacity)
    return fail(REG_E_INVALID, "%d workers exceed the %d wavefronts that can be resident", workers, capacity);
  int khz = 0;
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g.device));
  if (khz <= 0) return fail(REG_E_HIP, "wall-clock rate unavailable");
  hipStream_t s = (hipStream_t)stream;

  // the plan: the whole scan (level modes) or the global phase over the workers
  std::vector<PlanOp> plan;
  int n_levels = 0;
  const int n_base = segs ? workers : M;
  try {
    if (rs::build_plan(n_base, segs ? global_algo : algo, segs ? 0 : chunk, global_algo, plan, n_levels) != 0)
      return fail(REG_E_INVALID, "invalid plan arguments");
  } catch (const std::exception& e) {
    return fail(REG_E_INVALID, "plan construction failed: %s", e.what());
  }
  const int n_ops = (int)plan.size();
  const size_t n_nodes = (size_t)n_base + n_ops;
  TRY(ensure(g.mock, mock_bytes(n_nodes, n_ops, n_base, n_levels, workers)));
  MockBuf mb{(char*)g.mock.p};
  int* err = mb.take<int>(8);
  int2* nodes = mb.take<int2>(n_nodes);
  MockOp* d_ops = mb.take<MockOp>(n_ops);
  int* d_fin = mb.take<int>(n_base);
  int* tickets = mb.take<int>(n_levels + 1);
  int* deps = mb.take<int>(n_ops);
  int* ready = mb.take<int>(n_ops);
  int* flowbuf = mb.take<int>(3 * (size_t)n_ops + 1 + 2 * (size_t)n_ops);   // deps0, ready0, cons_off, cons
  int* ctrl = mb.take<int>(8);
  unsigned long long* gaps = mb.take<unsigned long long>(workers);
  float* rate = mb.take<float>(workers);
  int2* total = mb.take<int2>(workers);
  int2* seg = seg_out ? (int2*)seg_out : mb.take<int2>(workers);
  int2* gpre = mb.take<int2>(workers);

  std::vector<MockOp> hops(n_ops);
  for (int q = 0; q < n_ops; ++q) hops[q] = {plan[q].out, plan[q].a, plan[q].b, 0};
  const std::vector<int> fin = final_nodes(plan, n_base);
  const Flow f = plan_flow(plan, n_base);
  std::vector<int> flow_host;
  flow_host.insert(flow_host.end(), f.deps0.begin(), f.deps0.end());
  flow_host.insert(flow_host.end(), f.ready0.begin(), f.ready0.end());
  flow_host.insert(flow_host.end(), f.cons_off.begin(), f.cons_off.end());
  flow_host.insert(flow_host.end(), f.cons.begin(), f.cons.end());
  std::vector<int> zeros(std::max(8, n_levels + 1), 0);
  HIPCHK(hipMemcpyAsync(d_ops, hops.data(), n_ops * sizeof(MockOp), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_fin, fin.data(), n_base * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(flowbuf, flow_host.data(), flow_host.size() * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(err, zeros.data(), 8 * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(tickets, zeros.data(), (n_levels + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctrl, zeros.data(), 8 * sizeof(int), hipMemcpyHostToDevice, s));
  const int* deps0 = flowbuf;
  const int* ready0 = flowbuf + n_ops;
  const int* cons_off = flowbuf + 2 * n_ops;
  const int* cons = flowbuf + 3 * n_ops + 1;

  MockArgs a;
  a.mean_us = p->mean_us;
  a.cap_us = std::max(p->mean_us * 64.0, p->mean_us);
  a.ticks_per_us = khz / 1000.0;
  a.seed = p->seed;
  a.dist = p->dist;
  a.spin_limit = g.spin_limit;
  a.err = err;

  hipEvent_t ev[4];
  for (int i = 0; i < 4; ++i) HIPCHK(hipEventCreate(&ev[i]));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  auto run_plan = [&](int n_workers) -> int {
    if (mode == MOCK_DATAFLOW || segs) {
      HIPCHK(launch_mock_dataflow(a, d_ops, n_ops, nodes, deps, deps0, ready, ready0, f.n_ready0, cons_off, cons,
                                  n_base, ctrl, std::min(n_workers, std::max(n_ops, 1)), s));
    } else {
      for (int lvl = 1, first = 0; lvl <= n_levels; ++lvl) {
        int n = 0;
        while (first + n < n_ops && plan[first + n].level == lvl) ++n;
        HIPCHK(launch_mock_level(a, d_ops, first, n, nodes, n_workers, mode == MOCK_LEVEL_QUEUED, tickets + lvl, s));
        first += n;
      }
    }
    return REG_OK;
  };
  int64_t cnt[5] = {0, 0, 0, 0, 0};
  if (!segs) {
    HIPCHK(launch_mock_elements(nodes, M, 0, s));
    HIPCHK(hipEventRecord(ev[0], s));
    TRY(run_plan(workers));
    HIPCHK(hipEventRecord(ev[1], s));
    HIPCHK(hipEventRecord(ev[2], s));
    HIPCHK(hipEventRecord(ev[3], s));
    HIPCHK(launch_mock_gather(nodes, d_fin, (int2*)prefix, M, s));
    cnt[0] = n_ops;
  } else {
    HIPCHK(hipEventRecord(ev[0], s));
    HIPCHK(launch_mock_phase1(a, M, workers, mode == MOCK_FLEX, gaps, rate, total, seg, (int2*)prefix, s));
    HIPCHK(hipEventRecord(ev[1], s));
    HIPCHK(hipMemcpyAsync(nodes, total, workers * sizeof(int2), hipMemcpyDeviceToDevice, s));
    TRY(run_plan(workers));
    HIPCHK(launch_mock_gather(nodes, d_fin, gpre, workers, s));
    HIPCHK(hipEventRecord(ev[2], s));
    HIPCHK(launch_mock_phase3(a, workers, seg, gpre, (int2*)prefix, s));
    HIPCHK(hipEventRecord(ev[3], s));
    cnt[0] = M - workers;
    cnt[1] = n_ops;
  }
  HIPCHK(hipStreamSynchronize(s));
  int h_err[8] = {};
  HIPCHK(hipMemcpy(h_err, err, sizeof h_err, hipMemcpyDeviceToHost));
  int h_ctrl[3] = {};
  if (mode == MOCK_DATAFLOW || segs) HIPCHK(hipMemcpy(h_ctrl, ctrl, sizeof h_ctrl, hipMemcpyDeviceToHost));
  if (h_ctrl[2]) return fail(REG_E_HIP, "mock scan abandoned by the forward-progress watchdog");
  if (segs) {
    int2 s0;
    HIPCHK(hipMemcpy(&s0, seg, sizeof s0, hipMemcpyDeviceToHost));
    cnt[2] = M - (s0.y - s0.x + 1);
  }
  cnt[3] = cnt[0] + cnt[1] + cnt[2];
  cnt[4] = h_err[0];
  if (counts)
    for (int i = 0; i < 5; ++i) counts[i] = cnt[i];
  if (ms) {
    float t01 = 0, t12 = 0, t23 = 0;
    HIPCHK(hipEventElapsedTime(&t01, ev[0], ev[1]));
    HIPCHK(hipEventElapsedTime(&t12, ev[1], ev[2]));
    HIPCHK(hipEventElapsedTime(&t23, ev[2], ev[3]));
    ms[0] = t01;
    ms[1] = t12;
    ms[2] = t23;
    ms[3] = (double)t01 + t12 + t23;
  }
  return REG_OK;
}

void reg_release(void) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!g.init) return;
  (void)hipDeviceSynchronize();
  for (DevBuf* b : {&g.pyr, &g.slots, &g.part, &g.ctrl, &g.tasks, &g.nodes, &g.upair, &g.iters, &g.status,
                    &g.misc, &g.lvl, &g.flow, &g.mock, &g.flexw, &g.flexn, &g.flext, &g.flexf, &g.rnodes,
                    &g.rtasks, &g.rpart, &g.rctrl, &g.rflow}) {
    if (b->p) (void)hipFree(b->p);
    b->p = nullptr;
    b->n = 0;
  }
  for (auto& e : g.events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  g.events.clear();
  g.events_used = 0;
  drop_graphs();
  g.generation++;
}

}  // extern "C"
