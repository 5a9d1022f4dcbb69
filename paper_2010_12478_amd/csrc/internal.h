// Internal interfaces between the C-ABI host layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rs {

constexpr int kMaxLevelsHost = 8;
constexpr int kCtrlHead = 64;     // ints before the per-group control words
constexpr int kMaxGroup = 128;    // workgroups per group at most
constexpr int kCtrlGroup = 512;   // ints per group: [0..127] member arrival epochs, [128..129] ticket,
                                  // [256..383] member XCC ids

// One registration of a batch (device array element).
struct TaskDesc {
  int32_t ref, tmpl;     // frame indices
  int32_t kind;          // 0 identity, 1 composition (ua o ub), 2 given guess ua
  int32_t pad;
  const float* ua;       // u_ij or u0: [2][H][W]
  const float* ub;       // u_jk: [2][H][W]
  float* out;            // [2][H][W]
  int32_t* iters;        // [levels] or nullptr
  int32_t* status;       // [1] or nullptr
};

struct SolveArgs {
  // padded pyramid: pixel (0, 0) of level l of frame f at pyr[l] + f * fstride[l],
  // rows pitch[l] apart, a one-pixel replicate border around every frame
  const float* pyr[kMaxLevelsHost];
  size_t fstride[kMaxLevelsHost];
  int pitch[kMaxLevelsHost];
  int H, W, levels;
  int max_iter, fixed_iter;
  double tau, lam;
  double rel_tol;
  const TaskDesc* tasks;
  int n_tasks;
  int g;                 // workgroups per registration (group)
  int thl[kMaxLevelsHost];   // tile rows per pyramid level
  int resident;          // levels that fit the group run register-resident
  int max_tiles;         // energy slots per buffer (>= tiles of every level, >= g)
  int* ctrl;             // [0] work-queue ticket, [1] abort flag, group q at ctrl + kCtrlHead + kCtrlGroup*q
  double* part;          // [groups][3][max_tiles]: tile energies / resident energy slots
  float* ws;             // [groups][slot_floats]
  size_t slot_floats;
  size_t lvl_off[kMaxLevelsHost];     // offsets of the pyramid-shaped buffer A per level
  size_t bufB_off;       // offset of buffer B inside a slot
  size_t colx_off;       // column-halo exchange area inside a slot: 2 parities of colx_stride floats
  size_t colx_stride;    // floats per parity: 16 * kMaxRPT per tile
  unsigned spin_limit;
  // dataflow execution (dataflow != 0): task t enters ready[] (tail ctrl[3],
  // head ctrl[2]) once deps[t] drops to 0; the consumers of task t are
  // cons[cons_off[t] .. cons_off[t + 1])
  int dataflow;
  int* deps;
  int* ready;
  const int* cons_off;
  const int* cons;
  // phase 1 of the reduce-then-scan with flexible segment boundaries
  // (flex != 0, Algorithm 1): group w is worker w of flex_workers
  int flex;
  int flex_workers;
  int flex_M;                 // elements
  unsigned long long* gaps;   // [workers - 1]: unclaimed elements (lo, hi) between w and w + 1
  float* rates;               // [workers]: time per registration so far
  const int* starts;          // [workers]: first element of every worker
  float* flex_buf;            // [workers][2][2][H][W]: a worker's running result, ping-pong
  const float* elem;          // [M][2][H][W]: the elements u_{e,e+1}
  float* phi0;                // [M][2][H][W]: worker 0 writes its partial results (prefixes) here
  int* flex_seg;              // [workers][4] out: pl, pr, applications, -
  int* elem_step;             // [M] out: 1-based step at which the element was absorbed (0: a start)
  int* elem_iters;            // [M][levels] out: iterations of that registration
  int* elem_status;           // [M] out
  unsigned long long* flex_desc;   // [workers][8]: descriptor broadcast from a worker's leader
};

size_t slot_floats_for(int H, int W, int levels, size_t* lvl_off, size_t* bufB_off);

// Rigid registration with normalized cross-correlation (solver.hip).
struct RigidTask {
  int32_t ref, tmpl;     // frame indices
  int32_t kind;          // 0 identity, 1 composition of ta and tb, 2 given ta
  int32_t pad;
  const double* ta;      // theta_ij or theta0: (alpha, G_x, G_y)
  const double* tb;      // theta_jk
  double* out;           // [3]
  int32_t* iters;        // [levels] or nullptr
  int32_t* status;       // [1] or nullptr
};
constexpr int kRigidSums = 14;   // sum a, b, aa, bb, ab; per parameter sum g, a g, b g
constexpr int kRigidMaxGroup = 16;   // workgroups per rigid registration
constexpr int kRigidSlotBuf = kRigidMaxGroup * 16;   // u64 moment slots of one pass buffer: [member][16]
struct RigidArgs {
  const float* pyr[kMaxLevelsHost];   // padded pyramid (see SolveArgs)
  size_t fstride[kMaxLevelsHost];
  int pitch[kMaxLevelsHost];
  int H, W, levels, max_iter, fixed_iter;
  double tau, rel_tol;
  const RigidTask* tasks;
  int n_tasks;
  int g;                 // workgroups per registration
  int* ctrl;             // [0] ticket, [1] abort, per group at kCtrlHead + kCtrlGroup * id
  double* part;          // [groups][3][kRigidSlotBuf]: per-member moment sums (u64 slots), by pass mod 3
  unsigned spin_limit;
  // dataflow mode (ctrl[2] / ctrl[3]: ready-queue head / tail): dependency
  // counts, the ready queue (-1: not yet filled), consumers of every task
  int dataflow;
  int* deps;
  int* ready;
  const int* cons_off;
  const int* cons;
};
const void* rigid_kernel();
hipError_t launch_rigid(const RigidArgs& a, int grid, hipStream_t s);
hipError_t launch_reset_rigid(int* ctrl, int n_ints, const RigidTask* tasks, int n_tasks, unsigned long long* slots,
                              int n_slots, hipStream_t s);

// Mock-operator scan (mock.hip).  A node is the frame range (i, k) as int2.
struct MockOp {
  int out, a, b, pad;   // node ids: out = a (.) b
};
struct MockArgs {
  double mean_us;        // operator time t
  double cap_us;         // longest drawn time
  double ticks_per_us;   // wall-clock rate
  unsigned long long seed;
  int dist;              // 0 static, 1 exponential with rate 1/t
  unsigned spin_limit;   // ready-queue polls before the watchdog abandons a dataflow run
  int* err;              // adjacency violations (device counter)
};
const void* mock_worker_kernel();
hipError_t launch_mock_elements(int2* nodes, int n, int first_frame, hipStream_t s);
hipError_t launch_mock_level(const MockArgs& a, const MockOp* ops, int first, int n, int2* nodes, int workers,
                             bool queued, int* ticket, hipStream_t s);
hipError_t launch_mock_dataflow(const MockArgs& a, const MockOp* ops, int n_ops, int2* nodes, int* deps,
                                const int* deps0, int* ready, const int* ready0, int n_ready0, const int* cons_off,
                                const int* cons, int n_base, int* ctrl, int workers, hipStream_t s);
hipError_t launch_mock_phase1(const MockArgs& a, int M, int workers, bool steal, unsigned long long* gaps,
                              float* rate, int2* total, int2* seg, int2* prefix, hipStream_t s);
hipError_t launch_mock_phase3(const MockArgs& a, int workers, const int2* seg, const int2* gprefix, int2* prefix,
                              hipStream_t s);
hipError_t launch_mock_gather(const int2* nodes, const int* final_node, int2* out, int n, hipStream_t s);

// kernels.hip
// out = scale * 2x2 block mean of in (the restriction of displacements)
hipError_t launch_restrict(const void* in, void* out, double scale, int B, int H, int W, bool f64, hipStream_t s);
// out = order-5 binomial frame restriction of in; its transpose (H x W is the fine size)
hipError_t launch_restrict_frame(const void* in, void* out, int B, int H, int W, bool f64, hipStream_t s);
hipError_t launch_restrict_frame_adjoint(const void* dC, void* dF, int B, int H, int W, bool f64, hipStream_t s);
// Padded pyramid level (see SolveArgs): dst holds N frames of (h + 2) rows of
// `pitch` floats, pixel (0, 0) at dst + pitch + kPadLeft, every frame
// fstride = (h + 2) * pitch floats apart; rows -1 .. h and columns -1 .. w
// hold the nearest pixel's value.  src == level 0: frames [N][h][w]
// (copied); otherwise the padded level below (sp = its pitch, sfs = its
// frame stride, pointer at its pixel (0, 0)) under the frame restriction.
constexpr int kPadLeft = 32;   // columns before pixel 0 (keeps rows 128-byte aligned)
hipError_t launch_pad_level(const float* src, int sp, size_t sfs, bool copy, float* dst, int pitch, int N, int h,
                            int w, hipStream_t s);
hipError_t launch_prolong(const float* uc, float* uf, int B, int Hf, int Wf, hipStream_t s);
hipError_t launch_compose(const float* uij, const float* ujk, float* out, int B, int H, int W, hipStream_t s);
hipError_t launch_warp(const void* T, const void* u, void* out, int B, int H, int W, bool f64, hipStream_t s);
hipError_t launch_warp_adjoint(const void* g, const void* u, void* gT, int B, int H, int W, bool f64, hipStream_t s);
hipError_t launch_energy_grad(const void* R, const void* T, const void* u, double lam, double* E,
                              void* grad, double* gnorm2, int B, int H, int W, int th,
                              double* part, bool f64, hipStream_t s);
hipError_t launch_energy_backward_level(const void* Ia, const void* u, const void* Ib, double lam,
                                        const double* gE, void* dIa, void* du, void* dIb,
                                        const void* du_c, bool carry, int B, int h, int w,
                                        bool f64, hipStream_t s);
hipError_t launch_add_energy(const double* Ein, double* Eacc, int B, int first, hipStream_t s);
hipError_t launch_synth_frames(float* out, int F, int H, int W, hipStream_t s);

// solver.hip
// the persistent solver with (resident) or without the register-resident
// levels; SolveArgs::resident selects the instantiation at launch
const void* persistent_kernel(bool resident);
constexpr int kStreamWaves = 3;   // waves per SIMD of the instantiation without resident levels (no spills in its sweep loop)
hipError_t launch_persistent(const SolveArgs& a, int grid, hipStream_t s);
hipError_t launch_reset_ctrl(int* ctrl, int n_ints, hipStream_t s);
// *sticky |= (ctrl[1] != 0) after a persistent launch; clear: *sticky = 0
hipError_t launch_note_abort(const int* ctrl, int* sticky, bool clear, hipStream_t s);
hipError_t launch_reset_tasks(int* ctrl, int n_ints, const TaskDesc* tasks, int n_tasks, hipStream_t s);
// dataflow state: deps = deps0, ready = ready0, ctrl[3] (tail) = n_ready0
hipError_t launch_reset_dataflow(int* deps, const int* deps0, int* ready, const int* ready0, int n_tasks,
                                 int* ctrl, int n_ready0, hipStream_t s);
hipError_t launch_plain_init(const TaskDesc* d_task, const SolveArgs& a, float* dst, hipStream_t s);
hipError_t launch_plain_prolong(const float* uc, float* uf, int h, int w, hipStream_t s);
hipError_t launch_plain_sweep(const float* R, const float* T, int pitch, const float* u, float* un, int h, int w,
                              double tau, double lam, int th, double* part, hipStream_t s);
hipError_t launch_plain_reduce(const double* part, int n, double* E, hipStream_t s);
hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s);   // src == nullptr: fill NaN

}  // namespace rs
