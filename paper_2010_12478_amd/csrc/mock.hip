// Prefix scan with an artificial operator (the paper's microbenchmarks,
// Section 5): the scan machinery of the registration library - level
// launches with static or queued assignment, the dataflow ready queue, static
// segments and the work-stealing reduction of Algorithm 1 - run on an
// operator whose only work is to wait for a drawn time.
//
// A scan node is the frame range (i, k) it covers; an element is (e, e + 1).
// Applying the operator to (i, j) and (j', k) checks adjacency (j == j',
// otherwise a violation is counted), waits for the operator time of (i, k),
// and yields (i, k).  The time is t for a static operator; for a dynamic one
// it is exponential with rate 1/t, drawn from a counter-based generator keyed
// by (i, k), or the mean of two such per-frame draws (frames i and k): the
// same application always takes the same time, in every execution form.  One wavefront is one worker; lane 0 carries the state,
// the whole wavefront waits.
#include "internal.h"

namespace rs {

namespace {

constexpr int kMockWG = 64;

__device__ __forceinline__ int2 ld_node(const int2* p) {
  const unsigned long long v =
      __hip_atomic_load((const unsigned long long*)p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  return make_int2((int)(v & 0xffffffffu), (int)(v >> 32));
}
__device__ __forceinline__ void st_node(int2* p, int2 v) {
  const unsigned long long w = (unsigned long long)(unsigned)v.x | ((unsigned long long)(unsigned)v.y << 32);
  __hip_atomic_store((unsigned long long*)p, w, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// splitmix64 finaliser (Steele, Lea and Flood 2014) of the counter
// seed + golden * (1 + i + 2^32 k); the top 53 bits give u in [0, 1).
__device__ __forceinline__ double mock_uniform(unsigned long long seed, int i, int k) {
  unsigned long long z =
      seed + 0x9E3779B97F4A7C15ull * (1ull + (unsigned long long)(unsigned)i + ((unsigned long long)(unsigned)k << 32));
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}

// Operator time of the application yielding (i, k), in ticks of the
// constant-rate wall clock.
__device__ __forceinline__ double mock_exp(const MockArgs& a, int i, int k) {
  const double us = -a.mean_us * log1p(-mock_uniform(a.seed, i, k));
  return us < a.cap_us ? us : a.cap_us;
}

// dist 0: t; 1: exponential per application; 2: the mean of the frame
// difficulties d_i and d_k, each the exponential draw keyed (f, f).
__device__ __forceinline__ unsigned long long mock_ticks(const MockArgs& a, int i, int k) {
  double us = a.mean_us;
  if (a.dist == 1) us = mock_exp(a, i, k);
  else if (a.dist == 2) us = 0.5 * (mock_exp(a, i, i) + mock_exp(a, k, k));
  return (unsigned long long)(us * a.ticks_per_us + 0.5);
}

__device__ __forceinline__ void mock_wait(unsigned long long ticks) {
  const unsigned long long t0 = wall_clock64();
  while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(2);
}

// (i, j) (.) (j', k) -> (i, k), with the wait; returns the result.
__device__ int2 mock_apply(const MockArgs& a, int2 l, int2 r) {
  if (l.y != r.x) atomicAdd(a.err, 1);
  mock_wait(mock_ticks(a, l.x, r.y));
  return make_int2(l.x, r.y);
}

__global__ void __launch_bounds__(256) k_mock_elements(int2* nodes, int n, int first_frame) {
  for (int m = blockIdx.x * 256 + threadIdx.x; m < n; m += gridDim.x * 256)
    nodes[m] = make_int2(first_frame + m, first_frame + m + 1);
}

// One plan level: ops [first, first + n) of the plan; static assignment
// (op q to worker q mod workers) or the atomic ticket queue.
__global__ void __launch_bounds__(kMockWG) k_mock_level(MockArgs a, const MockOp* ops, int first, int n,
                                                        int2* nodes, int queued, int* ticket) {
  if (threadIdx.x != 0) return;   // lane 0 works and waits; the other lanes are idle
  for (int q = queued ? atomicAdd(ticket, 1) : (int)blockIdx.x; q < n;
       q = queued ? atomicAdd(ticket, 1) : q + (int)gridDim.x) {
    const MockOp op = ops[first + q];
    st_node(nodes + op.out, mock_apply(a, ld_node(nodes + op.a), ld_node(nodes + op.b)));
  }
}

// The whole plan in one launch: workers draw ready ops from a queue; a
// finished op releases the consumers whose last input it was, the 64 lanes of
// the worker sharing the consumer list (one node of a Ladner-Fischer plan
// feeds half of the plan).  ready[] is pre-filled with the ops whose inputs
// are elements (tail = ctrl[1]).
__global__ void __launch_bounds__(kMockWG) k_mock_dataflow(MockArgs a, const MockOp* ops, int n_ops, int2* nodes,
                                                           int* deps, int* ready, const int* cons_off,
                                                           const int* cons, int n_base, int* ctrl) {
  const int lane = threadIdx.x;
  for (;;) {
    int t = n_ops;   // lane 0: the next ready op, or n_ops to stop
    if (lane == 0) {
      const int pos = atomicAdd(&ctrl[0], 1);
      if (pos < n_ops) {
        unsigned spins = 0;
        for (;;) {
          const int v = __hip_atomic_load(&ready[pos], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          if (v >= 0) {
            t = v;
            break;
          }
          if (__hip_atomic_load(&ctrl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
          if (++spins > a.spin_limit) {   // forward-progress watchdog: abandon the run
            __hip_atomic_store(&ctrl[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
    }
    t = __shfl(t, 0, kMockWG);
    if (t >= n_ops) break;
    const MockOp op = ops[t];
    if (lane == 0) st_node(nodes + op.out, mock_apply(a, ld_node(nodes + op.a), ld_node(nodes + op.b)));
    __threadfence();   // the node is visible before any consumer is released
    const int c0 = cons_off[op.out - n_base], c1 = cons_off[op.out - n_base + 1];
    for (int c = c0 + lane; c < c1; c += kMockWG) {
      const int q = cons[c];
      if (atomicSub(&deps[q], 1) == 1) {
        const int slot = atomicAdd(&ctrl[1], 1);
        __hip_atomic_store(&ready[slot], q, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_mock_reset_dataflow(int* deps, const int* deps0, int* ready,
                                                             const int* ready0, int n, int* ctrl, int n_ready0) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    deps[i] = deps0[i];
    ready[i] = ready0[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl[0] = 0;
    ctrl[1] = n_ready0;
    ctrl[2] = 0;
  }
}

// Gap between workers w and w + 1: unclaimed elements lo .. hi packed in one
// word, lo taken from the left by w, hi from the right by w + 1.
__device__ __forceinline__ unsigned long long gap_word(int lo, int hi) {
  return (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32);
}
__device__ __forceinline__ int gap_left(unsigned long long g) {
  return (int)(g & 0xffffffffu);
}
__device__ __forceinline__ int gap_right(unsigned long long g) {
  return (int)(g >> 32);
}

// Claims the element next to worker w on one side: side 1 = the left end
// of gap w (w moves right), side 0 = the right end of gap w - 1 (w moves
// left).  Returns -1 if that gap is empty.
__device__ int gap_claim(unsigned long long* gaps, int gi, bool from_left) {
  unsigned long long g = __hip_atomic_load(gaps + gi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const int lo = gap_left(g), hi = gap_right(g);
    if (lo > hi) return -1;
    const unsigned long long nw = from_left ? gap_word(lo + 1, hi) : gap_word(lo, hi - 1);
    if (__hip_atomic_compare_exchange_strong(gaps + gi, &g, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return from_left ? lo : hi;
  }
}

__device__ __forceinline__ int gap_size(const unsigned long long* gaps, int gi) {
  const unsigned long long g =
      __hip_atomic_load((unsigned long long*)gaps + gi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return gap_right(g) - gap_left(g) + 1;
}

// Phase 1 of the reduce-then-scan over `workers` segments (static bounds
// s_w = w M / workers).  steal = 0: worker w folds its own segment left to
// right.  steal = 1: Algorithm 1 - worker 0 starts at element 0 and moves
// right, the last worker starts at M - 1 and moves left, every other worker
// starts at the middle of its segment; after a first step to the right each
// worker extends toward the side whose neighbour is slower (its time per
// operator application, published after every application), or toward the
// only side with unclaimed elements left, until both neighbouring gaps are
// empty.  Worker 0's partial results are prefixes and are written out.
__global__ void __launch_bounds__(kMockWG) k_mock_phase1(MockArgs a, int M, int workers, int steal,
                                                         unsigned long long* gaps, float* rate, int2* total,
                                                         int2* seg, int2* prefix) {
  if (threadIdx.x != 0) return;   // lane 0 works and waits; the other lanes are idle
  const int w = blockIdx.x;
  const int s0 = (int)((long long)w * M / workers), s1 = (int)((long long)(w + 1) * M / workers);
  if (!steal) {
    int2 res = make_int2(s0, s0 + 1);
    if (w == 0) prefix[s0] = res;
    for (int e = s0 + 1; e < s1; ++e) {
      res = mock_apply(a, res, make_int2(e, e + 1));
      if (w == 0) prefix[e] = res;
    }
    total[w] = res;
    seg[w] = make_int2(s0, s1 - 1);
    return;
  }
  int start = (s0 + s1 - 1) / 2;
  if (w == 0) start = 0;
  else if (w == workers - 1) start = M - 1;
  int pl = start, pr = start, ops = 0;
  int2 res = make_int2(start, start + 1);
  if (w == 0) prefix[0] = res;
  const unsigned long long t_begin = wall_clock64();
  for (;;) {
    const int sL = w > 0 ? gap_size(gaps, w - 1) : 0;
    const int sR = w < workers - 1 ? gap_size(gaps, w) : 0;
    if (sL <= 0 && sR <= 0) break;
    bool right;
    if (ops == 0 && sR > 0) right = true;
    else if (sL > 0 && sR > 0)
      right = !(__hip_atomic_load(rate + w - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >
                __hip_atomic_load(rate + w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    else right = sL <= 0;
    const int e = right ? gap_claim(gaps, w, true) : gap_claim(gaps, w - 1, false);
    if (e < 0) continue;   // the neighbour took the last element: look again
    if (right) {
      res = mock_apply(a, res, make_int2(e, e + 1));
      pr = e;
      if (w == 0) prefix[e] = res;
    } else {
      res = mock_apply(a, make_int2(e, e + 1), res);
      pl = e;
    }
    ++ops;
    const float r = (float)((double)(wall_clock64() - t_begin) / ops);
    __hip_atomic_store(rate + w, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  total[w] = res;
  seg[w] = make_int2(pl, pr);
}

__global__ void __launch_bounds__(256) k_mock_gaps(unsigned long long* gaps, float* rate, int M, int workers) {
  for (int w = blockIdx.x * 256 + threadIdx.x; w < workers; w += gridDim.x * 256) {
    rate[w] = 0.f;
    if (w + 1 < workers) {
      auto start = [&](int v) {
        const int s0 = (int)((long long)v * M / workers), s1 = (int)((long long)(v + 1) * M / workers);
        return v == 0 ? 0 : v == workers - 1 ? M - 1 : (s0 + s1 - 1) / 2;
      };
      gaps[w] = gap_word(start(w) + 1, start(w + 1) - 1);
    }
  }
}

// Phase 3: worker w >= 1 rescans its final segment from the global prefix of
// the workers before it.
__global__ void __launch_bounds__(kMockWG) k_mock_phase3(MockArgs a, int workers, const int2* seg,
                                                         const int2* gprefix, int2* prefix) {
  if (threadIdx.x != 0) return;
  const int w = blockIdx.x + 1;
  if (w >= workers) return;
  const int2 sg = seg[w];
  int2 cur = gprefix[w - 1];
  for (int e = sg.x; e <= sg.y; ++e) {
    cur = mock_apply(a, cur, make_int2(e, e + 1));
    prefix[e] = cur;
  }
}

__global__ void __launch_bounds__(256) k_mock_gather(const int2* nodes, const int* final_node, int2* out, int n) {
  for (int m = blockIdx.x * 256 + threadIdx.x; m < n; m += gridDim.x * 256) out[m] = nodes[final_node[m]];
}

inline int blocks_for(long long n) {
  const long long b = (n + 255) / 256;
  return (int)(b < 65535 ? (b > 0 ? b : 1) : 65535);
}

}  // namespace

const void* mock_worker_kernel() { return (const void*)k_mock_dataflow; }

hipError_t launch_mock_elements(int2* nodes, int n, int first_frame, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mock_elements, dim3(blocks_for(n)), dim3(256), 0, s, nodes, n, first_frame);
  return hipGetLastError();
}

hipError_t launch_mock_level(const MockArgs& a, const MockOp* ops, int first, int n, int2* nodes, int workers,
                             bool queued, int* ticket, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int grid = queued ? (workers < n ? workers : n) : (workers < n ? workers : n);
  hipLaunchKernelGGL(k_mock_level, dim3(grid), dim3(kMockWG), 0, s, a, ops, first, n, nodes, queued ? 1 : 0,
                     ticket);
  return hipGetLastError();
}

hipError_t launch_mock_dataflow(const MockArgs& a, const MockOp* ops, int n_ops, int2* nodes, int* deps,
                                const int* deps0, int* ready, const int* ready0, int n_ready0, const int* cons_off,
                                const int* cons, int n_base, int* ctrl, int workers, hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mock_reset_dataflow, dim3(blocks_for(n_ops)), dim3(256), 0, s, deps, deps0, ready, ready0,
                     n_ops, ctrl, n_ready0);
  hipLaunchKernelGGL(k_mock_dataflow, dim3(workers), dim3(kMockWG), 0, s, a, ops, n_ops, nodes, deps, ready,
                     cons_off, cons, n_base, ctrl);
  return hipGetLastError();
}

hipError_t launch_mock_phase1(const MockArgs& a, int M, int workers, bool steal, unsigned long long* gaps,
                              float* rate, int2* total, int2* seg, int2* prefix, hipStream_t s) {
  hipLaunchKernelGGL(k_mock_gaps, dim3(blocks_for(workers)), dim3(256), 0, s, gaps, rate, M, workers);
  hipLaunchKernelGGL(k_mock_phase1, dim3(workers), dim3(kMockWG), 0, s, a, M, workers, steal ? 1 : 0, gaps, rate,
                     total, seg, prefix);
  return hipGetLastError();
}

hipError_t launch_mock_phase3(const MockArgs& a, int workers, const int2* seg, const int2* gprefix, int2* prefix,
                              hipStream_t s) {
  if (workers < 2) return hipSuccess;
  hipLaunchKernelGGL(k_mock_phase3, dim3(workers - 1), dim3(kMockWG), 0, s, a, workers, seg, gprefix, prefix);
  return hipGetLastError();
}

hipError_t launch_mock_gather(const int2* nodes, const int* final_node, int2* out, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mock_gather, dim3(blocks_for(n)), dim3(256), 0, s, nodes, final_node, out, n);
  return hipGetLastError();
}

}  // namespace rs
