/*
 * regscan.h - C interface of the MI355X (gfx950) series-registration library.
 *
 * The library computes the paper's series registration (Copik et al.,
 * "Work-stealing prefix scan: addressing load imbalance in large-scale image
 * registration"): every frame f_k of a series is registered to f_0 by the
 * prefix scan phi_{0,k} = phi_{0,1} (.) phi_{1,2} (.) ... (.) phi_{k-1,k}
 * (Section 3), where phi_{i,j} (.) phi_{j,k} = B(phi_ij, phi_jk) registers f_i
 * and f_k starting from the composition of the two deformations
 * (Section 2.3.2), and the elements phi_{k-1,k} = A(f_{k-1}, f_k) come from
 * registrations of consecutive frames started at the identity.
 *
 * Registration operator (Section 2.3.1, multilevel gradient flow), in the
 * dense-displacement form implemented here: phi(x) = x + u(x),
 *   E(u) = sum_x (T(x + u(x)) - R(x))^2
 *        + lambda * sum_{c in x,y} sum_x [ (u_c(x+e1) - u_c(x))^2 + (u_c(x+e2) - u_c(x))^2 ]
 * with forward differences taken only between pixels of the grid, T sampled
 * bilinearly with edge-clamped taps, minimised by u <- u - tau * dE/du on a
 * frame pyramid (coarse to fine) whose levels are binomial low-passes of the
 * level below (see reg_pyramid); displacements pass between levels by half
 * the 2x2 block mean (down) and bilinear prolongation (up).
 *
 * Arithmetic is double precision throughout; stored data (images,
 * displacements, gradients of the float32 entry points) are float32, each
 * stored value being the double result rounded once.
 *
 * Conventions shared by every entry point
 *   - Images are row-major float [H][W]: x = column, y = row, pixel centres at
 *     integer coordinates.  Displacements are planar [2][H][W]: plane 0 holds
 *     the x component, plane 1 the y component, in pixels of that grid.
 *     Batches stack these along a leading dimension.
 *   - Every array pointer is DEVICE memory owned by the caller, contiguous,
 *     4-byte aligned (8-byte for double), unless the description says "host".
 *     The library never frees caller memory.  It owns a lazily grown
 *     workspace (pyramids, ping-pong fields, queue, partial sums) that
 *     reg_release() frees.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All work is enqueued on it asynchronously; outputs are valid once the
 *     stream has synchronised.  Entry points returning counts on the host say so.
 *   - Return value: REG_OK (0) on success; a negative REG_E_* code if the call
 *     was rejected or failed, with a message from reg_last_error().  Argument
 *     errors are detected on the host before anything is enqueued.  No C++
 *     exception crosses this interface.
 *   - Calls from several host threads are serialised inside the library.
 */
#ifndef REGSCAN_H
#define REGSCAN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
enum {
  REG_OK = 0,
  REG_E_INVALID = -1,   /* bad argument: size, pointer, parameter or plan */
  REG_E_NOMEM = -2,     /* workspace allocation failed */
  REG_E_HIP = -3,       /* a HIP runtime call failed */
  REG_E_NODEVICE = -4   /* no usable gfx950 device */
};

/* per-registration status bits (status[] outputs) */
enum {
  REG_S_OK = 0,
  REG_S_MAXITER = 1,    /* some level used its whole iteration budget without
                           meeting the relative-decrease rule (not set when the
                           iteration count is fixed) */
  REG_S_NONFINITE = 2,  /* the energy became NaN or infinite; the solve stopped
                           at that iteration and skipped the finer levels */
  REG_S_ABORTED = 4     /* a batched solve was abandoned by the forward-progress
                           watchdog; the output is not a solution */
};

/* scan algorithms (Section 2.1 Table 1; Section 4.1-4.2) */
enum {
  SCAN_SEQ = 0,            /* left fold, the sequential recursion */
  SCAN_DISSEMINATION = 1,  /* Kogge-Stone / Hillis-Steele rounds */
  SCAN_LADNER_FISCHER = 2, /* P_0 circuit, depth log2 M */
  SCAN_BRENT_KUNG = 3,     /* up-sweep + down-sweep */
  SCAN_HIER = 4            /* reduce-then-scan over chunks, global phase with
                              any of the four algorithms above */
};

/* execution modes */
enum {
  REG_PLAIN = 0,   /* one registration at a time; one kernel launch per
                      gradient-descent iteration and a host read-back of the
                      energy for the stopping rule */
  REG_BATCHED = 1, /* all registrations of a batch (a scan level) in one
                      persistent launch fed by a device atomic work queue */
  REG_DATAFLOW = 2 /* scan_run: the pairwise registrations and every op of
                      the plan in a single persistent launch; an op enters
                      the device ready queue as soon as both of its inputs
                      exist, so no level waits for the slowest registration
                      of the previous one (reg_solve_batch: as REG_BATCHED) */
};

/* scan_run flags */
enum {
  SCAN_F_GRAPH = 1   /* capture the whole run in a HIP graph on first use and
                        replay it on later calls with identical arguments */
};

typedef struct {
  int32_t levels;      /* pyramid levels L >= 1 (level 0 = full resolution) */
  int32_t max_iter;    /* gradient-descent iterations per level, >= 1 */
  int32_t fixed_iter;  /* nonzero: exactly max_iter updates per level */
  double tau;          /* gradient-descent step, > 0 */
  double lambda;       /* smoothness weight, >= 0 */
  double rel_tol;      /* stop a level at iteration t > 0 once
                          E_{t-1} - E_t <= rel_tol * E_{t-1} */
} reg_params_t;

/* One operator application (i, j) (.) (j, k) -> (i, k) of a scan plan.
 * Nodes 0..M-1 are the elements x_1..x_M (x_k = phi_{k-1,k}); node M + n is
 * the output of op n.  a and b are the input nodes (ranges (i,j) and (j,k)).
 * level is as-soon-as-possible: 1 + max(level of a, level of b), elements at
 * level 0.  Ops are sorted by (level, k, i, j). */
typedef struct {
  int32_t level, out, a, b, i, j, k;
} scan_op_t;

/* Text of the last error of this thread (never NULL; "" if none). */
const char* reg_last_error(void);

/* Interface version (major * 100 + minor). */
int reg_version(void);

/* Frame pyramid (multilevel scheme, Section 2.3.1): pixel (Y, X) of level l+1
 * is the separable order-5 binomial low-pass of level l centred on its 2x2
 * block,
 *   sum_{a,b=0..5} w_a w_b F_l[clamp(2Y+a-2)][clamp(2X+b-2)],
 *   w = (1, 5, 10, 10, 5, 1) / 32, taps clamped to the level,
 * each row summed over b first, then the rows over a, in double precision
 * (a reading: the paper does not say how images are coarsened; the 2x2 block
 * mean would pass lattice content that the coarser grid cannot resolve).
 *   frames  [N][H][W]             level 0, read only
 *   pyr     levels 1..L-1 back to back, level l is [N][H>>l][W>>l]
 *           (sum_{l=1}^{L-1} N*(H>>l)*(W>>l) floats); untouched if L == 1
 * H and W must be divisible by 2^(L-1) and H>>(L-1), W>>(L-1) >= 8. */
int reg_pyramid(const float* frames, float* pyr, int N, int H, int W, int levels, void* stream);

/* Deformed template (Definition "Image registration problem", T o phi):
 *   out[b](x) = T[b](x + u[b](x)), bilinear, edge-clamped taps.
 *   T [B][H][W], u [B][2][H][W], out [B][H][W] (out must not alias T or u). */
int reg_warp(const float* T, const float* u, float* out, int B, int H, int W, void* stream);
int reg_warp_f64(const double* T, const double* u, double* out, int B, int H, int W, void* stream);

/* Transpose of the warp with respect to T (scatter-add of the bilinear taps;
 * the derivative of the deformed template T o phi of the Definition "Image
 * registration problem" with respect to T, used by the backward pass):
 *   gT[b][tap(x)] += w_tap(x) * gout[b](x) for the four taps of x + u[b](x).
 *   gout [B][H][W], u [B][2][H][W], gT [B][H][W] accumulated (not cleared).
 * Uses atomic additions: the summation order, and so the last bits of gT,
 * may vary between runs. */
int reg_warp_adjoint(const float* gout, const float* u, float* gT, int B, int H, int W, void* stream);
int reg_warp_adjoint_f64(const double* gout, const double* u, double* gT, int B, int H, int W, void* stream);

/* Energy and gradient of the registration functional (one level; the
 * functional D(R, T o phi) of the Definition "Image registration problem",
 * Section 2.3.1, in the dense form above, and its gradient, the direction of
 * the gradient flow):
 *   E[b]      = E(u[b]) for reference R[b], template T[b]     (double, device)
 *   grad[b]   = dE/du at u[b] (exact away from integer sample positions;
 *               at an integer position the right-sided derivative), or NULL
 *   gnorm2[b] = sum_x |grad[b](x)|^2 (double), or NULL
 *   R, T [B][H][W]; u, grad [B][2][H][W].  Sums are accumulated in double
 *   in a fixed order (bitwise reproducible). */
int reg_energy_grad(const float* R, const float* T, const float* u, double lambda,
                    double* E, float* grad, double* gnorm2, int B, int H, int W, void* stream);
int reg_energy_grad_f64(const double* R, const double* T, const double* u, double lambda,
                        double* E, double* grad, double* gnorm2, int B, int H, int W, void* stream);

/* reg_energy_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results (bitwise, at the same tile height), but the per-tile
 * partial sums live in a fixed 2 MiB device array that every GPU holds for
 * the life of the process, instead of library workspace; no hipMalloc,
 * hipFree or other allocation happens in the call.
 * Limit: (gnorm2 ? 2 : 1) * B * tiles <= 262144, tiles = ceil(W / 64) *
 * ceil(H / tile_rows) (tile_rows: reg_set_tuning, default 64; e.g. B <= 1024
 * at 1024x1024 for the energy alone); larger calls return REG_E_INVALID
 * before anything is enqueued.  Calls that overlap on one GPU (other
 * streams or threads) share the array and race; serialise them. */
int reg_energy_grad_noalloc(const float* R, const float* T, const float* u, double lambda,
                            double* E, float* grad, double* gnorm2, int B, int H, int W, void* stream);

/* Differentiable warp + energy over a pyramid of `levels` levels:
 *   E[b] = sum_l E_l with I_a, I_b restricted as in reg_pyramid and u by half
 *   the 2x2 block mean, E_l the functional above with T = I_a^l, R = I_b^l.
 *   Ia, Ib [B][H][W]; u [B][2][H][W]; E [B] double.  Only the full-resolution
 *   inputs are read; coarser levels live in library workspace. */
int reg_pyramid_energy(const float* Ia, const float* u, const float* Ib, double lambda, int levels,
                       double* E, int B, int H, int W, void* stream);
int reg_pyramid_energy_f64(const double* Ia, const double* u, const double* Ib, double lambda,
                           int levels, double* E, int B, int H, int W, void* stream);

/* Backward of reg_pyramid_energy for upstream gradients gE [B] (double):
 *   dIa = gE * dE/dIa (scatter-add transpose of the gather, restriction
 *   adjoints), du = gE * dE/du, dIb = gE * dE/dIb = -2 r gE (summed over
 *   levels).  The pyramid is recomputed, not stored.  dIa, du, dIb are
 *   overwritten (each may be NULL to skip it); dIa uses atomic additions. */
int reg_pyramid_energy_backward(const float* Ia, const float* u, const float* Ib, double lambda,
                                int levels, const double* gE, float* dIa, float* du, float* dIb,
                                int B, int H, int W, void* stream);
int reg_pyramid_energy_backward_f64(const double* Ia, const double* u, const double* Ib,
                                    double lambda, int levels, const double* gE, double* dIa,
                                    double* du, double* dIb, int B, int H, int W, void* stream);

/* Composition initial guess (Section 2.3.2): displacement of phi_jk o phi_ij,
 *   out[b](x) = u_ij[b](x) + u_jk[b](x + u_ij[b](x)) per component.
 *   u_ij, u_jk, out [B][2][H][W]; out must not alias the inputs. */
int reg_compose(const float* u_ij, const float* u_jk, float* out, int B, int H, int W, void* stream);

/* Restriction to the next coarser grid of the multilevel scheme (Section
 * 2.3.1) as applied to displacements: out[b] = scale * mean of 2x2 blocks.
 *   in [B][H][W], out [B][H/2][W/2]; H, W even.  scale = 0.5 restricts a
 *   displacement plane (pass each plane as its own batch item): how the
 *   initial guess reaches the coarsest level.  Frames are coarsened by
 *   reg_pyramid instead. */
int reg_restrict(const float* in, float* out, double scale, int B, int H, int W, void* stream);

/* Prolongation of a displacement to the finer grid (the coarse-to-fine step
 * of the multilevel scheme, Section 2.3.1):
 *   uf[b](x) = 2 * uc[b]((x - 1/2)/2, (y - 1/2)/2) (bilinear, clamped).
 *   uc [B][2][Hf/2][Wf/2], uf [B][2][Hf][Wf]; Hf, Wf even. */
int reg_prolong(const float* uc, float* uf, int B, int Hf, int Wf, void* stream);

/* Batch of multilevel registrations Reg(R = f_ref[b], T = f_tmpl[b], u0[b]):
 * the initial guess (zero if u0 == NULL) is restricted to the coarsest level,
 * solved there, and every finer level starts from the prolongation of the
 * coarser result (Section 2.3.1).  Per level, iteration t evaluates E_t and
 * the gradient at u_t; unless fixed_iter, the level returns u_t once t > 0 and
 * E_{t-1} - E_t <= rel_tol * E_{t-1}; otherwise u_{t+1} = u_t - tau * grad.
 *   frames    [N][H][W]    the series (level 0); coarser levels are built in
 *                          library workspace on every call
 *   ref_idx, tmpl_idx [B]  HOST int32 frame indices in [0, N)
 *   u0        [B][2][H][W] initial guesses or NULL (identity)
 *   u         [B][2][H][W] results (must not alias u0 or frames)
 *   iters     [B][levels]  iterations per level (level 0 first), or NULL
 *   status    [B]          REG_S_* bits, or NULL
 *   mode      REG_PLAIN, REG_BATCHED or REG_DATAFLOW; all give bitwise
 *             identical results.
 * REG_PLAIN synchronises the stream after every iteration. */
int reg_solve_batch(const float* frames, int N, int H, int W,
                    const int32_t* ref_idx, const int32_t* tmpl_idx,
                    const float* u0, float* u, int32_t* iters, int32_t* status, int B,
                    const reg_params_t* p, int mode, void* stream);

/* Plan of the prefix scan over M elements (host only, no GPU use): the
 * circuits of Section 2.1 (Table 1) and the reduce-then-scan of Section 4.1
 * with the hierarchy of Section 4.2 (SCAN_HIER).
 *   algo        SCAN_*; global_algo is the global phase of SCAN_HIER
 *               (SCAN_SEQ..SCAN_BRENT_KUNG) and is ignored otherwise
 *   chunk       SCAN_HIER chunk length (<= 0 or >= M: a single chunk)
 *   ops         HOST array of `cap` entries, or NULL to query the size
 *   n_ops       HOST out: number of ops;  n_levels: HOST out: plan depth
 * For SCAN_LADNER_FISCHER / SCAN_BRENT_KUNG (and those global phases) with a
 * size that is not a power of two, the circuit is built for the next power of
 * two and ops ending beyond the last element are dropped.
 * Returns REG_E_INVALID if cap is too small (n_ops is still set). */
int scan_plan(int M, int algo, int chunk, int global_algo, scan_op_t* ops, int cap,
              int* n_ops, int* n_levels);

/* Register every frame of a series to frame 0 (Section 3):
 *   phase A   u_pair[k-1] = A(f_{k-1}, f_k), k = 1..M, M = N - 1, one batch;
 *   scan      the plan of (algo, chunk, global_algo) level by level, each level
 *             one batch of B(phi_ij, phi_jk) registrations (REG_BATCHED: one
 *             persistent launch per level; REG_DATAFLOW: one launch for the
 *             whole series, ops started as their inputs complete; REG_PLAIN:
 *             one registration at a time).  Every mode gives bitwise
 *             identical outputs.
 *   frames   [N][H][W], N >= 2
 *   phi0     [M][2][H][W]  out: u_{0,k} for k = 1..M
 *   u_pair   [M][2][H][W]  out: u_{k-1,k}, or NULL (kept in workspace)
 *   op_iters [M + n_ops][levels] out: iterations of the A registrations
 *            (k = 1..M) then of the plan's ops in plan order, or NULL
 *   status   [M + n_ops] out: REG_S_* bits in the same order, or NULL
 *   flags    SCAN_F_* bits
 * Intermediate scan nodes live in library workspace (REG_BATCHED / REG_PLAIN:
 * reused once their last consumer's level has completed). */
int scan_run(const float* frames, int N, int H, int W, const reg_params_t* p,
             int algo, int chunk, int global_algo, int mode, int flags,
             float* phi0, float* u_pair, int32_t* op_iters, int32_t* status, void* stream);

/* Register every frame to frame 0 by the reduce-then-scan with flexible
 * segment boundaries (Section 4.3, Algorithm 1) on `workers` workers, each a
 * group of workgroups of one persistent launch:
 *   pairwise  u_pair[k-1] = A(f_{k-1}, f_k), one batch (as scan_run);
 *   phase 1   worker 0 starts at element 0 and moves right (its partial
 *             results are the prefixes phi0[e]), the last worker starts at
 *             element M - 1 and moves left, worker w in between starts at the
 *             middle of its static segment [w M / workers, (w + 1) M / workers);
 *             after one step to the right a worker extends its segment toward
 *             the neighbour with the larger time per registration so far
 *             (ties: right), or toward the only side with unclaimed elements,
 *             until both neighbouring gaps are empty; extending right runs
 *             B(res, x_e), left B(x_e, res);
 *   global    the global_algo plan (SCAN_SEQ .. SCAN_BRENT_KUNG) over the
 *             segment totals and then each worker's rescan of its segment from
 *             the prefix before it, as one dataflow launch planned on the host
 *             from the final segments.
 *   frames   [N][H][W], N >= 3;  workers 2 .. N - 1 (one group each, all
 *            resident)
 *   phi0     [M][2][H][W] out;  u_pair [M][2][H][W] out or NULL
 *   seg      HOST [workers][4] out or NULL: pl, pr (the final segment),
 *            registrations in phase 1, 0
 *   step     HOST [M] out or NULL: the 1-based phase-1 step at which the
 *            owning worker absorbed element e (0: a worker's start) - with the
 *            segments this gives the combination order of every worker
 *   counts   HOST [4] out or NULL: registrations in phase 1 (M - workers), the
 *            global plan, the rescans, and in all (with the M pairwise ones)
 *   ms       HOST [4] out or NULL: pairwise, phase 1, global + rescans (from
 *            the end of phase 1, including the host round trip that plans
 *            them), total
 * Synchronises the stream (phase 1's segments decide the rest). */
int scan_run_flex(const float* frames, int N, int H, int W, const reg_params_t* p, int workers, int global_algo,
                  float* phi0, float* u_pair, int32_t* seg, int32_t* step, int64_t* counts, double* ms,
                  void* stream);

/* Rigid registration with normalized cross-correlation, the paper's own
 * operator (Definition "Image registration problem", Section 2.3.1):
 *   phi(x) = Rot(alpha) (x - c) + c + G,  c = ((W - 1) / 2, (H - 1) / 2),
 *   theta = (alpha [rad], G_x, G_y [px]),
 *   E(theta) = 1 - NCC(R, T o phi), T sampled bilinearly with edge-clamped
 *   taps (E = 1 with zero gradient when either image is constant);
 * gradient flow theta <- theta - tau (dE/dalpha / r^2, dE/dG_x, dE/dG_y) with
 * r^2 = ((W^2 - 1) + (H^2 - 1)) / 12 (the mean squared pixel distance from c),
 * per level the stopping rule of reg_solve_batch, on the pyramid of
 * reg_pyramid: the
 * initial guess enters the coarsest level with G / 2^(levels-1), each finer
 * level starts from the coarser result with G doubled, alpha is unchanged.
 * p->lambda is not used.
 *   frames    [N][H][W]
 *   ref_idx, tmpl_idx [B]  HOST int32 frame indices in [0, N)
 *   theta0    [B][3] float64 initial guesses or NULL (identity)
 *   theta     [B][3] float64 results (must not alias theta0)
 *   iters     [B][levels] or NULL;  status [B] REG_S_* bits or NULL
 * One persistent launch; the per-launch probe below records it. */
int reg_rigid_solve_batch(const float* frames, int N, int H, int W,
                          const int32_t* ref_idx, const int32_t* tmpl_idx,
                          const double* theta0, double* theta, int32_t* iters, int32_t* status, int B,
                          const reg_params_t* p, void* stream);

/* The series registration of scan_run (Section 3) with the rigid operator:
 * the pairwise registrations theta_{k-1,k} from the identity, then the plan's
 * ops B(theta_ij, theta_jk) = reg_rigid(f_i, f_k) started from the
 * composition phi_jk o phi_ij, whose parameters are
 *   alpha = alpha_ij + alpha_jk,  G = Rot(alpha_jk) G_ij + G_jk.
 *   phi0     [M][3] float64 out: theta_{0,k}, k = 1..M, M = N - 1
 *   pairs    [M][3] float64 out: theta_{k-1,k}, or NULL (kept in workspace)
 *   op_iters [M + n_ops][levels], status [M + n_ops]: as scan_run, or NULL
 *   mode     REG_BATCHED: one persistent launch for the pairwise phase and one
 *            per plan level; REG_DATAFLOW: one launch for the whole series, a
 *            registration starting as soon as its two inputs are done (the
 *            results agree to rounding: the group size, and with it the order
 *            of the moment sums, may differ). */
int scan_run_rigid(const float* frames, int N, int H, int W, const reg_params_t* p,
                   int algo, int chunk, int global_algo, int mode,
                   double* phi0, double* pairs, int32_t* op_iters, int32_t* status, void* stream);

/* Kernel-duration probe: total device time in milliseconds of the persistent
 * solve launches of the last scan_run / reg_solve_batch in REG_BATCHED mode,
 * reg_rigid_solve_batch or scan_run_rigid
 * (HIP events recorded around every launch on the launch stream), and the
 * number of launches.  HOST outputs; waits for those events. */
int reg_last_solve_timing(double* total_ms, int* launches);

/* The same probe per launch, in launch order (for scan_run in REG_BATCHED
 * mode: the pairwise phase, then one launch per scan level): up to `cap`
 * durations in milliseconds into ms[] (HOST), the number of launches into
 * *n.  A call that replays a graph (SCAN_F_GRAPH) reports one duration, that
 * of the whole replay (pyramid, resets and every solver launch), from an
 * event pair recorded around it; the call that captures the graph runs the
 * launches directly and reports them one by one. */
int reg_last_solve_launch_ms(double* ms, int cap, int* n);

/* Prefix scan with an artificial operator (Section 5, microbenchmarks): the
 * scan machinery of scan_run applied to an operator whose only work is to wait.
 * A node is the frame range (i, k) it covers, element e = (e, e + 1); the
 * operator maps (i, j), (j', k) to (i, k), counting a violation if j != j',
 * after waiting for the operator time of (i, k): t = mean_us for
 * MOCK_STATIC_TIME, or exponential with rate 1/t for MOCK_EXP_TIME (capped at
 * 64 t), drawn from the splitmix64 finaliser of the counter
 * seed + 0x9E3779B97F4A7C15 * (1 + i + 2^32 k), u = top 53 bits / 2^53,
 * time = -t ln(1 - u); or for MOCK_FRAME_TIME (d_i + d_k) / 2, d_f being that
 * exponential draw for (f, f) (per-frame difficulty: every application
 * touching a slow frame is slow).  The same application takes the same time
 * in every execution form.  One worker is one wavefront.
 * Execution forms (`mode`):
 *   MOCK_LEVEL_STATIC  the plan (algo, chunk, global_algo) level by level, one
 *                      launch per level, op q of a level on worker q mod workers
 *   MOCK_LEVEL_QUEUED  the same, ops drawn from an atomic ticket per level
 *   MOCK_DATAFLOW      the plan in one launch, ops started as their inputs
 *                      complete (device ready queue)
 *   MOCK_SEGMENTS      reduce-then-scan (Section 4.1) over `workers` static
 *                      segments [w M / workers, (w + 1) M / workers): each worker
 *                      folds its segment, the global_algo plan scans the
 *                      segment totals, each worker rescans its segment
 *   MOCK_FLEX          the same with flexible segment boundaries
 *                      (Section 4.3, Algorithm 1): workers start in the middle
 *                      of their segments (worker 0 at the first element, the
 *                      last worker at the last) and extend toward whichever
 *                      neighbour is slower, claiming unprocessed elements
 *                      from the gap between them with atomics
 *   M         elements (>= 1)
 *   workers   1 .. the number of wavefronts that can be resident (>= 2 for
 *             MOCK_FLEX, <= M for the segment forms)
 *   prefix    [M][2] int32 DEVICE out: the range computed for element e,
 *             (0, e + 1) when the scan is correct
 *   seg       [workers][2] int32 DEVICE out or NULL: final segment [pl, pr] of
 *             every worker (segment forms)
 *   counts    HOST [5] out or NULL: operator applications in phase 1, the
 *             global phase, phase 3, in all (level forms: all in [0] and [3]),
 *             and adjacency violations (0 when correct)
 *   ms        HOST [4] out or NULL: durations of phase 1, the global phase,
 *             phase 3 and their sum (HIP events; level forms: [0] and [3])
 * Synchronises the stream before returning. */
enum { MOCK_STATIC_TIME = 0, MOCK_EXP_TIME = 1, MOCK_FRAME_TIME = 2 };
enum { MOCK_LEVEL_STATIC = 0, MOCK_LEVEL_QUEUED = 1, MOCK_DATAFLOW = 2, MOCK_SEGMENTS = 3, MOCK_FLEX = 4 };
typedef struct {
  double mean_us;       /* operator time t in microseconds, 0 .. 1e6 */
  int32_t dist;         /* MOCK_STATIC_TIME, MOCK_EXP_TIME or MOCK_FRAME_TIME */
  int32_t pad;
  uint64_t seed;
} mock_params_t;

int scan_mock_run(int M, int algo, int chunk, int global_algo, int mode, int workers, const mock_params_t* p,
                  int32_t* prefix, int32_t* seg, int64_t* counts, double* ms, void* stream);

/* Library tuning.
 *   tile_rows  tile height of the finest pyramid level (multiple of 4, 4..64;
 *              level l uses max(4, tile_rows / 4^l)); it fixes the order in
 *              which energies are summed, so results depend on it (within
 *              rounding), not on the other two settings.  Default 64.
 *   max_group  cap on workgroups per registration in REG_BATCHED and
 *              REG_DATAFLOW modes (1..128).  Default 64.
 *   resident   1: pyramid levels whose tiles are 64 columns wide, whose tile
 *              height is a power of two <= 64 dividing the level height, and
 *              whose tile count fits the group keep the field in registers
 *              across iterations (one workgroup per tile); 0: every level
 *              streams the field through memory.  Default 1.
 * 0 keeps tile_rows / max_group, -1 keeps resident.  See also reg_autotune. */
int reg_set_tuning(int tile_rows, int max_group, int resident);

/* Autotuner: on synthetic lattice frames of the given shape, time a batch of
 * `batch` pairwise registrations (REG_BATCHED, 20 fixed iterations per
 * level) for every tile height in {16, 32, 64} and workgroup cap in
 * {1, 4, 8, 16, 32, 64, 128}; keep the fastest as the library tuning and
 * return it (HOST outputs, optional).  Results are cached per shape for the
 * process.  The workgroup cap never changes results; the tile height changes
 * them only within rounding (the order of the energy sums). */
int reg_autotune(int H, int W, int levels, int batch, int* tile_rows, int* max_group, void* stream);

/* Free the library workspace and cached graphs. */
void reg_release(void);

#ifdef __cplusplus
}
#endif

#endif /* REGSCAN_H */
