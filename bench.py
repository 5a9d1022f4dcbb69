"""Benchmark: series registration by prefix scan on one MI355X.

Headline workload: 4096 synthetic 1024x1024 lattice frames (spacing 12 px,
drift <= 16 px, distortion 2 px, noise 0.1), a 4-level pyramid,
relative-decrease stopping (1e-5, at most 200 iterations per level), the
hierarchical reduce-then-scan plan (chunks of 64 elements, Ladner-Fischer
global phase).  Frames are generated on the device.  One step = frame
pyramid + the 4095 pairwise registrations + every scan op through scan_run in
dataflow mode: one persistent launch in which an op starts as soon as its two
inputs are done; inputs resident in HBM.

Prints one JSON line: frames registered per second over the K timed steps
(with the per-step times and their 95% confidence interval); the roofline of
the dominant kernel (the persistent gradient-descent solver, timed with HIP
events the library records around its launch on the launch stream); the
level-synchronous form (one launch per scan level) and the plain
one-registration-per-launch form on the same GPU (the latter timed on a
sample of registrations and extrapolated); the CPU oracle timed on a bounded
sample on the host cores; the deviation of the GPU's float32-stored fields
from a plain float64 oracle.  The 256 x 256x256 series follows as a
secondary section with the flexible-segment scan (Algorithm 1), the rigid
normalized-cross-correlation operator, the deviation from the sequential
recursion, the standalone kernels and the mock-operator scan
microbenchmarks.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames registered/sec over full prefix scan; warp/grad kernel HBM GB/s vs peak"
PEAK_HBM_GBS = 8000.0
SWEEP_BYTES = 24      # per pixel and kept update: R 4 + T 4 + u 8 read, u' 8 written
EVAL_BYTES = 16       # per pixel of the final evaluation sweep (no update kept)
FIELD_BYTES = 8       # one float32 displacement vector
TILE_ROWS, MAX_GROUP = 64, 64   # the library defaults, set explicitly
HEADLINE = 5                    # series4096-1024x1024-hier
SECONDARY = 2                   # series256-256x256-hier
CPU_SAMPLE_MAX_ITER = 60        # iteration cap per level of the oracle's timing sample


def progress(msg):
    """A progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=HEADLINE, choices=(2, 3, 5),
                    help="series of the headline (5: 4096 x 1024x1024; 3: 1024 x 512x512; 2: 256 x 256x256)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the level-synchronous comparison")
    ap.add_argument("--no-fp64-deviation", action="store_true",
                    help="skip the deviation of the GPU's fields from a plain float64 oracle")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 256 x 256x256 section (flex, rigid, kernels, mock scan, ...)")
    ap.add_argument("--no-mock", action="store_true", help="skip the mock-operator scan microbenchmarks")
    ap.add_argument("--no-flex", action="store_true", help="skip the flexible-segment (Algorithm 1) scan")
    ap.add_argument("--no-rigid", action="store_true", help="skip the rigid NCC operator scan")
    ap.add_argument("--no-kernels", action="store_true", help="skip the standalone warp / energy kernel timings")
    ap.add_argument("--no-seq-deviation", action="store_true",
                    help="skip the report of the scan's deviation from the sequential recursion")
    ap.add_argument("--cpu-sample", type=int, default=0, help="registrations in the oracle sample")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (calibrates the HBM byte counters)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only time the C ABI's standalone kernels on 64 x 512x512 float32 (counter runs)")
    ap.add_argument("--level-probe", type=int, default=-1, metavar="L",
                    help="only run one solver launch on pyramid level L of the headline series, shaped like the "
                         "headline launch at that level: 64 pairwise registrations, 20 fixed iterations, that "
                         "level alone (per-level counter runs)")
    return ap.parse_args()


def copy_probe(mib):
    """A plain copy kernel of known size: what FETCH_SIZE / WRITE_SIZE read
    for it scales the counters of the solver to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3}), flush=True)


def level_probe(level, workload):
    """One solver launch on pyramid level `level` of the workload's series,
    shaped like the headline launch at that level: 64 pairwise registrations
    of frames 0..64 with 20 fixed iterations on that level alone (its frames
    restricted by the library's pyramid), the headline's tile height rule for
    the level (the finest level's, divided by 4 per level, at least 4; the
    library streams such a level in tiles of at least 16 rows), every level
    streamed (the headline's dataflow groups hold no level resident on the
    1024x1024 series), and the same group size (64 tasks give the group the
    dataflow rule gives for 64 resident groups).  Prints the launch's
    duration and its pixel-updates (for counter runs split by level)."""
    import torch
    from dataclasses import replace

    from synth import get_config, make_series
    import paper_2010_12478_amd as rs

    B, iters = 64, 20
    cfg = get_config(workload, n_frames=B + 1)
    S = make_series(cfg.series, device="cuda")
    f = S.frames if level == 0 else rs.pyramid(S.frames, level + 1)[level - 1].contiguous()
    _, H, W = f.shape
    p = replace(cfg.solver, levels=1, max_iter=iters, fixed_iter=True)
    tile_rows = max(4, TILE_ROWS >> (2 * level))
    rs.set_tuning(tile_rows, MAX_GROUP, resident=False)
    out = []
    for _ in range(2):
        rs.solve_batch(f, list(range(B)), list(range(1, B + 1)), p)
        torch.cuda.synchronize()
        out.append(sum(rs.last_solve_launch_ms()))
    rs.set_tuning(TILE_ROWS, MAX_GROUP, resident=True)
    px = B * iters * H * W
    print(json.dumps({"level_probe": level, "workload": cfg.name, "height": H, "width": W, "registrations": B,
                      "iterations": iters, "level_tile_rows": tile_rows, "resident": False, "pixel_updates": px,
                      "kernel_ms": [round(x, 4) for x in out],
                      "gpx_per_s": round(px / (out[-1] / 1000) / 1e9, 2),
                      "algorithmic_gbs": round(SWEEP_BYTES * px / (out[-1] / 1000) / 1e9, 1)}), flush=True)


def algorithmic_bytes(iters, n_pair, H, W, levels, max_iter):
    """Bytes the method must move in the solver launches: per level the kept
    gradient-descent updates (24 B/px), the final evaluation sweep of a level
    that stopped early (16 B/px), the prolongation (coarse read + fine write),
    and the initial guess (identity: coarse write; composition: both fields
    read at full resolution + coarse write)."""
    import numpy as np
    it = np.asarray(iters, dtype=np.int64)
    total = 0
    for l in range(levels):
        px = (H >> l) * (W >> l)
        k = it[:, l]
        total += int(px * (SWEEP_BYTES * k + EVAL_BYTES * (k < max_iter)).sum())
        if l < levels - 1:
            total += int(it.shape[0] * FIELD_BYTES * ((H >> l) * (W >> l) + (H >> (l + 1)) * (W >> (l + 1))))
    pxc = (H >> (levels - 1)) * (W >> (levels - 1))
    n_ops = it.shape[0] - n_pair
    total += int(n_pair * FIELD_BYTES * pxc)
    total += int(n_ops * (2 * FIELD_BYTES * H * W + FIELD_BYTES * pxc))
    return total


def traffic_file(workload_name):
    return os.path.join(ROOT, "profiles", f"k_persistent_{workload_name}.traffic.json")


# float64 operations of one rigid-operator pass over one pixel: the sample
# position (12), the bilinear value and its two derivatives (23), the angle
# derivative (9) and the 14 moment sums (5 additions, 9 fused multiply-adds).
RIGID_FLOP_PER_PIXEL_PASS = 67
PEAK_FP64_TFLOPS = 78.6


def pixel_passes(iters, H, W, levels, max_iter):
    """Pixel passes of a solver (one energy-and-gradient evaluation of one
    pixel): a level that stopped at iteration t evaluated t + 1 times, a
    capped level max_iter times."""
    import numpy as np
    px = 0
    for l in range(levels):
        px += int(np.minimum(iters[:, l] + 1, max_iter).sum()) * (H >> l) * (W >> l)
    return px


def kernel_sources_sha256():
    """Hash of the HIP library sources the solver kernel is built from."""
    import hashlib
    d = os.path.join(ROOT, "paper_2010_12478_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_record(workload_name):
    """The committed counter record of the workload's solver launch, or None
    when there is none or the kernel sources have changed since it was
    taken."""
    try:
        with open(traffic_file(workload_name)) as f:
            t = json.load(f)
    except OSError:
        return None
    return t if t.get("sources_sha256") == kernel_sources_sha256() else None


def measured_traffic(workload_name):
    """HBM bytes per solver launch from rocprofv3 counter runs of that launch
    (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a plain
    device copy of known size), or None."""
    t = traffic_record(workload_name)
    return int(t["hbm_bytes_per_dispatch"]) if t and "hbm_bytes_per_dispatch" in t else None


def traffic_estimate(workload_name, iters, H, W, levels, max_iter, alg_bytes):
    """HBM bytes of a launch composed from counter runs of one launch per
    pyramid level (the level probe): the measured bytes per pixel pass of
    each level times the launch's pixel passes on that level.  None without
    such a record."""
    import numpy as np
    t = traffic_record(workload_name)
    if not t or "bytes_per_pixel_pass" not in t:
        return None
    bpp = t["bytes_per_pixel_pass"]
    est = 0.0
    for l in range(levels):
        est += bpp[l] * int(np.minimum(iters[:, l] + 1, max_iter).sum()) * (H >> l) * (W >> l)
    return {"bytes": int(est), "per_algorithmic": round(est / alg_bytes, 4),
            "method": "per-level counter runs of the same instantiation (bytes per pixel pass x pixel passes)"}


def ci95(xs):
    """Half-width of the 95% confidence interval of the mean (Student t)."""
    n = len(xs)
    if n < 2:
        return None
    from scipy.stats import t
    m = sum(xs) / n
    sd = math.sqrt(sum((x - m) ** 2 for x in xs) / (n - 1))
    return float(t.ppf(0.975, n - 1) * sd / math.sqrt(n))


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        return None


def _timed_pool(fn, args, cores):
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(fn, args))
    return res, time.perf_counter() - t0


def cpu_baseline(cfg, sample):
    """Oracle throughput on the host cores: `sample` pairwise registrations
    (frames 0..sample of the workload's series, generated on the host) spread
    over one worker process per core, with the iteration cap lowered to
    CPU_SAMPLE_MAX_ITER per level to bound the run, measured as pixel passes
    per second (a pass: one energy-and-gradient evaluation of one pixel; a
    level stopped at iteration t makes t + 1 passes, a capped level max_iter).
    finish_cpu_baseline turns it into frames/s for the workload's pixel
    passes, taken from the GPU run's iteration counts (the oracle's are the
    same), assuming they pack perfectly onto the same cores (which favours the
    oracle: the scan's dependencies are ignored)."""
    import numpy as np
    from dataclasses import replace

    from synth import make_series

    cores = min(len(os.sched_getaffinity(0)), 16)
    sample = min(sample or cores, cfg.series.n_frames - 1)
    fr = make_series(replace(cfg.series, n_frames=sample + 1)).frames.double().numpy()
    p = replace(cfg.solver, max_iter=min(cfg.solver.max_iter, CPU_SAMPLE_MAX_ITER))
    H, W = fr.shape[1:]
    res, wall = _timed_pool(_oracle_pair, [(fr[k - 1], fr[k], p) for k in range(1, sample + 1)], cores)
    passes = pixel_passes(np.array(res), H, W, p.levels, p.max_iter)
    return {"value": None, "unit": "frames/s", "cores": cores, "kind": "oracle", "cpu_model": host_cpu_model(),
            "sample": (f"{sample} pairwise registrations (frames 0..{sample}) of the workload's series, generated "
                       f"on the host, iteration cap lowered to {p.max_iter} per level, on {cores} worker processes "
                       f"(one per host core), {wall:.1f} s wall, {passes:.3g} pixel passes; scaled to the "
                       f"workload's pixel passes assuming perfect packing"),
            "pixel_passes_per_s": passes / wall}


def finish_cpu_baseline(base, M, workload_passes):
    if base is not None:
        base["value"] = M / (workload_passes / base["pixel_passes_per_s"])
        base["workload_pixel_passes"] = int(workload_passes)
    return base


def rigid_cpu_baseline(cfg):
    """The rigid operator's oracle on the host cores, as cpu_baseline: every
    pairwise registration of the rigid series."""
    import numpy as np
    from dataclasses import replace

    from synth import RIGID_TAU, rigid_series

    cores = min(len(os.sched_getaffinity(0)), 16)
    S = rigid_series(cfg.series)
    fr = S.frames.double().numpy()
    sample = fr.shape[0] - 1   # every pairwise registration: about a second on 16 cores
    p = replace(cfg.solver, tau=RIGID_TAU)
    H, W = fr.shape[1:]
    res, wall = _timed_pool(_oracle_rigid_pair, [(fr[k - 1], fr[k], p) for k in range(1, sample + 1)], cores)
    passes = pixel_passes(np.array(res), H, W, p.levels, p.max_iter)
    return {"value": None, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": (f"{sample} pairwise rigid registrations of the rigid series on {cores} worker processes, "
                       f"{wall:.1f} s wall, {passes:.3g} pixel passes; scaled to the workload's pixel passes "
                       f"assuming perfect packing"),
            "pixel_passes_per_s": passes / wall}


def _oracle_rigid_pair(a):
    from oracle import rigid
    from oracle.registration import pyramid
    R, T, p = a
    return rigid.register(pyramid(R, p.levels), pyramid(T, p.levels), None, p).iters


def _oracle_pair(a):
    from oracle.registration import pyramid, register
    R, T, p = a
    r = register(pyramid(R, p.levels), pyramid(T, p.levels), None, p)
    return r.iters


def mock_scan_report(rs):
    """The paper's microbenchmarks (Section 5) on the GPU: 98,304 elements,
    1024 workers (one wavefront each), operator time 10 us, static or
    exponential (rate 1/t, independent per application, or per-frame
    difficulty); every execution form of the scan machinery, device time from
    HIP events.  Each result is also checked: every prefix (0, e + 1) and no
    adjacency violation."""
    import numpy as np
    M, P, t = 98304, 1024, 10.0
    want = np.stack([np.zeros(M, np.int64), np.arange(1, M + 1)], axis=1)
    runs = [("static", "level_static", "lf"), ("static", "segments", "lf"), ("static", "flex", "lf"),
            ("exp", "level_static", "lf"), ("exp", "level_queued", "lf"), ("exp", "dataflow", "lf"),
            ("exp", "level_static", "dissemination"), ("exp", "dataflow", "dissemination"),
            ("exp", "segments", "lf"), ("exp", "flex", "lf"), ("exp", "segments", "dissemination"),
            ("exp", "flex", "dissemination"),
            ("frame", "dataflow", "lf"), ("frame", "segments", "lf"), ("frame", "flex", "lf"),
            ("frame", "segments", "dissemination"), ("frame", "flex", "dissemination")]
    out = []
    for dist, form, algo in runs:
        seg_form = form in ("segments", "flex")
        prefix, _, counts, ms = rs.scan_mock(M, form, P, t, dist, 1410, "lf" if seg_form else algo, 0, algo)
        ok = bool(np.array_equal(prefix.cpu().numpy().astype(np.int64), want)) and counts[4] == 0
        row = {"time": dist, "form": form, "plan": algo, "ms": round(ms[3], 3), "ops": int(counts[3]), "correct": ok}
        if seg_form:
            row["phases_ms"] = [round(x, 3) for x in ms[:3]]
        out.append(row)
    return {"elements": M, "workers": P, "mean_us": t, "runs": out}


def rigid_report(rs, cfg, steps):
    """The series scan with the rigid NCC operator on the same workload shape
    (a lattice series under rigid motion, the same plan and stopping rule)."""
    import torch
    from dataclasses import replace

    from synth import RIGID_TAU, rigid_series

    import numpy as np
    S = rigid_series(cfg.series)
    p = replace(cfg.solver, tau=RIGID_TAU)
    frames = S.frames.cuda()
    N, H, W = frames.shape
    M = N - 1
    def run(mode):
        rs.scan_run_rigid(frames, p, cfg.algo, cfg.chunk, cfg.global_algo, mode=mode)
        torch.cuda.synchronize()
        ts, kern = [], []
        for _ in range(steps):
            t1 = time.perf_counter()
            out = rs.scan_run_rigid(frames, p, cfg.algo, cfg.chunk, cfg.global_algo, mode=mode)
            launch = rs.last_solve_launch_ms()
            torch.cuda.synchronize()
            ts.append(1000.0 * (time.perf_counter() - t1))
            kern.append(launch)
        return out, ts, kern

    mean = lambda xs: sum(xs) / len(xs)
    _, ts_b, kern_b = run("batched")
    (phi0, _, iters, status), ts, kern = run("dataflow")
    iters = iters.cpu().numpy()
    status = status.cpu().numpy()
    kms = mean([sum(k) for k in kern])
    n_launch = len(kern[0])
    flop = RIGID_FLOP_PER_PIXEL_PASS * pixel_passes(iters, H, W, p.levels, p.max_iter)
    achieved = flop / (kms / 1000.0) / 1e12
    err = np.abs(phi0.cpu().numpy() - S.theta[1:])
    r = math.sqrt(((W * W - 1) + (H * H - 1)) / 12.0)
    return {"value": round(M / (mean(ts) / 1000.0), 3), "unit": "frames/s", "ms_per_step": round(mean(ts), 3),
            "steps": steps, "registrations": int(len(iters)),
            "mean_iterations_per_level": [round(float(x), 2) for x in iters.mean(axis=0)],
            "maxiter_registrations": int((status & 1).sum()), "tau": p.tau,
            "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                         "kernel": "k_rigid (rigid NCC solver, dataflow)", "kernel_ms_per_step": round(kms, 3),
                         "launches_per_step": n_launch, "kernel_ms_per_launch": round(kms / n_launch, 4),
                         "flop_per_pixel_pass": RIGID_FLOP_PER_PIXEL_PASS, "flop_per_step": flop},
            "vs_known_motion": {"max_translation_px": round(float(err[:, 1:].max()), 4),
                                "max_angle_times_radius_px": round(float(err[:, 0].max()) * r, 4)},
            "mode": "dataflow: the whole series in one persistent launch, device ready queue",
            "batched": {"value": round(M / (mean(ts_b) / 1000.0), 3), "ms_per_step": round(mean(ts_b), 3),
                        "kernel_ms_per_step": round(mean([sum(k) for k in kern_b]), 3),
                        "mode": "one persistent launch for the pairwise phase and one per scan level"}}


def standalone_kernels(rs):
    """The C ABI's standalone kernels on the autograd workload's shape (64
    pairs of 512x512 float32, a smooth +-3 px displacement): mean duration over
    10 calls from HIP events on the stream the library launches on, and the
    achieved algorithmic bandwidth (warp 16 B/px: u 8 + T 4 + out 4;
    energy and gradient 24 B/px: R 4 + T 4 + u 8 + gradient 8; energy only
    16 B/px; adjoint 16 B/px: gout 4 + u 8 + the gathered tap values' scatter
    counted as 4; backward of the one-level energy 32 B/px: Ia 4 gathered +
    u 8 + Ib 4 read, du 8 + dIb 4 written, dIa 4 scattered)."""
    import torch
    B, H, W = 64, 512, 512
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    T = torch.rand((B, H, W), device="cuda", generator=g)
    R = torch.rand((B, H, W), device="cuda", generator=g)
    yy = torch.arange(H, device="cuda", dtype=torch.float32).view(1, H, 1)
    xx = torch.arange(W, device="cuda", dtype=torch.float32).view(1, 1, W)
    ph = torch.rand((B, 1, 1), device="cuda", generator=g) * 6.28
    u = torch.stack([3.0 * torch.sin(2 * math.pi * yy / H + ph) + 0 * xx,
                     3.0 * torch.sin(2 * math.pi * xx / W + ph) + 0 * yy], dim=1).contiguous()
    out = torch.empty_like(T)
    gT = torch.zeros_like(T)
    gE = torch.ones(B, dtype=torch.float64, device="cuda")
    px = B * H * W

    def timeit(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    rows = {}
    for name, fn, bpp in (("reg_warp", lambda: rs.warp(T, u, out), 16),
                          ("reg_energy_grad", lambda: rs.energy_grad(R, T, u, 0.1, want_grad=True), 24),
                          ("reg_energy_grad (energy only)", lambda: rs.energy_grad(R, T, u, 0.1, want_grad=False), 16),
                          ("reg_warp_adjoint", lambda: rs.warp_adjoint(out, u, gT), 16),
                          ("reg_pyramid_energy_backward (1 level)",
                           lambda: rs.pyramid_energy_backward(T, u, R, 0.1, 1, gE), 32)):
        ms = timeit(fn)
        gbs = bpp * px / (ms / 1000.0) / 1e9
        rows[name] = {"ms": round(ms, 4), "GB/s": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}
    return {"shape": "64 x 512x512 float32", "kernels": rows}


def _oracle_pair64(a):
    from oracle.registration import pyramid, register
    R, T, p = a
    r = register(pyramid(R, p.levels, "f64"), pyramid(T, p.levels, "f64"), None, p, "f64")
    return r.u.astype("float32"), r.u, r.iters


def fp64_reference():
    """Host side of the float64 deviation report (run before the GPU is
    touched): the oracle in plain float64 on the 16 x 64x64 sequential scan,
    16 pairwise registrations of the 256x256 series and 4 of the 512x512
    series (frames generated on the host, handed to the GPU afterwards)."""
    import numpy as np
    from dataclasses import replace

    from oracle.scan import run_scan
    from synth import get_config, make_series

    cores = min(len(os.sched_getaffinity(0)), 16)
    t0 = time.perf_counter()
    c1 = get_config(1)
    f1 = make_series(c1.series).frames
    scan = run_scan(f1.double().numpy(), c1.solver, "seq", storage="f64")
    legs = {"scan": (c1, f1, scan.phi0, scan.u_pair)}
    jobs, owners = [], []
    for idx, n in ((2, 16), (3, 4)):
        c = get_config(idx, n_frames=n + 1)
        fr = make_series(c.series).frames
        legs[idx] = (c, fr, n)
        f64 = fr.double().numpy()
        jobs += [(f64[k - 1], f64[k], c.solver) for k in range(1, n + 1)]
        owners += [idx] * n
    res, _ = _timed_pool(_oracle_pair64, jobs, cores)
    for idx in (2, 3):
        c, fr, n = legs[idx]
        legs[idx] = (c, fr, np.stack([r[1] for r, o in zip(res, owners) if o == idx]))
    legs["host_s"] = time.perf_counter() - t0
    return legs


def fp64_deviation(rs, legs):
    """GPU side: the same registrations on the GPU (float64 arithmetic,
    float32 storage) against the float64 oracle: per registration max-abs and
    the number of values above 1e-3 px."""
    import numpy as np
    import torch

    def stats(got, want):
        d = np.abs(got.astype(np.float64) - want).reshape(len(got), -1)
        mx = d.max(axis=1)
        return {"registrations": int(len(mx)), "max_abs_px": float(mx.max()),
                "median_max_abs_px": float(np.median(mx)),
                "registrations_within_1e-3_px": int((mx <= 1e-3).sum()),
                "values_above_1e-3_px": int((d > 1e-3).sum()), "values": int(d.size)}

    c1, f1, phi0_ref, pair_ref = legs["scan"]
    phi0, u_pair, _, _ = rs.scan_run(f1.cuda(), c1.solver, "seq", mode="dataflow")
    torch.cuda.synchronize()
    out = {"series16-64x64-seq (prefixes)": stats(phi0.cpu().numpy(), phi0_ref),
           "series16-64x64-seq (pairs)": stats(u_pair.cpu().numpy(), pair_ref)}
    for idx in (2, 3):
        c, fr, ref = legs[idx]
        n = len(ref)
        u, _, _ = rs.solve_batch(fr.cuda(), list(range(n)), list(range(1, n + 1)), c.solver)
        torch.cuda.synchronize()
        out[f"{c.series.height}x{c.series.width} pairwise, first {n}"] = stats(u.cpu().numpy(), ref)
    out["note"] = ("float64 oracle: frames rounded to float32 once, no other rounding; the GPU stores every "
                   "field in float32 and matches the oracle's float32-storage mode bit for bit")
    out["host_s"] = round(legs["host_s"], 1)
    return out


def plain_report(rs, frames, cfg, workload_passes, value, n_pairs=16, n_plain_iter=2):
    """The plain form on the same GPU, timed on a sample and extrapolated:
    one persistent launch per registration (reg_solve_batch with one
    registration; the library's largest group, 128 workgroups, on it), over
    n_pairs pairwise registrations and the n_pairs - 1 prefixes of the first
    chunk, each started from the composition of the previous prefix and the
    next pair (a chain: one registration at a time); and, as an extra field,
    the one-launch-per-iteration path with a host read-back of the energy.
    Rates are pixel passes per second; the workload's frames/s follows from
    its pixel passes (from the headline run's iteration counts)."""
    import torch
    H, W = frames.shape[1:]
    p = cfg.solver
    rs.set_tuning(TILE_ROWS, 128, resident=True)
    pairs = [frames[k - 1:k + 1] for k in range(1, n_pairs + 1)]
    ends = [torch.stack([frames[0], frames[k]]) for k in range(2, n_pairs + 1)]
    torch.cuda.synchronize()
    import numpy as np
    t_reg, passes = [], 0
    u_prev = None
    rs.solve_batch(pairs[0], [0], [1], p)   # warm
    torch.cuda.synchronize()
    us = []
    for k in range(n_pairs):
        t0 = time.perf_counter()
        u, it, _ = rs.solve_batch(pairs[k], [0], [1], p)
        torch.cuda.synchronize()
        t_reg.append(time.perf_counter() - t0)
        passes += pixel_passes(it.cpu().numpy(), H, W, p.levels, p.max_iter)
        us.append(u)
    u_prev = us[0]
    for k in range(2, n_pairs + 1):
        t0 = time.perf_counter()
        u0 = rs.compose(u_prev, us[k - 1])
        u_prev, it, _ = rs.solve_batch(ends[k - 2], [0], [1], p, u0=u0)
        torch.cuda.synchronize()
        t_reg.append(time.perf_counter() - t0)
        passes += pixel_passes(it.cpu().numpy(), H, W, p.levels, p.max_iter)
    rate = passes / sum(t_reg)
    plain_value = (cfg.series.n_frames - 1) / (workload_passes / rate)
    # one launch per iteration, host read-back of the energy
    t_it, passes_it = 0.0, 0
    for k in range(n_plain_iter):
        t0 = time.perf_counter()
        _, it, _ = rs.solve_batch(pairs[k], [0], [1], p, mode="plain")
        torch.cuda.synchronize()
        t_it += time.perf_counter() - t0
        passes_it += pixel_passes(it.cpu().numpy(), H, W, p.levels, p.max_iter)
    rs.set_tuning(TILE_ROWS, MAX_GROUP, resident=True)
    rate_it = passes_it / t_it
    return {"value": round(plain_value, 3), "unit": "frames/s", "extrapolated": True,
            "mode": "one persistent launch per registration (reg_solve_batch with one registration, group of "
                    "up to 128 workgroups), registrations one after another",
            "sample": (f"{n_pairs} pairwise registrations and the {n_pairs - 1} prefixes of the first chunk "
                       f"(a chain, each from the composition of the previous prefix and the next pair), "
                       f"{sum(t_reg):.2f} s wall, {passes:.3g} pixel passes; scaled to the workload's pixel passes"),
            "ms_per_registration": round(1000 * sum(t_reg) / len(t_reg), 3),
            "pixel_passes_per_s": rate,
            "batched_over_plain": round(value / plain_value, 2),
            "per_iteration_launches": {
                "value": round((cfg.series.n_frames - 1) / (workload_passes / rate_it), 3), "unit": "frames/s",
                "extrapolated": True, "pixel_passes_per_s": rate_it,
                "sample": f"{n_plain_iter} pairwise registrations, {t_it:.2f} s wall",
                "mode": "one registration at a time, one launch per iteration, host energy read-back"}}


def _timed_scan(rs, frames, cfg, out, mode, steps, warmup):
    """warmup untimed calls, then `steps` calls each fenced by a device
    synchronisation; per call the wall time and the solver launches'
    durations (HIP events on the launch stream)."""
    import torch
    for k in range(warmup):
        rs.scan_run(frames, cfg.solver, cfg.algo, cfg.chunk, cfg.global_algo, mode=mode, out=out)
        torch.cuda.synchronize()
        progress(f"{cfg.name} {mode} warmup {k + 1}/{warmup}")
    step_ms, launches = [], []
    t0 = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        rs.scan_run(frames, cfg.solver, cfg.algo, cfg.chunk, cfg.global_algo, mode=mode, out=out)
        launch = rs.last_solve_launch_ms()      # waits for this step's solver events
        torch.cuda.synchronize()
        step_ms.append(1000.0 * (time.perf_counter() - ts))
        launches.append(launch)
        progress(f"{cfg.name} {mode} step {k + 1}/{steps}: {step_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    return step_ms, launches, time.perf_counter() - t0


def _scan_out(cfg, n_regs, dev):
    import torch
    s, L = cfg.series, cfg.solver.levels
    M = s.n_frames - 1
    return dict(phi0=torch.empty((M, 2, s.height, s.width), device=dev),
                u_pair=torch.empty((M, 2, s.height, s.width), device=dev),
                iters=torch.empty((n_regs, L), dtype=torch.int32, device=dev),
                status=torch.empty(n_regs, dtype=torch.int32, device=dev))


def scan_roofline(cfg, iters, launches, steps, M):
    """Roofline of k_persistent from the step's iteration counts and the
    launch durations."""
    s, p = cfg.series, cfg.solver
    H, W = s.height, s.width
    kern_ms = sum(sum(l) for l in launches)
    kern_launches = sum(len(l) for l in launches)
    alg_step = algorithmic_bytes(iters, M, H, W, p.levels, p.max_iter)
    achieved = alg_step * steps / (kern_ms / 1000.0) / 1e9
    per_launch = kern_launches // max(1, steps)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(cfg.name),
            "kernel": "k_persistent (gradient-descent solver, dataflow)",
            "kernel_ms_per_step": round(kern_ms / steps, 3),
            "kernel_ms_steps": [round(sum(l), 3) for l in launches],
            "launches_per_step": per_launch,
            "kernel_ms_per_launch": round(kern_ms / max(1, kern_launches), 4),
            "algorithmic_bytes_per_step": alg_step,
            "algorithmic_bytes_per_launch": alg_step // max(1, per_launch),
            "traffic_estimate": traffic_estimate(cfg.name, iters, H, W, p.levels, p.max_iter,
                                                 alg_step) if per_launch == 1 else None}


def stream_reference():
    """Context for the spec peak: what a plain streaming kernel moves on this
    GPU.  torch.add over 1 GiB float32 operands (two reads and one write per
    element, near the solver's mix of about 2.5 read bytes per written
    byte), mean of 10 calls timed with HIP events on the current stream after
    one untimed call."""
    import torch
    n = 256 << 20
    a = torch.rand(n, device="cuda")
    b = torch.rand(n, device="cuda")
    c = torch.empty(n, device="cuda")
    torch.add(a, b, out=c)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.add(a, b, out=c)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b, c
    torch.cuda.empty_cache()
    gbs = 12 * n / (ms / 1000.0) / 1e9
    return {"kernel": "torch.add over 1 GiB float32 operands (read 2 : write 1)", "ms": round(ms, 4),
            "GB/s": round(gbs, 1), "of_peak": round(gbs / PEAK_HBM_GBS, 4)}


def level_report(iters, max_iter):
    import numpy as np
    return {"mean_iterations_per_level": [round(float(x), 2) for x in iters.mean(axis=0)],
            "capped_per_level": [int(x) for x in (iters >= max_iter).sum(axis=0)]}


def secondary_report(rs, cfg, args, rigid_base):
    """The 256 x 256x256 series: dataflow headline form, level-synchronous
    form, Algorithm 1, deviation from the sequential recursion, the rigid
    operator."""
    import torch

    from synth import make_series

    s, p = cfg.series, cfg.solver
    M = s.n_frames - 1
    series = make_series(s)
    frames = series.frames.cuda()
    ops, n_levels = rs.plan(M, cfg.algo, cfg.chunk, cfg.global_algo)
    out = _scan_out(cfg, M + len(ops), frames.device)
    steps = max(args.steps, 5)
    step_ms, launches, wall = _timed_scan(rs, frames, cfg, out, "dataflow", steps, 2)
    iters = out["iters"].cpu().numpy()
    status = out["status"].cpu().numpy()
    value = M / (wall / steps)
    res = {"workload": cfg.name, "value": round(value, 3), "unit": "frames/s", "steps": steps,
           "ms_per_step": round(1000.0 * wall / steps, 3),
           "step_ms_ci95": None if ci95(step_ms) is None else round(ci95(step_ms), 3),
           "registrations": int(M + len(ops)), "plan_levels": int(n_levels),
           "maxiter_registrations": int((status & 1).sum()), **level_report(iters, p.max_iter),
           "roofline": scan_roofline(cfg, iters, launches, steps, M)}
    mean = lambda xs: sum(xs) / len(xs)
    if not args.no_batched:
        ts_b, launch_b, wall_b = _timed_scan(rs, frames, cfg, out, "batched", steps, 1)
        kb = sum(sum(l) for l in launch_b)
        res["batched"] = {"value": round(M / (wall_b / steps), 3), "unit": "frames/s",
                          "ms_per_step": round(1000.0 * wall_b / steps, 3),
                          "kernel_ms_per_step": round(kb / steps, 3), "launches_per_step": len(launch_b[0]),
                          "phases_ms": {"pairwise": round(mean([l[0] for l in launch_b]), 3),
                                        "scan_levels": round(mean([sum(l[1:]) for l in launch_b]), 3)}}
    if not args.no_seq_deviation:
        rs.scan_run(frames, p, cfg.algo, cfg.chunk, cfg.global_algo, mode="dataflow", out=out)
        seq = rs.scan_run(frames, p, "seq", 0, cfg.global_algo, mode="dataflow", want_pairs=False)
        d = (out["phi0"] - seq[0]).abs()
        per_frame = d.flatten(1).amax(dim=1)
        res["deviation_from_sequential"] = {
            "max_abs_px": round(float(d.max()), 4), "rms_px": round(float(d.pow(2).mean().sqrt()), 5),
            "median_frame_max_abs_px": round(float(per_frame.median()), 4),
            "frames_within_1e-3_px": int((per_frame <= 1e-3).sum()), "frames": M}
    if not args.no_flex:
        progress(f"{cfg.name} Algorithm 1")
        workers = M // cfg.chunk
        rs.scan_run_flex(frames, p, workers, cfg.global_algo, want_pairs=False)
        torch.cuda.synchronize()
        ts, phases = [], []
        for _ in range(steps):
            t1 = time.perf_counter()
            _, _, seg, _, counts, fms = rs.scan_run_flex(frames, p, workers, cfg.global_algo, want_pairs=False)
            torch.cuda.synchronize()
            ts.append(1000.0 * (time.perf_counter() - t1))
            phases.append(fms)
        res["flex"] = {"value": round(M / (mean(ts) / 1000.0), 3), "unit": "frames/s",
                       "ms_per_step": round(mean(ts), 3), "workers": workers, "registrations": int(counts[3]),
                       "phases_ms": {"pairwise": round(mean([x[0] for x in phases]), 3),
                                     "phase1": round(mean([x[1] for x in phases]), 3),
                                     "global_and_rescan": round(mean([x[2] for x in phases]), 3)},
                       "mode": "reduce-then-scan, flexible segment boundaries (Algorithm 1)"}
    if not args.no_rigid:
        progress(f"{cfg.name} rigid operator")
        res["rigid"] = rigid_report(rs, cfg, steps)
        res["rigid"]["cpu_baseline"] = finish_cpu_baseline(
            rigid_base, M, res["rigid"]["roofline"]["flop_per_step"] // RIGID_FLOP_PER_PIXEL_PASS)
    return res


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.level_probe >= 0:
        level_probe(args.level_probe, args.workload)
        return
    if args.kernels_only:
        import paper_2010_12478_amd as rs
        print(json.dumps(standalone_kernels(rs)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the scan shards across GPUs "
              "by its reduce-then-scan hierarchy, which is not built here.", file=sys.stderr)
        sys.exit(2)

    import torch

    from synth import get_config, make_series

    cfg = get_config(args.workload)
    spec, p = cfg.series, cfg.solver
    N, H, W = spec.n_frames, spec.height, spec.width
    M = N - 1
    sec_cfg = get_config(SECONDARY)

    # host-side legs first: their worker pools fork before the GPU is touched
    progress("host legs: oracle sample, float64 references")
    base = None if args.no_cpu_baseline else cpu_baseline(cfg, args.cpu_sample)
    f64_legs = None if args.no_fp64_deviation else fp64_reference()
    rigid_base = None
    if not (args.no_cpu_baseline or args.no_rigid or args.no_secondary):
        rigid_base = rigid_cpu_baseline(sec_cfg)

    lib_path = os.path.join(ROOT, "paper_2010_12478_amd", "libregscan.so")
    if not os.path.exists(lib_path):
        import importlib.util   # build.py by path: the package needs the library to import
        bspec = importlib.util.spec_from_file_location(
            "_regscan_build", os.path.join(ROOT, "paper_2010_12478_amd", "build.py"))
        mod = importlib.util.module_from_spec(bspec)
        bspec.loader.exec_module(mod)
        mod.build()
    import paper_2010_12478_amd as rs

    dev = torch.device("cuda:0")
    progress(f"generating {cfg.name} on the device")
    t0 = time.perf_counter()
    series = make_series(spec, device=dev)          # seeded, generated on the device
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    frames = series.frames
    ops, n_levels = rs.plan(M, cfg.algo, cfg.chunk, cfg.global_algo)
    n_regs = M + len(ops)
    out = _scan_out(cfg, n_regs, dev)
    rs.set_tuning(TILE_ROWS, MAX_GROUP, resident=True)

    step_ms, launches, wall = _timed_scan(rs, frames, cfg, out, "dataflow", args.steps, args.warmup)
    ms_per_step = 1000.0 * wall / args.steps
    iters = out["iters"].cpu().numpy()
    status = out["status"].cpu().numpy()
    value = M / (ms_per_step / 1000.0)
    workload_passes = pixel_passes(iters, H, W, p.levels, p.max_iter)

    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "frames": N, "height": H, "width": W, "levels": p.levels,
                   "spacing_px": spec.spacing, "drift_px": spec.drift, "distortion_px": spec.distort,
                   "noise": spec.noise,
                   "plan": f"{cfg.algo}(chunk={cfg.chunk}, global={cfg.global_algo})",
                   "plan_ops": int(len(ops)), "plan_levels": int(n_levels),
                   "registrations": int(n_regs), "max_iter": p.max_iter, "rel_tol": p.rel_tol,
                   "tau": p.tau, "lambda": p.lam, "storage": "f32", "parallelism": "single-gpu",
                   "frames_generated_on": "device", "pyramid": "binomial [1 5 10 10 5 1]/32 restriction",
                   "execution": "dataflow: pairwise registrations and every scan op in one persistent launch, "
                                "an op started as soon as its inputs are done (device ready queue)",
                   "tile_rows": TILE_ROWS, "max_group": MAX_GROUP,
                   **level_report(iters, p.max_iter),
                   "maxiter_registrations": int((status & 1).sum()),
                   "aborted_registrations": int((status & 4).sum())},
        "step_ms": [round(x, 3) for x in step_ms],
        "step_ms_ci95": None if ci95(step_ms) is None else round(ci95(step_ms), 3),
        "roofline": scan_roofline(cfg, iters, launches, args.steps, M),
        "cpu_baseline": finish_cpu_baseline(base, M, workload_passes),
        "workload_pixel_passes": int(workload_passes),
    }

    mean = lambda xs: sum(xs) / len(xs)
    if not args.no_batched:
        # the level-synchronous form: one persistent launch for the pairwise
        # phase and one per scan level
        nb = min(args.steps, 2)
        _, launch_b, wall_b = _timed_scan(rs, frames, cfg, out, "batched", nb, 1)
        kb = sum(sum(l) for l in launch_b)
        result["batched"] = {"value": round(M / (wall_b / nb), 3), "unit": "frames/s",
                             "ms_per_step": round(1000.0 * wall_b / nb, 3), "steps": nb,
                             "kernel_ms_per_step": round(kb / nb, 3), "launches_per_step": len(launch_b[0]),
                             "phases_ms": {"pairwise": round(mean([l[0] for l in launch_b]), 3),
                                           "scan_levels": round(mean([sum(l[1:]) for l in launch_b]), 3)},
                             "mode": "one persistent launch for the pairwise phase and one per scan level"}
    if not args.no_plain:
        progress("plain one-registration-per-launch sample")
        result["plain"] = plain_report(rs, frames, cfg, workload_passes, value)
        result["batched_over_plain"] = result["plain"]["batched_over_plain"]
    if f64_legs is not None:
        progress("float64 deviation (GPU side)")
        result["deviation_from_fp64_oracle"] = fp64_deviation(rs, f64_legs)
    if not args.no_secondary:
        del out, series, frames
        torch.cuda.empty_cache()
        rs.release()
        result["secondary"] = secondary_report(rs, sec_cfg, args, rigid_base)
        if not args.no_kernels:
            progress("standalone kernels")
            result["secondary"]["standalone_kernels"] = standalone_kernels(rs)
        if not args.no_mock:
            progress("mock-operator scans")
            result["secondary"]["mock_scan"] = mock_scan_report(rs)
    # the launch's real traffic rate against a plain streaming kernel's
    progress("streaming reference")
    roof = result["roofline"]
    ref = stream_reference()
    est = roof.get("traffic_estimate")
    real_bytes = est["bytes"] if est else roof.get("traffic")
    if real_bytes and roof["launches_per_step"] == 1:
        real = real_bytes / (roof["kernel_ms_per_step"] / 1000.0) / 1e9
        ref["solver_real_GB/s"] = round(real, 1)
        ref["solver_real_over_stream"] = round(real / ref["GB/s"], 4)
    roof["stream_reference"] = ref
    result["input_generation_s"] = round(gen_s, 2)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
