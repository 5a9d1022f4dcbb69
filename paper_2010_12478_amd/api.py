"""Tensor-level entry points: the C ABI called with torch device memory and the
current HIP stream.  Argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import (MOCK_DISTS, MOCK_MODES, MODES, SCAN_ALGOS, SCAN_F_GRAPH, check, lib, mock_params_t,
                   params_struct)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, name, dtype=torch.float32, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _bhw(img, name):
    if img.dim() == 2:
        return 1, img.shape[0], img.shape[1]
    if img.dim() == 3:
        return img.shape
    raise ValueError(f"{name} must be [H][W] or [B][H][W]")


def warp(T, u, out=None):
    """T(x + u(x)): T [B][H][W] (or [H][W]), u [B][2][H][W] (or [2][H][W])."""
    f64 = T.dtype == torch.float64
    dt = torch.float64 if f64 else torch.float32
    B, H, W = _bhw(T, "T")
    _need(T, "T", dt)
    _need(u, "u", dt)
    if u.numel() != B * 2 * H * W:
        raise ValueError("u must hold [B][2][H][W]")
    if out is None:
        out = torch.empty_like(T)
    _need(out, "out", dt, T.shape)
    fn = lib.reg_warp_f64 if f64 else lib.reg_warp
    check(fn(_ptr(T), _ptr(u), _ptr(out), B, H, W, _stream()))
    return out


def warp_adjoint(gout, u, gT=None):
    """gT += transpose of the warp applied to gout (atomic scatter-add)."""
    f64 = gout.dtype == torch.float64
    dt = torch.float64 if f64 else torch.float32
    B, H, W = _bhw(gout, "gout")
    _need(gout, "gout", dt)
    _need(u, "u", dt)
    if u.numel() != B * 2 * H * W:
        raise ValueError("u must hold [B][2][H][W]")
    if gT is None:
        gT = torch.zeros_like(gout)
    _need(gT, "gT", dt, gout.shape)
    fn = lib.reg_warp_adjoint_f64 if f64 else lib.reg_warp_adjoint
    check(fn(_ptr(gout), _ptr(u), _ptr(gT), B, H, W, _stream()))
    return gT


def energy_grad(R, T, u, lam, want_grad=True, want_gnorm=False):
    """(E [B] double, dE/du [B][2][H][W] or None, |grad|^2 [B] or None)."""
    f64 = R.dtype == torch.float64
    dt = torch.float64 if f64 else torch.float32
    B, H, W = _bhw(R, "R")
    for t, n in ((R, "R"), (T, "T"), (u, "u")):
        _need(t, n, dt)
    if T.numel() != B * H * W or u.numel() != B * 2 * H * W:
        raise ValueError("T must hold [B][H][W] and u [B][2][H][W]")
    dev = R.device
    E = torch.empty(B, dtype=torch.float64, device=dev)
    g = torch.empty((B, 2, H, W), dtype=dt, device=dev) if want_grad else None
    gn = torch.empty(B, dtype=torch.float64, device=dev) if want_gnorm else None
    fn = lib.reg_energy_grad_f64 if f64 else lib.reg_energy_grad
    check(fn(_ptr(R), _ptr(T), _ptr(u), float(lam), _ptr(E), _ptr(g), _ptr(gn), B, H, W, _stream()))
    return E, g, gn


def energy_grad_noalloc(R, T, u, lam, want_grad=True, want_gnorm=False, E=None, grad=None, gnorm=None):
    """energy_grad through the allocation-free entry point (float32 inputs;
    the library allocates nothing; outputs may be passed in)."""
    B, H, W = _bhw(R, "R")
    for t, n in ((R, "R"), (T, "T"), (u, "u")):
        _need(t, n)
    if T.numel() != B * H * W or u.numel() != B * 2 * H * W:
        raise ValueError("T must hold [B][H][W] and u [B][2][H][W]")
    dev = R.device
    if E is None:
        E = torch.empty(B, dtype=torch.float64, device=dev)
    if grad is None and want_grad:
        grad = torch.empty((B, 2, H, W), dtype=torch.float32, device=dev)
    if gnorm is None and want_gnorm:
        gnorm = torch.empty(B, dtype=torch.float64, device=dev)
    check(lib.reg_energy_grad_noalloc(_ptr(R), _ptr(T), _ptr(u), float(lam), _ptr(E), _ptr(grad), _ptr(gnorm),
                                      B, H, W, _stream()))
    return E, grad, gnorm


def pyramid_energy(Ia, u, Ib, lam, levels=1):
    f64 = Ia.dtype == torch.float64
    dt = torch.float64 if f64 else torch.float32
    B, H, W = Ia.shape
    for t, n in ((Ia, "Ia"), (u, "u"), (Ib, "Ib")):
        _need(t, n, dt)
    E = torch.empty(B, dtype=torch.float64, device=Ia.device)
    fn = lib.reg_pyramid_energy_f64 if f64 else lib.reg_pyramid_energy
    check(fn(_ptr(Ia), _ptr(u), _ptr(Ib), float(lam), int(levels), _ptr(E), B, H, W, _stream()))
    return E


def pyramid_energy_backward(Ia, u, Ib, lam, levels, gE, need=(True, True, True)):
    f64 = Ia.dtype == torch.float64
    dt = torch.float64 if f64 else torch.float32
    B, H, W = Ia.shape
    _need(gE, "gE", torch.float64, (B,))
    dIa = torch.empty_like(Ia) if need[0] else None
    du = torch.empty_like(u) if need[1] else None
    dIb = torch.empty_like(Ib) if need[2] else None
    fn = lib.reg_pyramid_energy_backward_f64 if f64 else lib.reg_pyramid_energy_backward
    check(fn(_ptr(Ia), _ptr(u), _ptr(Ib), float(lam), int(levels), _ptr(gE), _ptr(dIa), _ptr(du),
             _ptr(dIb), B, H, W, _stream()))
    return dIa, du, dIb


def compose(u_ij, u_jk, out=None):
    B = u_ij.shape[0] if u_ij.dim() == 4 else 1
    H, W = u_ij.shape[-2:]
    _need(u_ij, "u_ij")
    _need(u_jk, "u_jk", shape=u_ij.shape)
    if out is None:
        out = torch.empty_like(u_ij)
    _need(out, "out", shape=u_ij.shape)
    check(lib.reg_compose(_ptr(u_ij), _ptr(u_jk), _ptr(out), B, H, W, _stream()))
    return out


def restrict(x, scale=1.0):
    """scale * 2x2 block mean of every [H][W] plane of x."""
    _need(x, "x")
    H, W = x.shape[-2:]
    B = x.numel() // (H * W)
    out = torch.empty(x.shape[:-2] + (H // 2, W // 2), dtype=x.dtype, device=x.device)
    check(lib.reg_restrict(_ptr(x), _ptr(out), float(scale), B, H, W, _stream()))
    return out


def prolong(uc):
    """2 * bilinear upsampling of [B][2][h][w] displacements to [B][2][2h][2w]."""
    _need(uc, "uc")
    squeeze = uc.dim() == 3
    if squeeze:
        uc = uc.unsqueeze(0)
    B, _, h, w = uc.shape
    out = torch.empty((B, 2, 2 * h, 2 * w), dtype=uc.dtype, device=uc.device)
    check(lib.reg_prolong(_ptr(uc), _ptr(out), B, 2 * h, 2 * w, _stream()))
    return out[0] if squeeze else out


def pyramid(frames, levels):
    """Levels 1..L-1 of the frame pyramid as a list of tensors."""
    _need(frames, "frames")
    N, H, W = frames.shape
    sizes = [(N, H >> l, W >> l) for l in range(1, levels)]
    total = sum(a * b * c for a, b, c in sizes)
    buf = torch.empty(max(total, 1), dtype=torch.float32, device=frames.device)
    check(lib.reg_pyramid(_ptr(frames), _ptr(buf), N, H, W, levels, _stream()))
    out, off = [], 0
    for s in sizes:
        n = s[0] * s[1] * s[2]
        out.append(buf[off:off + n].view(*s))
        off += n
    return out


def solve_batch(frames, ref_idx, tmpl_idx, params, u0=None, mode="batched"):
    """Batch of multilevel registrations; returns (u, iters [B][L], status [B])."""
    _need(frames, "frames")
    N, H, W = frames.shape
    ref = np.ascontiguousarray(np.asarray(ref_idx, dtype=np.int32))
    tmp = np.ascontiguousarray(np.asarray(tmpl_idx, dtype=np.int32))
    B = len(ref)
    if len(tmp) != B:
        raise ValueError("ref_idx and tmpl_idx differ in length")
    dev = frames.device
    if u0 is not None:
        _need(u0, "u0", shape=(B, 2, H, W))
    u = torch.empty((B, 2, H, W), dtype=torch.float32, device=dev)
    iters = torch.empty((B, params.levels), dtype=torch.int32, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    p = params_struct(params)
    check(lib.reg_solve_batch(_ptr(frames), N, H, W, ref.ctypes.data_as(ctypes.c_void_p),
                              tmp.ctypes.data_as(ctypes.c_void_p), _ptr(u0), _ptr(u), _ptr(iters),
                              _ptr(status), B, ctypes.byref(p), MODES[mode], _stream()))
    return u, iters, status


def scan_run(frames, params, algo="seq", chunk=0, global_algo="lf", mode="batched", graph=False,
             want_pairs=True, out=None):
    """Register every frame to frame 0.  Returns (phi0 [M][2][H][W],
    u_pair [M][2][H][W] or None, op_iters [M + n_ops][L], status [M + n_ops])."""
    _need(frames, "frames")
    N, H, W = frames.shape
    M = N - 1
    from ._lib import plan as _plan
    n_ops = len(_plan(M, algo, chunk, global_algo)[0])
    dev = frames.device
    if out is None:
        out = dict(
            phi0=torch.empty((M, 2, H, W), dtype=torch.float32, device=dev),
            u_pair=torch.empty((M, 2, H, W), dtype=torch.float32, device=dev) if want_pairs else None,
            iters=torch.empty((M + n_ops, params.levels), dtype=torch.int32, device=dev),
            status=torch.empty(M + n_ops, dtype=torch.int32, device=dev))
    p = params_struct(params)
    check(lib.scan_run(_ptr(frames), N, H, W, ctypes.byref(p), SCAN_ALGOS[algo], int(chunk),
                       SCAN_ALGOS[global_algo], MODES[mode], SCAN_F_GRAPH if graph else 0,
                       _ptr(out["phi0"]), _ptr(out["u_pair"]), _ptr(out["iters"]),
                       _ptr(out["status"]), _stream()))
    return out["phi0"], out["u_pair"], out["iters"], out["status"]


def scan_run_flex(frames, params, workers, global_algo="lf", want_pairs=True):
    """Reduce-then-scan with flexible segment boundaries (Algorithm 1).
    Returns (phi0, u_pair or None, seg [workers][4] int32 numpy, step [M]
    int32 numpy, counts [phase 1, global, rescans, all], ms [pairwise, phase 1,
    global + rescans, total])."""
    _need(frames, "frames")
    N, H, W = frames.shape
    M = N - 1
    dev = frames.device
    phi0 = torch.empty((M, 2, H, W), dtype=torch.float32, device=dev)
    u_pair = torch.empty((M, 2, H, W), dtype=torch.float32, device=dev) if want_pairs else None
    seg = np.zeros((workers, 4), dtype=np.int32)
    step = np.zeros(M, dtype=np.int32)
    counts = (ctypes.c_int64 * 4)()
    ms = (ctypes.c_double * 4)()
    p = params_struct(params)
    check(lib.scan_run_flex(_ptr(frames), N, H, W, ctypes.byref(p), int(workers), SCAN_ALGOS[global_algo],
                            _ptr(phi0), _ptr(u_pair), seg.ctypes.data_as(ctypes.c_void_p),
                            step.ctypes.data_as(ctypes.c_void_p), ctypes.cast(counts, ctypes.c_void_p),
                            ctypes.cast(ms, ctypes.c_void_p), _stream()))
    return phi0, u_pair, seg, step, list(counts), list(ms)


def rigid_solve_batch(frames, ref_idx, tmpl_idx, params, theta0=None):
    """Batch of multilevel rigid NCC registrations; returns (theta [B][3]
    float64 (alpha, G_x, G_y), iters [B][L], status [B])."""
    _need(frames, "frames")
    N, H, W = frames.shape
    ref = np.ascontiguousarray(np.asarray(ref_idx, dtype=np.int32))
    tmp = np.ascontiguousarray(np.asarray(tmpl_idx, dtype=np.int32))
    B = len(ref)
    if len(tmp) != B:
        raise ValueError("ref_idx and tmpl_idx differ in length")
    dev = frames.device
    if theta0 is not None:
        _need(theta0, "theta0", torch.float64, (B, 3))
    theta = torch.empty((B, 3), dtype=torch.float64, device=dev)
    iters = torch.empty((B, params.levels), dtype=torch.int32, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    p = params_struct(params)
    check(lib.reg_rigid_solve_batch(_ptr(frames), N, H, W, ref.ctypes.data_as(ctypes.c_void_p),
                                    tmp.ctypes.data_as(ctypes.c_void_p), _ptr(theta0), _ptr(theta), _ptr(iters),
                                    _ptr(status), B, ctypes.byref(p), _stream()))
    return theta, iters, status


def scan_run_rigid(frames, params, algo="seq", chunk=0, global_algo="lf", mode="batched", want_pairs=True):
    """Series registration with the rigid NCC operator.  Returns (phi0 [M][3],
    pairs [M][3] or None, op_iters [M + n_ops][L], status [M + n_ops])."""
    _need(frames, "frames")
    N, H, W = frames.shape
    M = N - 1
    from ._lib import plan as _plan
    n_ops = len(_plan(M, algo, chunk, global_algo)[0])
    dev = frames.device
    phi0 = torch.empty((M, 3), dtype=torch.float64, device=dev)
    pairs = torch.empty((M, 3), dtype=torch.float64, device=dev) if want_pairs else None
    iters = torch.empty((M + n_ops, params.levels), dtype=torch.int32, device=dev)
    status = torch.empty(M + n_ops, dtype=torch.int32, device=dev)
    p = params_struct(params)
    check(lib.scan_run_rigid(_ptr(frames), N, H, W, ctypes.byref(p), SCAN_ALGOS[algo], int(chunk),
                             SCAN_ALGOS[global_algo], MODES[mode], _ptr(phi0), _ptr(pairs), _ptr(iters),
                             _ptr(status), _stream()))
    return phi0, pairs, iters, status


def last_solve_timing():
    """(total ms, launches) of the persistent launches of the last batched call."""
    ms, n = ctypes.c_double(0), ctypes.c_int(0)
    check(lib.reg_last_solve_timing(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def last_solve_launch_ms():
    """Per-launch device durations (ms) of the last solve / scan_run."""
    n = ctypes.c_int(0)
    check(lib.reg_last_solve_launch_ms(None, 0, ctypes.byref(n)))
    buf = (ctypes.c_double * max(n.value, 1))()
    check(lib.reg_last_solve_launch_ms(buf, n.value, ctypes.byref(n)))
    return list(buf)[:n.value]


def set_tuning(tile_rows=0, max_group=0, resident=None):
    """Tile height of the finest level, workgroup cap per registration, and
    whether levels that fit run register-resident (None keeps it)."""
    check(lib.reg_set_tuning(int(tile_rows), int(max_group), -1 if resident is None else int(bool(resident))))


def autotune(H, W, levels, batch):
    tr, mg = ctypes.c_int(0), ctypes.c_int(0)
    check(lib.reg_autotune(H, W, levels, batch, ctypes.byref(tr), ctypes.byref(mg), _stream()))
    return tr.value, mg.value


def scan_mock(M, mode, workers, mean_us, dist="exp", seed=1410, algo="lf", chunk=0, global_algo="lf",
              want_seg=False, device="cuda"):
    """Prefix scan of M elements with the artificial operator (see scan_mock_run).
    Returns (prefix [M][2] int32, seg [workers][2] int32 or None,
    counts [phase 1, global, phase 3, total, violations], ms [phase 1, global,
    phase 3, total])."""
    prefix = torch.empty((M, 2), dtype=torch.int32, device=device)
    seg = torch.empty((workers, 2), dtype=torch.int32, device=device) if want_seg else None
    counts = (ctypes.c_int64 * 5)()
    ms = (ctypes.c_double * 4)()
    p = mock_params_t(float(mean_us), MOCK_DISTS[dist], 0, int(seed))
    check(lib.scan_mock_run(int(M), SCAN_ALGOS[algo], int(chunk), SCAN_ALGOS[global_algo], MOCK_MODES[mode],
                            int(workers), ctypes.byref(p), _ptr(prefix), _ptr(seg),
                            ctypes.cast(counts, ctypes.c_void_p), ctypes.cast(ms, ctypes.c_void_p), _stream()))
    return prefix, seg, list(counts), list(ms)


def release():
    lib.reg_release()
