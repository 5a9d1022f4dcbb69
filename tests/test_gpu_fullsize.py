"""GPU parity at the full sizes of the 512x512 and 1024x1024 series and of the
batched differentiation workload, on outputs the oracle can compute one by one.

Each series is generated on the GPU (same seeded recipe as on the host; the
noise comes from the device generator), registered whole by scan_run in
batched mode with the library defaults, and then sampled:

* pairwise registrations A(f_{k-1}, f_k) at the start, middle and end of the
  series (and one involving a frame with extra noise), recomputed by the
  oracle from the same frames;
* the prefixes phi_{0,2} (and phi_{0,3}) of the first chunk (a left fold in
  the hierarchical plan), recomputed by the oracle from its own pairwise
  results;
* iteration counts of those registrations, which must agree exactly.

Properties that hold at any size are checked on every output: all fields are
finite and no registration is flagged non-finite or aborted.  Recovery of the
generator's known deformation (Section 2.3.2: each frame registered to frame 0
through the chain of its neighbours) is bounded on prefixes phi_{0,k} spread
over the whole series, on the interior D + 2 px from the border: rms <= 0.35
px, the bound of the oracle's recovery pins, and max <= 3 px, below half the
8 px lattice period (a prefix that lost the lattice would be a period off).
"""
import multiprocessing as mp
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest
import torch

from oracle import autodiff as oad
from oracle import plans as oplans
from oracle import registration as oreg
from synth import get_config, ground_truth, make_series

from _helpers import announce, host

pytestmark = pytest.mark.gpu

TOL_PX = 1e-3
GT_RMS_PX = 0.35
GT_MAX_PX = 3.0


@pytest.fixture(scope="module")
def rs():
    import paper_2010_12478_amd as rs
    rs.set_tuning(64, 64, resident=True)   # the library defaults
    return rs


def _reg(args):
    R, T, u0, p = args
    r = oreg.register(R, T, u0, p)
    return r.u, r.iters


def _compare(name, got, want, it_got, it_want):
    err = float(np.abs(got - want).max())
    ndiff = int((got != want).sum())
    print(f"{name}: max-abs {err:.2e} px, {ndiff} of {got.size} values differ, "
          f"iterations gpu {list(it_got)} oracle {list(it_want)}")
    assert err <= TOL_PX, name
    assert list(it_got) == list(it_want), name


def _series_case(rs, index, pair_ks, n_prefix, gt_ks):
    cfg = get_config(index)
    spec, p = cfg.series, cfg.solver
    M = spec.n_frames - 1
    announce(f"full size {cfg.name}: generate")
    S = make_series(spec, device="cuda")
    torch.cuda.synchronize()
    announce(f"full size {cfg.name}: scan_run batched")
    phi0_d, u_pair_d, iters_d, status_d = rs.scan_run(S.frames, p, cfg.algo, cfg.chunk,
                                                      cfg.global_algo, mode="batched")
    torch.cuda.synchronize()
    status = host(status_d)
    iters = host(iters_d)
    assert (status & 6 == 0).all(), "non-finite or aborted registrations"
    assert bool(torch.isfinite(phi0_d).all()) and bool(torch.isfinite(u_pair_d).all())
    print(f"{cfg.name}: {int((status & 1).sum())} of {len(status)} registrations stopped at the cap; "
          f"per level (finest first) {list((iters >= p.max_iter).sum(axis=0))} capped, "
          f"mean iterations {[round(float(v), 1) for v in iters.mean(axis=0)]}")
    ops, _ = oplans.make_plan(M, cfg.algo, cfg.chunk, cfg.global_algo)
    prefix_op = {}
    for k in range(2, n_prefix + 1):
        row = [n for n, r in enumerate(ops) if r[4] == 0 and r[5] == k - 1 and r[6] == k]
        assert len(row) == 1, f"phi_0,{k} is not a left-fold op of the first chunk"
        prefix_op[k] = M + row[0]

    extra = [int(k) for k in S.noisy if k >= 1][:1]    # a frame with extra noise, if any
    ks = sorted(set(range(1, n_prefix + 1)) | set(pair_ks) | set(extra))
    need = sorted({f for k in ks for f in (k - 1, k)})
    P = {f: oreg.pyramid(S.frames[f].double().cpu().numpy(), p.levels) for f in need}
    announce(f"full size {cfg.name}: oracle, {len(ks)} pairwise + {n_prefix - 1} composed registrations")
    with ProcessPoolExecutor(max_workers=len(ks), mp_context=mp.get_context("fork")) as ex:
        A = dict(zip(ks, ex.map(_reg, [(P[k - 1], P[k], None, p) for k in ks])))
    for k in ks:
        _compare(f"{cfg.name} u_{k - 1},{k}", host(u_pair_d[k - 1]).astype(np.float64), A[k][0],
                 iters[k - 1], A[k][1])
    _compare(f"{cfg.name} phi_0,1", host(phi0_d[0]).astype(np.float64), A[1][0], iters[0], A[1][1])
    y = A[1][0]
    for k in range(2, n_prefix + 1):
        y, it = _reg((P[0], P[k], oreg.compose(y, A[k][0]), p))
        _compare(f"{cfg.name} phi_0,{k}", host(phi0_d[k - 1]).astype(np.float64), y, iters[prefix_op[k]], it)

    S_host = type(S)(S.spec, None, S.drift, S.theta, S.origin, S.noisy)
    b = int(spec.drift + 2)
    worst = []
    for k in gt_ks:
        e = (host(phi0_d[k - 1]) - ground_truth(S_host, 0, k))[:, b:-b, b:-b]
        rms, mx = float(np.sqrt((e ** 2).mean())), float(np.abs(e).max())
        worst.append((rms, mx, k))
        print(f"{cfg.name} phi_0,{k} vs generator: rms {rms:.3f} px, max {mx:.2f} px, "
              f"drift {np.abs(S.drift[k] - S.drift[0]).max():.1f} px")
    for rms, mx, k in worst:
        assert rms <= GT_RMS_PX and mx <= GT_MAX_PX, f"phi_0,{k} lost the generator's deformation"


def test_full_size_series1024_512x512(rs):
    """1024 frames 512x512, 3 levels, 10% of frames with extra noise,
    hierarchical plan (chunks of 32, Ladner-Fischer global phase)."""
    _series_case(rs, 3, pair_ks=[511, 1023], n_prefix=3, gt_ks=list(range(1, 1024, 64)) + [1023])


@pytest.mark.timeout(900)
def test_full_size_series4096_1024x1024(rs):
    """4096 frames 1024x1024, 4 levels, lattice spacing 12 px, drift up to
    16 px, hierarchical plan (chunks of 64, Ladner-Fischer global phase)."""
    _series_case(rs, 5, pair_ks=[2048, 4095], n_prefix=2, gt_ks=list(range(1, 4096, 256)) + [4095])


def test_full_size_autograd_64_pairs_512x512(rs):
    """Batched warp + energy with its backward over 64 consecutive frame
    pairs at 512x512 (3-level pyramid recomputed in the backward), displacement
    = the generator's known deformation; sampled pairs against the oracle's
    analytic energy and gradients."""
    cfg = get_config(4)
    spec = cfg.series
    announce("full size autograd 64 x 512x512: generate")
    S = make_series(spec, device="cuda")
    B = cfg.pairs
    Ia = S.frames[1:B + 1].clone().requires_grad_()
    Ib = S.frames[:B].clone().requires_grad_()
    S_host = type(S)(S.spec, None, S.drift, S.theta, S.origin, S.noisy)
    sample = [0, 31, 63]
    gt = {b: ground_truth(S_host, b, b + 1) for b in sample}
    u_np = np.zeros((B, 2, spec.height, spec.width), np.float32)
    for b in range(B):
        u_np[b] = gt[b] if b in gt else ground_truth(S_host, b, b + 1)
    u = torch.from_numpy(u_np).cuda().requires_grad_()
    levels = 3
    announce("full size autograd 64 x 512x512: forward + backward")
    import paper_2010_12478_amd as pkg
    E = pkg.warp_energy(Ia, u, Ib, 0.1, levels)
    E.sum().backward()
    torch.cuda.synchronize()
    for b in sample:
        a64 = Ia[b].detach().double().cpu().numpy()
        b64 = Ib[b].detach().double().cpu().numpy()
        Ew, gA, gU, gB = oad.pyramid_energy_grads(a64, u_np[b].astype(np.float64), b64, 0.1, levels)
        print(f"pair {b}: E gpu {host(E)[b]:.6e} oracle {Ew:.6e}")
        assert host(E)[b] == pytest.approx(Ew, rel=2e-6)
        np.testing.assert_allclose(host(Ia.grad)[b], gA, atol=1e-4, rtol=1e-5)
        np.testing.assert_allclose(host(u.grad)[b], gU, atol=1e-4, rtol=1e-5)
        np.testing.assert_allclose(host(Ib.grad)[b], gB, atol=1e-4, rtol=1e-5)
