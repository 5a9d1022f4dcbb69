"""The allocation-free energy entry point (reg_energy_grad_noalloc) against
reg_energy_grad, through the C ABI: two calls in a row, the second with a
smaller input, each bitwise equal to the allocating entry point (same kernels,
same tile height); a call beyond the scratch limit is rejected."""
import numpy as np
import pytest
import torch

from _helpers import announce, gpu, host, smooth_field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import paper_2010_12478_amd as rs
    rs.set_tuning(64, 64, resident=True)
    return rs


def _inputs(seed, B, H, W):
    rng = np.random.default_rng(seed)
    R = rng.uniform(0, 1, size=(B, H, W)).astype(np.float32)
    T = rng.uniform(0, 1, size=(B, H, W)).astype(np.float32)
    u = smooth_field(rng, B, H, W, 2.5)
    return gpu(R), gpu(T), gpu(u)


def test_noalloc_matches_energy_grad_on_two_calls(rs):
    for seed, (B, H, W) in ((1, (6, 200, 136)), (2, (2, 72, 64))):   # second call smaller
        announce(f"noalloc energy_grad B={B} {H}x{W}")
        R, T, u = _inputs(seed, B, H, W)
        E0, g0, n0 = rs.energy_grad(R, T, u, 0.1, want_grad=True, want_gnorm=True)
        E1, g1, n1 = rs.energy_grad_noalloc(R, T, u, 0.1, want_grad=True, want_gnorm=True)
        E2, _, _ = rs.energy_grad_noalloc(R, T, u, 0.1, want_grad=False, want_gnorm=False)
        torch.cuda.synchronize()
        assert np.array_equal(host(E1), host(E0)) and np.array_equal(host(E2), host(E0))
        assert np.array_equal(host(g1), host(g0))
        assert np.array_equal(host(n1), host(n0))


def test_noalloc_rejects_inputs_beyond_its_scratch(rs):
    from paper_2010_12478_amd import RegError
    R = torch.zeros((1, 8, 8), device="cuda")
    u = torch.zeros((1, 2, 8, 8), device="cuda")
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    # 1024x1024 at the default tile height has 256 tiles: 1025 frames need
    # 262400 energy sums, beyond the 262144 of the scratch
    rc = rs.lib.reg_energy_grad_noalloc(R.data_ptr(), R.data_ptr(), u.data_ptr(), 0.1, E.data_ptr(), None,
                                        None, 1025, 1024, 1024, None)
    assert rc == -1 and "allocation-free" in rs.lib.reg_last_error().decode()
