"""The allocation-free fused pair (fftpim_apply_pair_noalloc) against the
allocating one (fftpim_apply_pair): same kernels, work arrays in the
library's fixed per-device array.  Two calls in a row, the second on a
smaller problem (stale contents of the shared array must not leak in), and a
plan too large for the array, which is refused before anything runs."""
import numpy as np
import pytest

from paper_2312_02376_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TWO_PI = 2 * np.pi


def _fp():
    from paper_2312_02376_amd import fftpim
    return fftpim


def _surface_plan(N, seed, nrhs):
    src = W.smooth_closed_surface(N, seed)
    plan = _fp().Plan(torch.tensor(src, device="cuda"), 2, [1.0, 1.0], k0=TWO_PI, kt=[0.3 * TWO_PI, 0.1 * TWO_PI],
                      near_n=(16, 16, 8), near_order=4, corr_radius=4, far_n=(10, 10, 8), far_order=5,
                      nrhs_max=nrhs)
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N))
    v = rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N))
    return plan, torch.tensor(q, device="cuda"), torch.tensor(v, device="cuda")


def _cube_plan(N, seed, nrhs):
    src = W.uniform_cube(N, seed)
    plan = _fp().Plan(torch.tensor(src, device="cuda"), 3, [1.0, 1.0, 1.0], near_n=(16, 16, 16), near_order=4,
                      corr_radius=4, far_n=(10, 10, 10), far_order=5, value_type="real", nrhs_max=nrhs)
    q = torch.tensor(W.gaussian_neutral(nrhs, N, seed), device="cuda")
    v = torch.tensor(W.gaussian_neutral(nrhs, N, seed + 1), device="cuda")
    return plan, q, v


def _check(plan, q, v):
    bytes_before = plan.info()["device_bytes"]
    u0, w0 = torch.empty_like(q), torch.empty_like(v)
    plan.apply_pair_noalloc(q, v, u0, w0)
    torch.cuda.synchronize()
    assert plan.last_status() == 0
    # nothing was allocated on the plan's behalf
    assert plan.info()["device_bytes"] == bytes_before
    u1, w1 = plan.apply_pair(q, v)
    # the same kernels in the same order: identical results
    assert torch.equal(u0, u1) and torch.equal(w0, w1)
    assert float(u1.abs().max()) > 0 and float(w1.abs().max()) > 0


@pytest.mark.parametrize("make", [_surface_plan, _cube_plan])
def test_noalloc_pair_matches_pair_twice(make):
    print("case", make.__name__, flush=True)
    big = make(3000, 5, 3)
    _check(*big)
    small = make(700, 9, 2)
    _check(*small)
    # and the larger plan again after the smaller one used the array
    _check(*big)
    for plan in (big[0], small[0]):
        plan.close()


def test_noalloc_pair_refuses_oversized_plan():
    fp = _fp()
    src = W.uniform_cube(2000, 3)
    plan = fp.Plan(torch.tensor(src, device="cuda"), 3, [1.0, 1.0, 1.0], near_n=(128, 128, 128), near_order=2,
                   corr_radius=2, far_n=(8, 8, 8), far_order=3, nrhs_max=1)
    q = torch.zeros(2000, dtype=torch.complex128, device="cuda")
    u, w = torch.empty_like(q), torch.empty_like(q)
    with pytest.raises(fp.FFTPIMError) as e:
        plan.apply_pair_noalloc(q, q.clone(), u, w)
    assert e.value.name == "SCRATCH_LIMIT"
    plan.close()
