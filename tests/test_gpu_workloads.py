"""The three workloads at full size, in the launch configuration the
benchmark uses, against stored exact sums (tests/golden, written by
make_golden.py from the direct-sum oracle) at the stated tolerances, and
against the step-by-step oracle on sampled rows."""
import os

import numpy as np
import pytest

from oracle import pgf as P
from oracle import steps as S
from paper_2312_02376_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TWO_PI = 2 * np.pi

# launch configurations (the benchmark's for the Helmholtz workload)
C1 = dict(near_n=(16, 16, 16), near_order=4, corr_radius=14, far_n=(16, 16, 16), far_order=7, n_images=1)
C2 = dict(near_n=(64, 64, 32), near_order=4, corr_radius=10, corr_ball=10.5, far_n=(24, 24, 16), far_order=7,
          n_images=1)
C3 = dict(near_n=(128, 128, 128), near_order=4, corr_radius=5, far_n=(14, 14, 14), far_order=5, n_images=1)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_elem(a, b):
    """Largest element error in units of the reference's RMS value: a single
    wrong row shows up here even when the rel-L2 over all rows stays small."""
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / np.sqrt(np.mean(np.abs(b) ** 2)))


def _fp():
    from paper_2312_02376_amd import fftpim
    return fftpim


def test_coulomb_cube_1k_fp64_within_1e6():
    src, q = W.coulomb_cube_1k()
    gold = np.loadtxt(os.path.join(GOLD, "coulomb_cube_1k_exact.txt"))[:, 1]
    plan = _fp().Plan(torch.tensor(src, device="cuda"), 3, [1, 1, 1], value_type="real", **C1)
    qd = torch.tensor(q, device="cuda")
    u = plan.apply(qd).cpu().numpy()
    assert plan.last_status() == 0
    e = rel(u, gold)
    print("C1 forward rel-L2 %.3e max elem %.3e" % (e, max_elem(u, gold)))
    assert e <= 1e-6 and max_elem(u, gold) <= 3e-6
    # the exact operator is real symmetric: A^H q = A q, defined up to its mean
    w = plan.adjoint(qd).cpu().numpy()
    g = gold - gold.mean()
    e = rel(w, g)
    print("C1 adjoint rel-L2 %.3e" % e)
    assert e <= 1e-6 and max_elem(w, g) <= 3e-6


@pytest.fixture(scope="module")
def helmholtz_plan():
    src, q64 = W.helmholtz_surface_100k()
    k = TWO_PI
    plan = _fp().Plan(torch.tensor(src, device="cuda"), 2, [1, 1], k0=k, kt=[0.3 * k, 0.1 * k], **C2)
    yield src, q64.astype(np.complex128), plan
    plan.close()


def test_helmholtz_surface_100k_fp64_within_1e6(helmholtz_plan):
    src, q, plan = helmholtz_plan
    v = W.gaussian_complex(1, len(src), 102)[0].astype(np.complex128)
    g = np.loadtxt(os.path.join(GOLD, "helmholtz_surface_100k_rows.txt"))
    rows = g[:, 0].astype(np.int64)
    u = plan.apply(torch.tensor(q, device="cuda")).cpu().numpy()[rows]
    w = plan.adjoint(torch.tensor(v, device="cuda")).cpu().numpy()[rows]
    gu, gw = g[:, 1] + 1j * g[:, 2], g[:, 3] + 1j * g[:, 4]
    eu, ew = rel(u, gu), rel(w, gw)
    mu, mw = max_elem(u, gu), max_elem(w, gw)
    print("C2 forward rel-L2 %.3e adjoint %.3e (%d rows); max elem %.3e / %.3e" % (eu, ew, len(rows), mu, mw))
    assert eu <= 1e-6 and ew <= 1e-6
    assert mu <= 3e-6 and mw <= 3e-6


def test_helmholtz_surface_100k_fp32_within_1e4():
    # the FP32 mode of the surface workload at full size (FP64 correction)
    src, q64 = W.helmholtz_surface_100k()
    k = TWO_PI
    plan = _fp().Plan(torch.tensor(src, device="cuda"), 2, [1, 1], k0=k, kt=[0.3 * k, 0.1 * k], precision="f32",
                      **C2)
    v = W.gaussian_complex(1, len(src), 102)[0]
    g = np.loadtxt(os.path.join(GOLD, "helmholtz_surface_100k_rows.txt"))
    rows = g[:, 0].astype(np.int64)
    u = plan.apply(torch.tensor(q64, device="cuda")).cpu().numpy()[rows]
    w = plan.adjoint(torch.tensor(v, device="cuda")).cpu().numpy()[rows]
    gu, gw = g[:, 1] + 1j * g[:, 2], g[:, 3] + 1j * g[:, 4]
    eu, ew = rel(u, gu), rel(w, gw)
    print("C2 FP32 forward rel-L2 %.3e adjoint %.3e; max elem %.3e / %.3e"
          % (eu, ew, max_elem(u, gu), max_elem(w, gw)))
    assert eu <= 1e-4 and ew <= 1e-4
    assert max_elem(u, gu) <= 3e-4 and max_elem(w, gw) <= 3e-4
    plan.close()


def test_helmholtz_surface_100k_matches_step_oracle(helmholtz_plan):
    # same launch configuration, sampled rows, every stage against the
    # step-by-step oracle at rounding level
    src, q, plan = helmholtz_plan
    k = TWO_PI
    lat = P.Lattice(2, [1, 1], k, [0.3 * k, 0.1 * k])
    ref = S.FFTPIM(lat, S.Params(C2["near_n"], 4, C2["corr_radius"], C2["far_n"], 7, 1, corr_ball=C2["corr_ball"]),
                   src)
    rows = np.sort(np.random.default_rng(3).choice(len(src), 6, replace=False))
    qd = torch.tensor(q, device="cuda")
    for part, bit in (("near_grid", 1), ("near_corr", 2), ("far", 4)):
        got = plan.apply_parts(qd, bit).cpu().numpy()[rows]
        want = ref.apply(q, rows=rows, parts=(part,))
        e = rel(got, want)
        print("C2 %s rel %.2e" % (part, e))
        assert e < 1e-10, part


def test_coulomb_cube_1m_batched_fp32_within_1e4():
    path = os.path.join(GOLD, "coulomb_cube_1m_rows.txt")
    if not os.path.exists(path):
        pytest.skip("golden values not generated")
    src, q = W.coulomb_cube_1m_batched()
    g = np.loadtxt(path)
    rows = np.unique(g[:, 0].astype(np.int64))
    nrhs = q.shape[0]
    gold = g[:, 2].reshape(len(rows), nrhs).T
    plan = _fp().Plan(torch.tensor(src, device="cuda"), 3, [1, 1, 1], value_type="real", precision="f32",
                      nrhs_max=nrhs, **C3)
    qd = torch.tensor(q, device="cuda")
    u = plan.apply(qd).cpu().numpy()[:, rows]
    assert plan.last_status() == 0
    e = rel(u, gold)
    print("C3 forward rel-L2 %.3e max elem %.3e (%d rows x %d)" % (e, max_elem(u, gold), len(rows), nrhs))
    assert e <= 1e-4 and max_elem(u, gold) <= 3e-4
    w = plan.adjoint(qd).cpu().numpy()
    # A^H q = A q for the exact real symmetric operator, up to each column's mean;
    # the sampled rows cannot give that mean, so compare row differences
    d_gpu = w[:, rows] - w[:, rows[:1]]
    d_gold = gold - gold[:, :1]
    e = rel(d_gpu[:, 1:], d_gold[:, 1:])
    print("C3 adjoint (row differences) rel-L2 %.3e" % e)
    assert e <= 1e-4 and max_elem(d_gpu[:, 1:], d_gold[:, 1:]) <= 3e-4
    plan.close()


def test_coulomb_cube_1m_batched_bf16_far_modes():
    # the bfloat16 far grid sums at the full batched size, against the stored
    # exact rows: the three-product split stays inside the 1e-4 FP32 gate;
    # plain bfloat16 does not (rounding the amplitudes of a neutral far sum
    # breaks its cancellation) and is recorded here as missing it
    path = os.path.join(GOLD, "coulomb_cube_1m_rows.txt")
    src, q = W.coulomb_cube_1m_batched()
    g = np.loadtxt(path)
    rows = np.unique(g[:, 0].astype(np.int64))
    nrhs = q.shape[0]
    gold = g[:, 2].reshape(len(rows), nrhs).T
    pos = torch.tensor(src, device="cuda")
    qd = torch.tensor(q, device="cuda")
    errs = {}
    for prec in ("f32_farbf16", "f32_farbf16x3"):
        plan = _fp().Plan(pos, 3, [1, 1, 1], value_type="real", precision=prec, nrhs_max=nrhs, **C3)
        u = plan.apply(qd).cpu().numpy()[:, rows]
        assert plan.last_status() == 0
        errs[prec] = rel(u, gold)
        print("C3 %s forward rel-L2 %.3e" % (prec, errs[prec]), flush=True)
        plan.close()
    assert errs["f32_farbf16x3"] <= 1e-4
    assert 1e-3 < errs["f32_farbf16"] < 0.1
