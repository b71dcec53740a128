"""The paper's validation and timing cases through the C ABI, against exact
sums of Eq. (1) from the direct-sum oracle:

  * the 1D-periodic coaxial shells of Sec. 4 (Fig. potential): the static
    (NPSP) case, whose axis potential is the analytic -ln(r2/r1) of two
    neutral line-charge shells, and the dynamic case k0 = 1, k_x0 = 1 - j;
  * the 3D-periodic cube of Sec. 4.2 (Fig. complex_real): period 101, points
    in a centred 100^3 cube, k0 set by a mean spacing of lambda/20 and phase
    wavenumbers 0.01 - 0.01j per axis, at the two accuracy levels 1e-3 and
    1e-5 (the second doubles the near grid and widens the correction from 4
    to 7 boxes), and its static counterpart."""
import math
import os

import numpy as np
import pytest

from oracle import pgf as P
from oracle import steps as S
from oracle.psp import host_workers, psp_forward
from paper_2312_02376_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fp():
    from paper_2312_02376_amd import fftpim
    return fftpim


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


COAX = dict(near_n=(16, 32, 32), near_order=4, corr_radius=4, far_n=(12, 24, 24), far_order=7, n_images=1)


@pytest.fixture(scope="module")
def coax():
    pts, q, ax = W.coax_shells(32, 64, 16)
    rows = np.r_[np.arange(ax.start, ax.stop), np.arange(0, ax.start, 257)]
    return pts, q, ax, rows


@pytest.mark.parametrize("case", ["static", "dynamic"])
def test_coax_shells(coax, case):
    pts, q, ax, rows = coax
    if case == "static":
        lat, kw, qq, vt = P.Lattice(1, [1.0]), {}, q, "real"
    else:
        lat, kw, qq, vt = P.Lattice(1, [1.0], 1.0, [1 - 1j]), dict(k0=1.0, kt=[1 - 1j]), q.astype(complex), "complex"
    print("coax", case, "N", len(pts), flush=True)
    plan = _fp().Plan(torch.tensor(pts, device="cuda"), 1, [1.0], value_type=vt, **kw, **COAX)
    u = plan.apply(torch.tensor(qq, device="cuda")).cpu().numpy()
    assert plan.last_status() == 0
    plan.close()
    # parity with the step-by-step oracle of the same discrete operator
    ref = S.FFTPIM(lat, S.Params(COAX["near_n"], 4, 4, COAX["far_n"], 7, 1), pts).apply(qq, rows=rows)
    e = rel(u[rows], ref)
    print("  vs oracle steps %.2e" % e)
    assert e < 1e-10
    # accuracy against the exact sum of Eq. (1)
    exact = psp_forward(lat, pts, qq, obs_index=rows, workers=host_workers())
    e = rel(u[rows], exact)
    print("  vs exact %.2e" % e)
    assert e < (1e-4 if case == "static" else 5e-4)
    axis = u[ax]
    if case == "static":
        # inside both shells the potential of the two neutral shells is
        # -(lambda2 / 2 pi) ln r2 = -ln 2; the 32 x 64 sampling of the
        # surfaces costs about 1e-3
        assert np.abs(axis - (-math.log(2.0))).max() < 2e-3
    else:
        assert np.abs(axis).min() > 1e-3


# the dynamic 3D cube: near grid, order, correction radius, far grid, far order
DYN = {"1e-3": ((32, 32, 32), 4, 4, (20, 20, 20), 7), "1e-5": ((64, 64, 64), 4, 7, (28, 28, 28), 7)}


@pytest.fixture(scope="module")
def cube():
    src, q = W.dynamic_cube(20000, 8)
    g = np.loadtxt(os.path.join(GOLD, "dynamic_cube_20k_rows.txt"))
    return src, q, g


@pytest.mark.parametrize("level", list(DYN))
@pytest.mark.parametrize("case", ["dynamic", "static"])
def test_dynamic_cube(cube, level, case):
    src, q, g = cube
    rows = g[:, 0].astype(np.int64)
    nn, qn, rc, nf, qf = DYN[level]
    N = len(src)
    if case == "dynamic":
        k0 = W.dynamic_cube_k0(N)
        kw, qq, vt, want = dict(k0=k0, kt=[0.01 - 0.01j] * 3), q.astype(np.complex128), "complex", g[:, 1] + 1j * g[:, 2]
    else:
        kw, qq, vt, want = {}, W.gaussian_neutral(1, N, 8)[0], "real", g[:, 3]
    print("cube", case, level, flush=True)
    plan = _fp().Plan(torch.tensor(src, device="cuda"), 3, [101.0] * 3, value_type=vt, near_n=nn, near_order=qn,
                      corr_radius=rc, far_n=nf, far_order=qf, n_images=1, **kw)
    u = plan.apply(torch.tensor(qq, device="cuda")).cpu().numpy()
    assert plan.last_status() == 0
    plan.close()
    e = rel(u[rows], want)
    print("  vs exact %.2e (%d rows)" % (e, len(rows)))
    assert e < float(level)
