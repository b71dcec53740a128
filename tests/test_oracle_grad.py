"""Pins of the oracle's position gradients (oracle/grad.py).

  * steps_grad, the gradient of the discrete operator of Sec. 3, against
    central finite differences of that operator (positions moved by h = 1e-6
    inside their stencil boxes, the grids and tables held fixed);
  * psp_grad, the gradient of the exact sum of Eq. (1), against the plain
    image sum of Eq. (2) differentiated term by term for a lossy k0 (which
    converges like exp(Im(k0) R));
  * the discrete gradient approaching the exact one as the method is refined.
"""
import copy
import math

import numpy as np
import pytest

from oracle import grad as G
from oracle import pgf as P
from oracle import steps as S

FOUR_PI = 4 * math.pi


def _moved(m, src):
    """The same discrete operator (grids and tables fixed) for moved points."""
    mm = copy.copy(m)
    mm.src = mm.obs = np.asarray(src, dtype=float)
    mm.st_src = mm.st_obs = S._Stencils(mm.src, m.origin, m.h, m.prm.near_q, m.prm.near_n)
    mm.fst_src = S._Stencils(mm.src, m.origin_fs, m.Df, m.prm.far_q, m.prm.far_n)
    mm.fst_obs = S._Stencils(mm.src, m.origin_fo, m.Df, m.prm.far_q, m.prm.far_n)
    return mm


def _loss(m, q, g):
    return float(np.real(np.sum(np.conj(g) * m.apply(q))))


CASES = [
    ("npsp3", P.Lattice(3, [1, 1, 1]), False),
    ("helm2_bloch", P.Lattice(2, [1, 1.2], 2 * math.pi, [0.3 * 2 * math.pi, 0.1 * 2 * math.pi]), True),
    ("helm1_cphase", P.Lattice(1, [1.0], 3.0, [0.7 - 0.2j]), True),
    ("phase3_lossy", P.Lattice(3, [1, 1.1, 0.9], 2.0 - 0.5j, [0.4, -0.3, 0.2]), True),
]


@pytest.mark.parametrize("name,lat,cplx", CASES, ids=[c[0] for c in CASES])
def test_discrete_gradient_matches_finite_differences(name, lat, cplx):
    rng = np.random.default_rng(5)
    N = 36
    src = rng.random((N, 3)) * lat.L
    if lat.dims < 3:
        src[:, lat.dims:] = 0.1 + 0.3 * rng.random((N, 3 - lat.dims))
    lo, hi = np.zeros(3), np.array(lat.L, float)
    lo[lat.dims:], hi[lat.dims:] = 0.0, 0.5
    m = S.FFTPIM(lat, S.Params(10, 3, 3, 9, 3, 1), src, lo=lo, hi=hi)
    if cplx:
        q = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    else:
        q = rng.standard_normal(N)
        q -= q.mean()
        g = rng.standard_normal(N)
    rows = np.array([0, 7, 19])
    got = G.steps_grad(m, q, g, rows)
    h = 1e-6
    for t, k in enumerate(rows):
        for c in range(3):
            sp, sm = src.copy(), src.copy()
            sp[k, c] += h
            sm[k, c] -= h
            mp, mn = _moved(m, sp), _moved(m, sm)
            # the moved point keeps its stencil boxes on every grid
            assert np.array_equal(mp.st_src.s, m.st_src.s) and np.array_equal(mn.st_src.s, m.st_src.s)
            assert np.array_equal(mp.fst_src.s, m.fst_src.s) and np.array_equal(mp.fst_obs.s, m.fst_obs.s)
            fd = (_loss(mp, q, g) - _loss(mn, q, g)) / (2 * h)
            scale = np.abs(got).max()
            assert abs(got[t, c] - fd) <= 1e-6 * scale, (k, c, got[t, c], fd)


def _image_sum_grad(lat, r, reach):
    """grad of sum_i phi_i G0(r - R_i) over the images within reach cells."""
    rngs = [range(-reach, reach + 1) if c < lat.dims else range(0, 1) for c in range(3)]
    I = np.array(np.meshgrid(*rngs, indexing="ij")).reshape(3, -1).T
    R = I * lat.L
    terms = np.exp(-1j * (R @ lat.kt))[:, None] * G.grad_g0(r[None, :] - R, lat.k0)
    order = np.argsort(np.abs(terms).sum(axis=1))
    return terms[order].sum(axis=0)


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_exact_gradient_against_lossy_image_sum(dims):
    lat = P.Lattice(dims, [1.0, 1.2, 0.9][:dims], k0=2.0 - 3.0j, kt=[0.7, -0.4, 0.3][:dims])
    rng = np.random.default_rng(30 + dims)
    src = rng.random((6, 3)) * np.array([1.0, 1.2, 0.9])
    q = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    g = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    rows = [0, 3]
    got = G.psp_grad(lat, src, q, g, rows)
    for t, k in enumerate(rows):
        want = np.zeros(3)
        for n in range(6):
            if n == k:
                continue
            a = _image_sum_grad(lat, src[k] - src[n], 16)
            b = -_image_sum_grad(lat, src[n] - src[k], 16)
            want += np.real(np.conj(g[k]) * a * q[n] + np.conj(g[n]) * b * q[k])
        assert np.abs(got[t] - want).max() <= 1e-9 * np.abs(want).max(), (got[t], want)


def test_discrete_gradient_approaches_exact():
    # the same surface problem at two correction radii: the error of the
    # discrete gradient against the exact one falls
    from paper_2312_02376_amd import workloads as W
    k = 2 * math.pi
    lat = P.Lattice(2, [1.0, 1.0], k, [0.3 * k, 0.1 * k])
    src = W.smooth_closed_surface(400, 3)
    rng = np.random.default_rng(2)
    q = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    g = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    rows = np.arange(0, 400, 80)
    exact = G.psp_grad(lat, src, q, g, rows)
    errs = []
    for rc in (4, 8):
        m = S.FFTPIM(lat, S.Params((32, 32, 16), 4, rc, (20, 20, 14), 7, 1), src)
        d = G.steps_grad(m, q, g, rows)
        errs.append(np.linalg.norm(d - exact) / np.linalg.norm(exact))
    assert errs[1] < 0.3 * errs[0] and errs[1] < 1e-3, errs
