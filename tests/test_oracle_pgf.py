"""Pins of the oracle's periodic Green's function (Sec. 2) against closed
forms, tabulated lattice sums, brute-force image sums and invariants.

Every representation (the paper's series Eq. (pgf) / Eq. (lgf), the Ewald
splittings, the real-space 1D form) is checked against something that does
not come from the oracle itself.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import pgf as P
from oracle.psp import psp_forward

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lattice_constants.json")))
FOUR_PI = 4 * math.pi


def _u_at(lat, pos, q, m):
    """Potential at point m of a cell of charges, images of m kept."""
    d = pos[m][None, :] - np.delete(pos, m, axis=0)
    return np.dot(np.delete(q, m), P.pgf(d, lat)) + q[m] * P.pgf_self(lat)


# ---------------------------------------------------------------- 3D static

def test_nacl_madelung():
    lat = P.Lattice(3, [1, 1, 1])
    na = [[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]]
    cl = [[.5, 0, 0], [0, .5, 0], [0, 0, .5], [.5, .5, .5]]
    pos = np.array(na + cl, float)
    q = np.array([1.0] * 4 + [-1.0] * 4)
    u = _u_at(lat, pos, q, 0)
    assert abs(u.imag) < 1e-14
    assert u.real == pytest.approx(-GOLD["nacl_madelung"]["value"] / (FOUR_PI * 0.5), rel=1e-13)


def test_cscl_madelung_nonzero_dipole_cell():
    # the 2-ion cell carries a dipole: this pins the zero-cell-mean gauge
    lat = P.Lattice(3, [1, 1, 1])
    pos = np.array([[0, 0, 0], [.5, .5, .5]])
    q = np.array([1.0, -1.0])
    u = _u_at(lat, pos, q, 0)
    assert u.real == pytest.approx(-GOLD["cscl_madelung"]["value"] / (FOUR_PI * math.sqrt(3) / 2), rel=1e-13)


@pytest.mark.parametrize("L", [1.0, 2.5])
def test_simple_cubic_self_term(L):
    lat = P.Lattice(3, [L, L, L])
    assert (P.pgf_self(lat) * FOUR_PI * L).real == pytest.approx(GOLD["simple_cubic_self"]["value"], rel=1e-13)


def test_lgf3_series_matches_ewald():
    lat = P.Lattice(3, [1.0, 1.3, 0.8])
    rng = np.random.default_rng(11)
    r = rng.uniform(-0.5, 0.5, (60, 3)) * lat.L
    a = P.pgf(r, lat, "series")
    b = P.pgf(r, lat, "ewald")
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=0)


def test_lgf3_gauge_independent_of_axis_roles():
    # the zero-mean constant Lz/(12 Lx Ly) makes every role assignment agree
    L = np.array([1.0, 1.3, 0.8])
    x, y, z = 0.21, -0.33, 0.27
    vals = []
    for perm in [(0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1)]:
        r = np.array([x, y, z])[list(perm)]
        Lp = L[list(perm)]
        vals.append(P.lgf3_series(r[0:1], r[1:2], r[2:3], *Lp)[0])
    np.testing.assert_allclose(vals, vals[0], rtol=1e-12)


# ---------------------------------------------------------------- 2D static

def test_square_lattice_madelung_2d():
    lat = P.Lattice(2, [2.0, 2.0])
    pos = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0.0]])
    q = np.array([1.0, -1.0, -1.0, 1.0])
    u = _u_at(lat, pos, q, 0)
    assert (u * FOUR_PI).real == pytest.approx(-GOLD["square_2d_madelung"]["value"], rel=1e-12)


def test_lgf2_series_matches_ewald():
    lat = P.Lattice(2, [1.0, 1.4])
    rng = np.random.default_rng(12)
    r = rng.uniform(-0.5, 0.5, (60, 3))
    r[:, 2] = rng.uniform(-0.6, 0.6, 60)
    a = P.pgf(r, lat, "series")
    b = P.pgf(r, lat, "ewald")
    np.testing.assert_allclose(a, b, rtol=1e-11)


def test_dipole_layer_potential_jump_2d():
    # +1 at z=+a, -1 at z=-a per cell: u(+inf) - u(-inf) = P_z / A = 2a / A
    lat = P.Lattice(2, [1.0, 1.5])
    a = 0.2
    src = np.array([[0.1, 0.2, a], [0.4, 0.9, -a]])
    q = np.array([1.0, -1.0])
    obs = np.array([[0.3, 0.1, 12.0], [0.3, 0.1, -12.0]])
    u = psp_forward(lat, src, q, obs=obs, workers=1)
    assert (u[0] - u[1]).real == pytest.approx(2 * a / 1.5, rel=1e-12)


# ---------------------------------------------------------------- 1D static

def test_alternating_line_1d():
    lat = P.Lattice(1, [1.0])
    pos = np.array([[0, 0, 0], [0.5, 0, 0]])
    q = np.array([1.0, -1.0])
    u = _u_at(lat, pos, q, 0)
    assert u.real == pytest.approx(-GOLD["line_alternating"]["value"] / (FOUR_PI * 0.5), rel=1e-13)


def test_lgf1_series_matches_realspace_form():
    rng = np.random.default_rng(13)
    r = rng.uniform(-0.5, 0.5, (40, 3))
    a = P.lgf1_series(r[:, 0], np.hypot(r[:, 1], r[:, 2]), 1.0)
    b = P.lgf1_realspace(r[:, 0], r[:, 1], r[:, 2], 1.0)
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_coaxial_shells_uniform_axis_potential():
    # 1D-periodic coaxial shells r1=1 (sigma=-1) and r2=2 (sigma=+1/2), L=1:
    # a neutral cell whose on-axis potential is uniform and, in the gauge of
    # Eq. (lgf_1), equals -(lambda1 ln r1 + lambda2 ln r2)/(2 pi) = -ln 2.
    lat = P.Lattice(1, [1.0])
    nx, nt = 8, 16
    xs = (np.arange(nx) + 0.5) / nx
    th = 2 * np.pi * np.arange(nt) / nt
    pts, q = [], []
    for R, sigma in [(1.0, -1.0), (2.0, 0.5)]:
        for x in xs:
            for t in th:
                pts.append([x, R * np.cos(t), R * np.sin(t)])
                q.append(sigma * 2 * np.pi * R / (nx * nt))
    obs = np.array([[x, 0.0, 0.0] for x in np.linspace(0, 1, 5, endpoint=False)])
    u = psp_forward(lat, np.array(pts), np.array(q), obs=obs, workers=1)
    np.testing.assert_allclose(u.real, -math.log(2.0), rtol=1e-12)


# ---------------------------------------------------------------- Helmholtz

def _brute_force(lat, r, reach):
    """Direct Eq. (2) image sum; converges like exp(Im(k0) R) for lossy k0."""
    rng = [range(-reach, reach + 1) if c < lat.dims else range(0, 1) for c in range(3)]
    I = np.array(np.meshgrid(*rng, indexing="ij")).reshape(3, -1).T
    R = I * lat.L
    dist = np.linalg.norm(r[None, :] - R, axis=1)
    terms = np.exp(-1j * (R @ lat.kt)) * np.exp(-1j * lat.k0 * dist) / (FOUR_PI * dist)
    order = np.argsort(-np.abs(terms))
    return np.sum(terms[order][::-1])


@pytest.mark.parametrize("dims,reach", [(3, 14), (2, 40), (1, 14)])
def test_lossy_brute_force_image_sum(dims, reach):
    lat = P.Lattice(dims, [1.0, 1.2, 0.9][:dims], k0=2.0 - 3.0j, kt=[0.7, -0.4, 0.3][:dims])
    rng = np.random.default_rng(14 + dims)
    for _ in range(4):
        r = rng.uniform(-0.45, 0.45, 3)
        bf = _brute_force(lat, r, reach)
        for method in ("series", "ewald"):
            val = P.pgf(r[None, :], lat, method)[0]
            assert abs(val - bf) <= 1e-10 * abs(bf), (method, val, bf)


def test_bloch_series_2d_helmholtz_with_phase():
    k = 2 * np.pi
    Lx, Ly = 1.0, 1.0
    kx0, ky0 = 0.3 * k, 0.1 * k
    x = np.array([0.13]); y = np.array([-0.21]); z = np.array([0.37])
    base = P.pgf2_series(x, y, z, Lx, Ly, k, kx0, ky0)[0]
    sx = P.pgf2_series(x + Lx, y, z, Lx, Ly, k, kx0, ky0)[0]
    sy = P.pgf2_series(x, y - Ly, z, Lx, Ly, k, kx0, ky0)[0]
    assert sx == pytest.approx(np.exp(-1j * kx0 * Lx) * base, rel=1e-12)
    assert sy == pytest.approx(np.exp(+1j * ky0 * Ly) * base, rel=1e-12)


def test_2d_helmholtz_series_matches_ewald_c2_parameters():
    k = 2 * np.pi
    lat = P.Lattice(2, [1.0, 1.0], k0=k, kt=[0.3 * k, 0.1 * k])
    rng = np.random.default_rng(15)
    r = rng.uniform(-0.5, 0.5, (40, 3))
    r[:, 2] = rng.choice([-1, 1], 40) * rng.uniform(0.05, 0.5, 40)
    np.testing.assert_allclose(P.pgf(r, lat, "series"), P.pgf(r, lat, "ewald"), rtol=1e-11)


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_fig2_parameters_two_representations(dims):
    # Fig. 2 of the paper: L = 1, k0 = -1-j, k_t = (1-j, 1+j, -1+j), r = (1/2, 1/2, 1/2)
    lat = P.Lattice(dims, [1, 1, 1], k0=-1 - 1j, kt=[1 - 1j, 1 + 1j, -1 + 1j][:dims])
    r = np.array([[0.5, 0.5, 0.5]])
    a = P.pgf(r, lat, "series")[0]
    b = P.pgf(r, lat, "ewald")[0]
    assert a == pytest.approx(b, rel=1e-12)
    if dims == 1:
        # the spectral sum is also Bloch-consistent
        c = P.pgf1_series(r[:, 0] + 1.0, np.hypot(r[:, 1], r[:, 2]), 1.0, lat.k0, lat.kt[0])[0]
        assert c == pytest.approx(np.exp(-1j * lat.kt[0]) * a, rel=1e-12)


def test_reciprocity():
    k = 2 * np.pi
    rng = np.random.default_rng(16)
    r = rng.uniform(-0.5, 0.5, (20, 3))
    for dims in (2, 3):
        kt = np.array([0.3 * k, 0.1 * k, 0.2 * k])[:dims]
        a = P.pgf(r, P.Lattice(dims, [1, 1, 1], k0=k, kt=kt))
        b = P.pgf(-r, P.Lattice(dims, [1, 1, 1], k0=k, kt=-kt))
        np.testing.assert_allclose(a, b, rtol=1e-11)


def test_periodicity_without_phase():
    lat = P.Lattice(3, [1.0, 1.0, 1.0], k0=3.0)
    rng = np.random.default_rng(17)
    r = rng.uniform(-0.5, 0.5, (10, 3))
    shift = np.array([1.0, -2.0, 1.0])
    np.testing.assert_allclose(P.pgf(r + shift, lat, "ewald"), P.pgf(r, lat, "series"), rtol=1e-11)


def test_neutral_sum_gauge_invariance():
    # for neutral charges adding a constant to G changes nothing
    lat = P.Lattice(3, [1, 1, 1])
    rng = np.random.default_rng(18)
    src = rng.random((12, 3))
    q = rng.standard_normal(12)
    q -= q.mean()
    obs = rng.random((3, 3))
    u1 = psp_forward(lat, src, q, obs=obs, workers=1)
    G = P.pgf(obs[:, None, :] - src[None, :, :], lat) + 0.123
    np.testing.assert_allclose(G @ q, u1, rtol=1e-12, atol=1e-14)
