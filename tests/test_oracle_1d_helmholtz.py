"""Pins of the oracle's 1D-periodic Helmholtz and phase-shifted kernels
(Sec. 2, Eq. (pgf_1)) at every transverse distance, including the self
coefficient.

The paper's Hankel series converges only when the distance rho from the
periodic axis is not small; the oracle switches to a 1D Ewald splitting there.
Each part is checked against something it shares no code with:
  * the Ewald form against the paper's series where both converge (real,
    lossy and complex wavenumbers);
  * both against the direct image sum of Eq. (2) for a lossy k0 (which
    converges like exp(Im(k0) R)), down to rho = 0;
  * the self coefficient lim_{r->0}[G^p - G0] against the closed form of
    sum_{l != 0} exp(-j kx0 l L) exp(-j k0 |l| L)/(4 pi |l| L)
      = -(ln(1 - e^{-j(k0 + kx0)L}) + ln(1 - e^{-j(k0 - kx0)L}))/(4 pi L),
    the logarithmic series sum_l w^l / l = -ln(1 - w) (real kx0).
"""
import math

import numpy as np
import pytest

from oracle import pgf as P

FOUR_PI = 4 * math.pi


def _image_sum(lat, r, reach, skip_zero=False):
    l0 = int(round(r[0] / lat.L[0]))
    ls = np.arange(l0 - reach, l0 + reach + 1)
    if skip_zero:
        ls = ls[ls != 0]
    R = np.zeros((ls.size, 3))
    R[:, 0] = ls * lat.L[0]
    dist = np.linalg.norm(r[None, :] - R, axis=1)
    terms = np.exp(-1j * lat.kt[0] * R[:, 0]) * np.exp(-1j * lat.k0 * dist) / (FOUR_PI * dist)
    return np.sum(terms[np.argsort(np.abs(terms))])


@pytest.mark.parametrize("k0,kt", [(2 * math.pi * 0.8, 0.3), (3.0 - 0.5j, 0.7), (1.0, 1 - 1j),
                                   (0.0, 0.9), (1.3, 0.0), (5.0, 2.0 - 0.3j), (-1 - 1j, 1 - 1j)])
def test_ewald_matches_hankel_series(k0, kt):
    lat = P.Lattice(1, [1.0], k0, [kt])
    rng = np.random.default_rng(3)
    r = np.c_[rng.uniform(-1.5, 1.5, 24), rng.uniform(0.2, 0.5, 24), rng.uniform(-0.4, 0.4, 24)]
    a = P.ewald1(r, lat)
    b = P.pgf1_series(r[:, 0], np.hypot(r[:, 1], r[:, 2]), 1.0, lat.k0, lat.kt[0])
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-13 * np.abs(b).max())


@pytest.mark.parametrize("rho", [0.0, 1e-3, 0.05, 0.2])
def test_small_rho_against_lossy_image_sum(rho):
    lat = P.Lattice(1, [1.0], k0=2.0 - 2.5j, kt=[0.9])
    rng = np.random.default_rng(int(rho * 1000) + 5)
    for _ in range(4):
        x = rng.uniform(-0.45, 0.45)
        if abs(x) < 0.05:
            x = 0.3
        ang = rng.uniform(0, 2 * math.pi)
        r = np.array([x + rng.integers(-2, 3), rho * math.cos(ang), rho * math.sin(ang)])
        want = _image_sum(lat, r, 24)
        got = P.pgf(r[None, :], lat)[0]
        assert abs(got - want) <= 1e-11 * abs(want), (r, got, want)


@pytest.mark.parametrize("k0,kt", [(2.0, 0.5), (3.0 - 0.4j, 1.1), (0.0, 0.9), (4.0, 0.0), (2 * math.pi * 0.6, -1.7)])
def test_self_coefficient_closed_form(k0, kt):
    lat = P.Lattice(1, [1.3], k0, [kt])
    L = 1.3
    k0c = complex(k0)
    want = -(np.log(1 - np.exp(-1j * (k0c + kt) * L)) + np.log(1 - np.exp(-1j * (k0c - kt) * L))) / (FOUR_PI * L)
    got = P.pgf_self(lat)
    assert abs(got - want) <= 1e-12 * abs(want), (got, want)


def test_self_coefficient_lossy_image_sum():
    lat = P.Lattice(1, [1.0], k0=2.0 - 3.0j, kt=[0.7])
    want = _image_sum(lat, np.zeros(3), 24, skip_zero=True)
    got = P.pgf_self(lat)
    assert abs(got - want) <= 1e-12 * abs(want)
    # a flipped phase sign is visible only through exp(-j k0 |R|) pairing:
    # the coefficient is even in kx0, a dropped phase is not
    dropped = P.pgf_self(P.Lattice(1, [1.0], lat.k0, [0.0]))
    assert abs(dropped - got) > 1e-3 * abs(got)


def test_small_rho_limit_is_continuous():
    # G^p - G0 is smooth at the axis: the Ewald form at rho = 0 and at tiny
    # rho agree, and its r -> 0 limit is the self coefficient
    lat = P.Lattice(1, [1.0], k0=2.0, kt=[0.4])
    for x in (0.2, -0.31):
        a = P.pgf(np.array([[x, 0.0, 0.0]]), lat)[0]
        b = P.pgf(np.array([[x, 1e-6, 0.0]]), lat)[0]
        assert abs(a - b) <= 1e-9 * abs(a)
    d = 1e-6  # G^p - G0 - C_self is O(d) (a smooth function's first-order term)
    g0 = np.exp(-1j * 2.0 * d) / (FOUR_PI * d)
    assert abs(P.pgf(np.array([[d, 0.0, 0.0]]), lat)[0] - g0 - P.pgf_self(lat)) < 1e-6
