"""Pins of the oracle's phase-shifted and Helmholtz paths against the plain
image sum of Sec. 2, Eq. (2).

For a lossy free-space wavenumber (Im k0 < 0) and a real phase shift the
image sum of Eq. (2) converges like exp(Im(k0) R), so a direct sum over a
finite block of images is an exact reference that shares nothing with the
oracle's series or Ewald evaluators.  These tests pin:

  * the Bloch factor applied when a displacement is reduced into the cell
    (G^p(r) = exp(-j k_t . R_j) G^p(r - R_j), from Eq. (2)), at displacements
    several cells away from the zeroth cell;
  * the self coefficient lim_{r->0} [G^p(r) - G0(r)] = sum_{i != 0}
    exp(-j k_t . R_i) G0(-R_i) (the n = m term of Eq. (1) with the singular
    image removed) for 2D and 3D periodicity with a phase shift;
  * the step-by-step algorithm of Sec. 3 with a Helmholtz kernel and a phase
    shift, against the direct pair sum of Eq. (1), converging as the
    correction radius and the far grid grow.
"""
import math

import numpy as np
import pytest

from oracle import pgf as P
from oracle import steps as S
from oracle.psp import psp_forward

FOUR_PI = 4 * math.pi


def _image_block(lat, center, reach):
    rng = [range(center[c] - reach, center[c] + reach + 1) if c < lat.dims else range(0, 1) for c in range(3)]
    return np.array(np.meshgrid(*rng, indexing="ij")).reshape(3, -1).T


def _image_sum(lat, r, reach, skip_zero=False):
    """Eq. (2) summed directly over the images within `reach` cells of the
    image nearest to r, smallest terms first."""
    center = [int(round(r[c] / lat.L[c])) if c < lat.dims else 0 for c in range(3)]
    I = _image_block(lat, center, reach)
    if skip_zero:
        I = I[np.any(I != 0, axis=1)]
    R = I * lat.L
    dist = np.linalg.norm(r[None, :] - R, axis=1)
    terms = np.exp(-1j * (R @ lat.kt)) * np.exp(-1j * lat.k0 * dist) / (FOUR_PI * dist)
    order = np.argsort(np.abs(terms))
    return np.sum(terms[order])


LOSSY = {
    1: P.Lattice(1, [1.0], k0=2.0 - 3.0j, kt=[0.9]),
    2: P.Lattice(2, [1.0, 1.2], k0=2.5 - 3.0j, kt=[0.9, -1.3]),
    3: P.Lattice(3, [1.0, 1.2, 0.9], k0=2.0 - 3.0j, kt=[0.7, -1.1, 0.5]),
}


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_bloch_factor_outside_the_cell(dims):
    # displacements one to three cells away: the oracle reduces them into the
    # cell and multiplies by exp(-j k_t . R_j); the direct sum never reduces
    lat = LOSSY[dims]
    rng = np.random.default_rng(100 + dims)
    shifts = np.array([[1, -2, 1], [-3, 1, 2], [2, 2, -1], [0, -1, 3]])
    for s in shifts:
        r = rng.uniform(-0.45, 0.45, 3) * lat.L
        if dims == 1:
            # the 1D Helmholtz series needs a transverse distance (no small-rho form)
            r[1:] = rng.uniform(0.25, 0.4, 2)
        r = r + s * lat.L * (np.arange(3) < dims)
        want = _image_sum(lat, r, 16)
        got = P.pgf(r[None, :], lat)[0]
        assert abs(got - want) <= 1e-10 * abs(want), (s, got, want)


def test_bloch_factor_c2_displacement():
    # the displacement quoted for the 100k surface workload's lattice class,
    # (0.83, -0.71, 0.3): reduced by R_j = (1, -1, 0)
    lat = P.Lattice(2, [1.0, 1.0], k0=2 * math.pi - 3.0j, kt=[0.3 * 2 * math.pi, 0.1 * 2 * math.pi])
    r = np.array([0.83, -0.71, 0.3])
    want = _image_sum(lat, r, 16)
    for method in ("series", "ewald"):
        got = P.pgf(r[None, :], lat, method)[0]
        assert abs(got - want) <= 1e-11 * abs(want), (method, got, want)


@pytest.mark.parametrize("dims", [2, 3])
def test_self_coefficient_with_phase(dims):
    # lim_{r->0}[G^p - G0] is the image sum without the zeroth image
    lat = LOSSY[dims]
    want = _image_sum(lat, np.zeros(3), 16, skip_zero=True)
    got = P.pgf_self(lat)
    assert abs(got - want) <= 1e-11 * abs(want), (got, want)


def test_self_coefficient_c2_class():
    # the phase and wavenumber ratios of the surface workload, made lossy
    k = 2 * math.pi
    lat = P.Lattice(2, [1.0, 1.0], k0=k - 2.5j, kt=[0.3 * k, 0.1 * k])
    want = _image_sum(lat, np.zeros(3), 20, skip_zero=True)
    assert abs(P.pgf_self(lat) - want) <= 1e-11 * abs(want)


@pytest.mark.parametrize("dims", [2, 3])
def test_self_coefficient_phase_dependence(dims):
    # images i and -i pair up to cos(k_t . R_i) G0(|R_i|): the coefficient is
    # even in k_t, but a dropped phase (k_t -> 0) changes it, which the
    # image-sum pins above would see
    lat = LOSSY[dims]
    flipped = P.Lattice(dims, lat.L, lat.k0, -lat.kt)
    dropped = P.Lattice(dims, lat.L, lat.k0, 0 * lat.kt)
    a = P.pgf_self(lat)
    assert abs(P.pgf_self(flipped) - a) <= 1e-12 * abs(a)
    assert abs(P.pgf_self(dropped) - a) > 1e-2 * abs(a)


def test_algorithm_with_bloch_phase_converges_to_direct_sum():
    # the surface workload's lattice class (2D periodic, k0 = 2 pi, phase
    # (0.3, 0.1) k0) on a small point set: the method's error against the
    # direct pair sum of Eq. (1) falls as r_c and the far grid grow
    k = 2 * math.pi
    lat = P.Lattice(2, [1.0, 1.0], k0=k, kt=[0.3 * k, 0.1 * k])
    rng = np.random.default_rng(21)
    N = 90
    src = np.column_stack([rng.random(N), rng.random(N), 0.1 + 0.3 * rng.random(N)])
    q = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ref = psp_forward(lat, src, q, workers=1)
    errs = []
    for rc, nf, qf in [(4, (10, 10, 8), 4), (6, (14, 14, 10), 6)]:
        m = S.FFTPIM(lat, S.Params((16, 16, 8), 4, rc, nf, qf, 1), src)
        u = m.apply(q)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    # the far grid dominates at these sizes: 1.1e-2 -> 3.5e-4 (a dropped or
    # flipped phase anywhere gives an error of order one)
    assert errs[1] < errs[0] / 10 and errs[0] < 3e-2, errs
    assert errs[1] < 1e-3, errs
