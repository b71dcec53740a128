"""Seeded synthetic inputs shaped like the paper's workloads.

Positions and strengths only: nothing in this module computes any part of the
FFT-PIM method, so both the GPU path's tests and the CPU oracle can draw their
inputs from it.  The paper's tetrahedral meshes are not available; these
stand in with the shapes it describes (quasi-uniform volume points with a near
grid of about one node per point, Table "near-zone"; a closed surface in a
2D-periodic cell for the Helmholtz case).

Every generator uses numpy's default_rng(seed).
"""
import numpy as np


def uniform_cube(n, seed, L=(1.0, 1.0, 1.0)):
    """n points uniform in [0, Lx) x [0, Ly) x [0, Lz)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)) * np.asarray(L, dtype=float)


def plus_minus_charges(n, seed):
    """n/2 charges +1 and n/2 charges -1 in random order (a neutral set)."""
    rng = np.random.default_rng(seed)
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    if n % 2:
        q[-1] = 0.0
    rng.shuffle(q)
    return q


def gaussian_neutral(nrhs, n, seed, dtype=np.float64):
    """nrhs real N(0,1) vectors with the mean removed from each (neutral)."""
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((nrhs, n))
    q -= q.mean(axis=1, keepdims=True)
    return q.astype(dtype)


def gaussian_complex(nrhs, n, seed, dtype=np.complex64):
    """nrhs complex vectors with real and imaginary parts N(0,1)."""
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    return q.astype(dtype)


def _real_sph_harm(l, m, theta, phi):
    """Real spherical harmonic of degree l, order m (theta polar angle)."""
    from scipy.special import sph_harm_y
    y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2.0) * y.real
    if m < 0:
        return np.sqrt(2.0) * y.imag
    return y.real


def smooth_closed_surface(n, seed, center=(0.5, 0.5, 0.25), semi_axes=(0.35, 0.35, 0.17),
                          lmax=4, amp=0.1, clip=0.3):
    """n points, area-uniform, on a random smooth star-shaped closed surface.

    The radial profile is 1 + sum_{l=1..lmax} sum_m a_lm Y_lm(theta, phi) with
    a_lm ~ N(0, amp/l^2), clipped to |delta r| <= clip, scaled by semi_axes
    and shifted to center.  Points are drawn uniformly in area by rejection
    against the surface's area element.
    """
    rng = np.random.default_rng(seed)
    coef = [(l, m, rng.normal(0.0, amp / l ** 2)) for l in range(1, lmax + 1)
            for m in range(-l, l + 1)]
    c = np.asarray(center, float)
    ax = np.asarray(semi_axes, float)

    def surface(theta, phi):
        dr = np.zeros_like(theta)
        for l, m, a in coef:
            dr += a * _real_sph_harm(l, m, theta, phi)
        rr = 1.0 + np.clip(dr, -clip, clip)
        d = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], -1)
        return c + ax * (rr[..., None] * d)

    def area_density(theta, phi, eps=1e-6):
        # |dX/dtheta x dX/dphi| / sin(theta): density w.r.t. the uniform sphere measure
        xt = (surface(theta + eps, phi) - surface(theta - eps, phi)) / (2 * eps)
        xp = (surface(theta, phi + eps) - surface(theta, phi - eps)) / (2 * eps)
        return np.linalg.norm(np.cross(xt, xp), axis=-1) / np.maximum(np.sin(theta), 1e-300)

    # bound the density on a fine probe grid
    tt, pp = np.meshgrid(np.linspace(0.01, np.pi - 0.01, 200), np.linspace(0, 2 * np.pi, 400), indexing="ij")
    dmax = 1.2 * area_density(tt, pp).max()
    out = []
    have = 0
    while have < n:
        m = 2 * (n - have) + 1024
        u = rng.random(m)
        theta = np.arccos(1 - 2 * u)
        phi = 2 * np.pi * rng.random(m)
        keep = rng.random(m) * dmax < area_density(theta, phi)
        pts = surface(theta[keep], phi[keep])
        out.append(pts)
        have += pts.shape[0]
    return np.concatenate(out)[:n]


# ---------------------------------------------------------------------------
# the workloads (seed = workload number)
# ---------------------------------------------------------------------------

def coulomb_cube_1k():
    """3D-periodic static Coulomb, unit cube, 1000 uniform points, +-1 charges."""
    return uniform_cube(1000, 1), plus_minus_charges(1000, 1)


def helmholtz_surface_100k(n=100_000):
    """2D-periodic Helmholtz with phase shift: points on a closed surface in a
    1 x 1 x 0.5 wavelength cell; complex64 N(0,1) strengths."""
    return smooth_closed_surface(n, 2), gaussian_complex(1, n, 2)[0]


def coulomb_cube_1m_batched(n=1_000_000, nrhs=64):
    """3D-periodic static Coulomb, 1M uniform points, 64 neutral Gaussian
    right-hand sides (float32)."""
    return uniform_cube(n, 3), gaussian_neutral(nrhs, n, 3, np.float32)


# ---------------------------------------------------------------------------
# coaxial shells in a 1D-periodic cell (the potential figure of Sec. 4)
# ---------------------------------------------------------------------------

def coax_shells_random(n, seed, r1=1.0, r2=2.0, L=1.0):
    """n points on two coaxial cylinders around the x axis (a third on the
    inner radius r1, the rest on r2), x uniform in [0, L)."""
    rng = np.random.default_rng(seed)
    n1 = n // 3
    rad = np.where(np.arange(n) < n1, r1, r2)
    th = rng.uniform(0.0, 2 * np.pi, n)
    return np.c_[rng.random(n) * L, rad * np.cos(th), rad * np.sin(th)]


def coax_shells(nx, ntheta, n_axis, r1=1.0, r2=2.0, sigma1=-1.0, sigma2=0.5, L=1.0):
    """Uniform surface charge on two coaxial cylinders (densities sigma1 on
    radius r1 and sigma2 on r2; the defaults make the cell neutral) sampled
    on an nx x ntheta midpoint grid per shell, plus n_axis zero-charge points
    on the x axis where the potential is observed.

    Returns (positions [N][3], charges [N], slice of the axis points)."""
    x = (np.arange(nx) + 0.5) / nx * L
    th = 2 * np.pi * (np.arange(ntheta) + 0.5) / ntheta
    X, T = np.meshgrid(x, th, indexing="ij")
    pts, q = [], []
    for rad, sig in ((r1, sigma1), (r2, sigma2)):
        pts.append(np.c_[X.ravel(), rad * np.cos(T.ravel()), rad * np.sin(T.ravel())])
        q.append(np.full(X.size, sig * (L / nx) * (2 * np.pi * rad / ntheta)))
    xa = (np.arange(n_axis) + 0.25) / n_axis * L
    pts.append(np.c_[xa, np.zeros(n_axis), np.zeros(n_axis)])
    q.append(np.zeros(n_axis))
    P = np.concatenate(pts)
    return P, np.concatenate(q), slice(P.shape[0] - n_axis, P.shape[0])


def dynamic_cube(n, seed, D=100.0):
    """n points uniform in a cube of side D centred in a 3D-periodic cell of
    period D + 1 (the dynamic 3D timing runs of Sec. 4.2); complex64 N(0,1)
    strengths."""
    rng = np.random.default_rng(seed)
    pos = 0.5 + rng.random((n, 3)) * D
    return pos, gaussian_complex(1, n, seed)[0]


def dynamic_cube_k0(n, D=100.0):
    """Free-space wavenumber of the dynamic runs of Sec. 4.2: the mean point
    spacing D / n^(1/3) is a twentieth of the wavelength."""
    return 2.0 * np.pi / (20.0 * D / n ** (1.0 / 3.0))


def multi_cell(ncells, seed, n_lo=5000, n_hi=500000, nblobs=8, sigma=0.05):
    """Independent cells of uneven size: N log-uniform in [n_lo, n_hi],
    periodic dimension 1, 2 or 3 (period 1), static or Helmholtz with
    k0 L uniform in [pi/2, 4 pi] (phase wavenumbers 0), redrawn within 0.05
    of 2 pi sqrt(j), j = 1..4, where the lattice sums have Rayleigh-Wood
    anomalies for a zero phase shift; points in Gaussian blobs of width
    sigma, wrapped on periodic axes and clipped to [0, 1] on the others;
    complex N(0,1) strengths, mean removed on static cells.

    Returns a list of dicts: dims, L, k0, kt, pos [N][3], q [N] complex128."""
    rng = np.random.default_rng(seed)
    cells = []
    for _ in range(ncells):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        dims = int(rng.integers(1, 4))
        static = bool(rng.integers(0, 2))
        k0 = 0.0
        if not static:
            while True:
                k0 = rng.uniform(0.5 * np.pi, 4 * np.pi)
                x = k0 / (2 * np.pi)
                if all(abs(x - np.sqrt(j)) > 0.05 for j in range(1, 5)):
                    break
        centres = rng.random((nblobs, 3))
        which = rng.integers(0, nblobs, n)
        pos = centres[which] + sigma * rng.standard_normal((n, 3))
        pos[:, :dims] = np.mod(pos[:, :dims], 1.0)
        # a wrapped coordinate can round up to exactly 1.0
        pos[:, :dims] = np.where(pos[:, :dims] >= 1.0, 0.0, pos[:, :dims])
        pos[:, dims:] = np.clip(pos[:, dims:], 0.0, 1.0)
        q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        if static:
            q -= q.mean()
        cells.append(dict(dims=dims, L=[1.0] * dims, k0=k0, kt=[0.0] * dims, pos=pos, q=q))
    return cells
