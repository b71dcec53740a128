"""Periodic Green's function G^p of Sec. 2, evaluated in FP64 on the CPU.

Test infrastructure: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module.

Conventions (Sec. 2, Eq. (1)-(2)):
  * time dependence exp(+j w t); free-space kernel G0(r) = exp(-j k0 |r|)/(4 pi |r|);
  * periodic axes are x (1D), x and y (2D), x, y and z (3D);
  * the image i (a vector of integers on the periodic axes) sits at
    R_i = (i_x Lx, i_y Ly, i_z Lz) and carries the phase exp(-j k_t . R_i).

Representations used, per periodicity:
  * the paper's Floquet series, Eq. (pgf_1)-(pgf_3);
  * the paper's neutral static series, Eq. (lgf_1)-(lgf_3);
  * textbook Ewald splittings (3D, 2D and 1D, static and Helmholtz, with
    phase; the 1D spectral part in incomplete-gamma form) and, for the neutral
    1D static case at small transverse distance, the real-space series that
    follows from Gradshteyn & Ryzhik 8.526.1.
The paper's series converge exponentially only when the transverse distance is
not small (end of Sec. 2); the dispatcher `pgf` picks the paper's series when
it converges quickly and an Ewald splitting otherwise.  The test suite checks
the representations against one another, against closed forms (Madelung
constants) and against brute-force image sums.

Readings taken where the text is ambiguous or garbled:
  * k_yn = k_y0 + 2 pi n / L_y (the text after Eq. (pgf) prints L_z);
  * every square root has Im <= 0; on the real axis Re >= 0 (outgoing);
  * "k_xm^2" etc. are bilinear squares, so complex phase shifts continue
    the series analytically;
  * neutral static (NPSP) gauges: 3D adds Lz/(12 Lx Ly) to Eq. (lgf_3) so the
    potential has zero cell mean; 2D and 1D are taken as printed (their
    constants cancel for neutral sources anyway).
"""
import math

import numpy as np
from scipy import special as sp

FOUR_PI = 4.0 * math.pi
EULER_GAMMA = 0.57721566490153286061

# Transverse-distance thresholds (as a fraction of the shortest period) above
# which the paper's series are used; below them the Ewald splitting is used.
SERIES_MIN_FRACTION = {"npsp": 0.3, "dyn": 0.3}


class Lattice:
    """Periodicity, periods, free-space wavenumber and phase shift (Sec. 2)."""

    def __init__(self, dims, L, k0=0.0, kt=(0.0, 0.0, 0.0)):
        if dims not in (1, 2, 3):
            raise ValueError("dims must be 1, 2 or 3")
        self.dims = int(dims)
        Lf = np.ones(3)
        Lv = np.atleast_1d(np.asarray(L, dtype=float))
        Lf[: len(Lv)] = Lv
        self.L = Lf
        self.k0 = complex(k0)
        ktf = np.zeros(3, dtype=complex)
        ktv = np.atleast_1d(np.asarray(kt, dtype=complex))
        ktf[: min(len(ktv), 3)] = ktv[:3]
        ktf[self.dims:] = 0.0
        self.kt = ktf

    @property
    def npsp(self):
        """No-phase static periodic case (Sec. 2, before Eq. (neutral))."""
        return self.k0 == 0 and not np.any(self.kt != 0)

    @property
    def real_kernel(self):
        return self.npsp

    def __repr__(self):
        return "Lattice(dims=%d, L=%s, k0=%s, kt=%s)" % (
            self.dims, self.L.tolist(), self.k0, self.kt.tolist())


# ----------------------------------------------------------------------------
# basic pieces
# ----------------------------------------------------------------------------

def g0(r, k0):
    """Free-space kernel G0(r) = exp(-j k0 |r|)/(4 pi |r|) (Sec. 2, after Eq. (2))."""
    r = np.asarray(r, dtype=float)
    R = np.sqrt(np.sum(r * r, axis=-1))
    return np.exp(-1j * complex(k0) * R) / (FOUR_PI * R)


def csqrt_im_nonpos(w):
    """Square root with non-positive imaginary part (text after Eq. (pgf))."""
    s = np.sqrt(np.asarray(w, dtype=complex))
    return np.where(s.imag > 0, -s, s)


def reduce_to_cell(r, lat):
    """Shift r by a lattice vector R_j into [-L/2, L/2] on the periodic axes.

    From Eq. (2), G^p(r) = exp(-j k_t . R_j) G^p(r - R_j); returns r - R_j and
    that phase factor.
    """
    r = np.array(r, dtype=float, copy=True)
    phase_arg = np.zeros(r.shape[:-1], dtype=complex)
    for c in range(lat.dims):
        n = np.round(r[..., c] / lat.L[c])
        r[..., c] -= n * lat.L[c]
        phase_arg += lat.kt[c] * n * lat.L[c]
    return r, np.exp(-1j * phase_arg)


def _shell(s):
    """All (m, n) integer pairs with max(|m|, |n|) == s."""
    if s == 0:
        return np.array([0]), np.array([0])
    a = np.arange(-s, s + 1)
    m = np.concatenate([a, a, np.full(2 * s - 1, -s), np.full(2 * s - 1, s)])
    n = np.concatenate([np.full(2 * s + 1, -s), np.full(2 * s + 1, s),
                        np.arange(-s + 1, s), np.arange(-s + 1, s)])
    return m, n


def _shell_sum(term_fn, P, s_min, tol=1e-17, max_shell=20000):
    """Sum term_fn(m, n) -> (P, K) over square shells until converged."""
    total = np.zeros(P, dtype=complex)
    quiet = 0
    for s in range(max_shell):
        m, n = _shell(s)
        t = term_fn(m, n)
        total += t.sum(axis=1)
        mag = np.abs(t).max(axis=1)
        if s >= s_min and np.all(mag <= tol * np.maximum(np.abs(total), 1e-300)):
            quiet += 1
            if quiet >= 2:
                return total
        else:
            quiet = 0
    raise RuntimeError("spectral series did not converge in %d shells" % max_shell)


# ----------------------------------------------------------------------------
# the paper's Floquet series, Eq. (pgf)
# ----------------------------------------------------------------------------

def pgf2_series(x, y, z, Lx, Ly, k0, kx0, ky0):
    """Eq. (pgf_2): 2D-periodic (x, y) Floquet series; needs |z| > 0."""
    x, y, z = (np.asarray(v, dtype=float) for v in (x, y, z))
    A = Lx * Ly
    az = np.abs(z)
    k0 = complex(k0)

    def term(m, n):
        kx = kx0 + 2 * math.pi * m / Lx
        ky = ky0 + 2 * math.pi * n / Ly
        kz = csqrt_im_nonpos(k0 * k0 - kx * kx - ky * ky)
        arg = np.outer(x, kx) + np.outer(y, ky) + np.outer(az, kz)
        return np.exp(-1j * arg) / (2j * kz * A)

    s_min = int(math.ceil((abs(k0) + abs(kx0) + abs(ky0)) * max(Lx, Ly) / (2 * math.pi))) + 2
    return _shell_sum(term, x.size, s_min)


def pgf3_series(x, y, z, L, k0, kt):
    """Eq. (pgf_3): 3D-periodic Floquet series with the z images summed in
    closed form; valid for |z| <= Lz, needs |z| > 0."""
    x, y, z = (np.asarray(v, dtype=float) for v in (x, y, z))
    Lx, Ly, Lz = L
    kx0, ky0, kz0 = kt
    A = Lx * Ly
    az = np.abs(z)
    k0 = complex(k0)

    def term(m, n):
        kx = kx0 + 2 * math.pi * m / Lx
        ky = ky0 + 2 * math.pi * n / Ly
        kz = csqrt_im_nonpos(k0 * k0 - kx * kx - ky * ky)
        am = np.exp(-1j * (kz - kz0) * Lz)
        ap = np.exp(-1j * (kz + kz0) * Lz)
        lateral = np.exp(-1j * (np.outer(x, kx) + np.outer(y, ky)))
        zpart = (np.exp(-1j * np.outer(az, kz))
                 + am * np.exp(-1j * np.outer(z, kz)) / (1 - am)
                 + ap * np.exp(1j * np.outer(z, kz)) / (1 - ap))
        return lateral * zpart / (2j * kz * A)

    s_min = int(math.ceil((abs(k0) + np.abs(kt).max()) * max(Lx, Ly) / (2 * math.pi))) + 2
    return _shell_sum(term, x.size, s_min)


def pgf1_series(x, rho, Lx, k0, kx0, tol=1e-17, max_terms=200000):
    """Eq. (pgf_1): 1D-periodic (x) Floquet series of Hankel functions; needs rho > 0."""
    x = np.asarray(x, dtype=float)
    rho = np.asarray(rho, dtype=float)
    k0 = complex(k0)
    total = np.zeros(x.size, dtype=complex)
    m_min = int(math.ceil((abs(k0) + abs(kx0)) * Lx / (2 * math.pi))) + 2
    quiet = 0
    for s in range(max_terms):
        ms = np.array([0]) if s == 0 else np.array([-s, s])
        kx = kx0 + 2 * math.pi * ms / Lx
        krho = csqrt_im_nonpos(k0 * k0 - kx * kx)
        arg = np.outer(rho, krho)
        h = sp.hankel2(0, arg)
        t = np.exp(-1j * np.outer(x, kx)) * h / (4j * Lx)
        total += t.sum(axis=1)
        mag = np.abs(t).max(axis=1)
        if s >= m_min and np.all(mag <= tol * np.maximum(np.abs(total), 1e-300)):
            quiet += 1
            if quiet >= 2:
                return total
        else:
            quiet = 0
    raise RuntimeError("Eq. (pgf_1) series did not converge")


# ----------------------------------------------------------------------------
# the paper's neutral static series, Eq. (lgf)
# ----------------------------------------------------------------------------

K0_CUTOFF = 41.0   # K0(41) ~ 3e-19


def _log_layer(a, theta):
    """ln(1 - 2 e^{-a} cos(theta) + e^{-2a}) evaluated without cancellation."""
    return np.log(np.expm1(-a) ** 2 + 4.0 * np.exp(-a) * np.sin(0.5 * theta) ** 2)


def lgf1_series(x, rho, Lx):
    """Eq. (lgf_1): neutral static 1D-periodic series; needs rho > 0."""
    x = np.asarray(x, dtype=float)
    rho = np.asarray(rho, dtype=float)
    out = -np.log(rho) / (2 * math.pi * Lx)
    mmax = int(math.ceil(K0_CUTOFF * Lx / (2 * math.pi * rho.min()))) + 1
    for m in range(1, mmax + 1):
        out += sp.k0(2 * m * math.pi * rho / Lx) * np.cos(2 * m * math.pi * x / Lx) / (math.pi * Lx)
    return out


def _k0_lattice_sum(x, y, z, Lx, Ly, Lz, ks):
    """(1/(pi Lx)) sum_{m>=1} sum_{n, k in ks} K0(2 m pi rho_nk / Lx) cos(2 m pi x / Lx)."""
    out = np.zeros(x.size)
    m = 1
    while True:
        cutoff = K0_CUTOFF * Lx / (2 * math.pi * m)
        nmax = int(math.ceil(cutoff / Ly)) + 1
        any_term = False
        cosx = np.cos(2 * m * math.pi * x / Lx)
        for k in ks:
            zz = k * Lz + z
            if np.min(np.abs(zz)) > cutoff:
                continue
            for n in range(-nmax, nmax + 1):
                yy = n * Ly + y
                rho = np.sqrt(yy * yy + zz * zz)
                if rho.min() > cutoff:
                    continue
                any_term = True
                out += sp.k0(2 * m * math.pi * rho / Lx) * cosx
        if not any_term:
            break
        m += 1
    return out / (math.pi * Lx)


def lgf2_series(x, y, z, Lx, Ly):
    """Eq. (lgf_2): neutral static 2D-periodic (x, y) series; needs
    sqrt(y^2 + z^2) > 0."""
    x, y, z = (np.asarray(v, dtype=float) for v in (x, y, z))
    az = np.abs(z)
    out = -az / (2 * Lx * Ly)
    out -= _log_layer(2 * math.pi * az / Ly, 2 * math.pi * y / Ly) / (4 * math.pi * Lx)
    out += _k0_lattice_sum(x, y, z, Lx, Ly, 1.0, [0])
    return out


def lgf3_series(x, y, z, Lx, Ly, Lz, zero_mean=True):
    """Eq. (lgf_3): neutral static 3D-periodic series (|z| <= Lz); needs
    sqrt(y^2 + z^2) > 0.  With zero_mean the constant Lz/(12 Lx Ly) is added
    so that the cell mean of G vanishes."""
    x, y, z = (np.asarray(v, dtype=float) for v in (x, y, z))
    out = (z * z - np.abs(z) * Lz) / (2 * Lx * Ly * Lz)
    kmax = int(math.ceil(K0_CUTOFF * Ly / (2 * math.pi * Lz))) + 2
    for k in range(-kmax, kmax + 1):
        a = 2 * math.pi * np.abs(k * Lz + z) / Ly
        out -= _log_layer(a, 2 * math.pi * y / Ly) / (4 * math.pi * Lx)
    out += _k0_lattice_sum(x, y, z, Lx, Ly, Lz, range(-kmax, kmax + 1))
    if zero_mean:
        out += Lz / (12 * Lx * Ly)
    return out


def lgf1_realspace(x, y, z, Lx, P=4000):
    """Neutral static 1D kernel from Gradshteyn & Ryzhik 8.526.1, valid at
    rho = 0, in the gauge of Eq. (lgf_1):
      G = (gamma - ln 2L)/(2 pi L) + 1/(4 pi r)
          + (1/4 pi) sum_{l>=1} [1/|r - l L x| + 1/|r + l L x| - 2/(l L)],
    with the l > P tail summed from its large-l expansion."""
    x, y, z = (np.asarray(v, dtype=float) for v in (x, y, z))
    r2t = y * y + z * z
    r = np.sqrt(x * x + r2t)
    out = (EULER_GAMMA - math.log(2 * Lx)) / (2 * math.pi * Lx) + 1.0 / (FOUR_PI * r)
    acc = np.zeros(x.size)
    for l in range(P, 0, -1):        # small terms first
        lL = l * Lx
        acc += (1.0 / np.sqrt((x - lL) ** 2 + r2t) + 1.0 / np.sqrt((x + lL) ** 2 + r2t)
                - 2.0 / lL)
    tail = (3 * x * x - (x * x + r2t)) / Lx ** 3 * float(sp.zeta(3, P + 1))
    return out + (acc + tail) / FOUR_PI


# ----------------------------------------------------------------------------
# Ewald splittings (fallback where the paper's series converge slowly)
# ----------------------------------------------------------------------------

def _ewald_S(d, k0, E):
    """Real-space Ewald kernel
    [e^{-j k0 d} erfc(dE - j k0/2E) + e^{j k0 d} erfc(dE + j k0/2E)]/(8 pi d),
    written with erfcx to avoid overflow."""
    k0 = complex(k0)
    a = k0 / (2 * E)
    pref = np.exp(-(d * E) ** 2 + a * a)
    return pref * (sp.erfcx(d * E - 1j * a) + sp.erfcx(d * E + 1j * a)) / (8 * math.pi * d)


def _ewald_S_self(k0, E):
    """lim_{d->0} [S(d) - e^{-j k0 d}/(4 pi d)]."""
    k0 = complex(k0)
    a = k0 / (2 * E)
    return (2j * k0 * sp.erfc(1j * a) - 4 * E / math.sqrt(math.pi) * np.exp(a * a)) / (8 * math.pi)


def _lattice_vectors(dims, L, rmax):
    rng = [np.arange(-int(math.ceil(rmax / L[c])) - 1, int(math.ceil(rmax / L[c])) + 2)
           if c < dims else np.array([0]) for c in range(3)]
    I = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    R = I * L
    keep = np.sqrt(np.sum(R * R, axis=1)) <= rmax
    return I[keep], R[keep]


def _spatial_part(r, lat, E, self_term):
    k0 = lat.k0
    reach = math.sqrt(42.0 + max(0.0, (k0 * k0).real) / (4 * E * E)) / E
    rmax = reach + float(np.sqrt(np.sum(r * r, axis=1)).max())
    I, R = _lattice_vectors(lat.dims, lat.L, rmax)
    phase = np.exp(-1j * (R @ lat.kt))
    out = np.zeros(r.shape[0], dtype=complex)
    for Rv, ph, iv in zip(R, phase, I):
        d = np.sqrt(np.sum((r - Rv) ** 2, axis=1))
        if self_term and not np.any(iv):
            # only used for r == 0: regularized limit of the R = 0 term
            out += ph * _ewald_S_self(k0, E)
        else:
            out += ph * _ewald_S(d, k0, E)
    return out


def ewald3(r, lat, E=None, self_term=False):
    """3D-periodic Ewald splitting (static or Helmholtz, any phase).

    Spatial part: sum_R phi_R S(|r - R|).  Spectral part:
    (1/V) sum_G e^{-j kG.r} e^{-(kG.kG - k0^2)/(4E^2)} / (kG.kG - k0^2),
    kG = k_t + 2 pi (m/Lx, n/Ly, p/Lz).  For the NPSP case the G = 0 term is
    dropped and -1/(4 E^2 V) added (zero cell mean).  With self_term the
    singular R = 0 spatial term is replaced by lim [S - G0] (r must be 0)."""
    r = np.atleast_2d(np.asarray(r, dtype=float))
    L = lat.L
    V = L[0] * L[1] * L[2]
    k0 = lat.k0
    if E is None:
        E = max(math.sqrt(math.pi) / V ** (1.0 / 3.0), abs(k0) / 6.0)
    out = _spatial_part(r, lat, E, self_term)
    kmax = 2 * E * math.sqrt(42.0 + max(0.0, (k0 * k0).real) / (4 * E * E)) + float(np.abs(lat.kt).max())
    rng = [np.arange(-int(math.ceil(kmax * L[c] / (2 * math.pi))) - 1,
                     int(math.ceil(kmax * L[c] / (2 * math.pi))) + 2) for c in range(3)]
    M = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    kG = lat.kt[None, :] + 2 * math.pi * M / L[None, :]
    kk = np.sum(kG * kG, axis=1)
    keep = np.abs(np.sqrt(kk)) <= kmax
    if lat.npsp:
        keep &= np.any(M != 0, axis=1)
    kG, kk = kG[keep], kk[keep]
    den = kk - k0 * k0
    coef = np.exp(-den / (4 * E * E)) / den / V
    for j in range(0, kG.shape[0], 256):
        out += np.exp(-1j * (r @ kG[j:j + 256].T)) @ coef[j:j + 256]
    if lat.npsp:
        out += -1.0 / (4 * E * E * V)
    return out


def ewald2(r, lat, E=None, self_term=False):
    """2D-periodic (x, y) Ewald splitting (static or Helmholtz, any phase).

    Spectral part: (1/(4jA)) sum_mn e^{-j(kxm x + kyn y)}/kz
      [e^{j kz|z|} erfc(j kz/2E + |z|E) + e^{-j kz|z|} erfc(j kz/2E - |z|E)],
    which tends to Eq. (pgf_2) as E -> infinity.  For the NPSP case the (0,0)
    term becomes -(1/2A)[|z| erf(|z|E) + e^{-z^2 E^2}/(sqrt(pi) E)] (its
    divergent constant cancels for neutral sources), in the gauge of Eq. (lgf_2)."""
    r = np.atleast_2d(np.asarray(r, dtype=float))
    Lx, Ly = lat.L[0], lat.L[1]
    A = Lx * Ly
    k0 = lat.k0
    if E is None:
        E = max(math.sqrt(math.pi / A), abs(k0) / 6.0)
    out = _spatial_part(r, lat, E, self_term)
    x, y, az = r[:, 0], r[:, 1], np.abs(r[:, 2])
    kmax = 2 * E * math.sqrt(42.0 + max(0.0, (k0 * k0).real) / (4 * E * E)) + float(np.abs(lat.kt).max())
    mmax = int(math.ceil(kmax * Lx / (2 * math.pi))) + 1
    nmax = int(math.ceil(kmax * Ly / (2 * math.pi))) + 1
    for m in range(-mmax, mmax + 1):
        for n in range(-nmax, nmax + 1):
            kx = lat.kt[0] + 2 * math.pi * m / Lx
            ky = lat.kt[1] + 2 * math.pi * n / Ly
            if abs(np.sqrt(kx * kx + ky * ky)) > kmax:
                continue
            lateral = np.exp(-1j * (kx * x + ky * y))
            if lat.npsp and m == 0 and n == 0:
                out += -(az * sp.erf(az * E) + np.exp(-(az * E) ** 2) / (math.sqrt(math.pi) * E)) / (2 * A)
                continue
            kz = csqrt_im_nonpos(k0 * k0 - kx * kx - ky * ky)
            a = 1j * kz / (2 * E) + az * E
            b = 1j * kz / (2 * E) - az * E
            pref = np.exp(kz * kz / (4 * E * E) - (az * E) ** 2)
            out += lateral * pref * (sp.erfcx(a) + sp.erfcx(b)) / (4j * A * kz)
    return out


def _expint1(z):
    """E1(z) on the principal branch; on the negative real axis the value
    reached from above (the limit of a lossy k0 with Im k0 -> 0-)."""
    z = complex(z)
    if z.imag == 0.0 and z.real < 0.0:
        return -float(sp.expi(-z.real)) - 1j * math.pi
    return complex(sp.exp1(z))


def ewald1(r, lat, E=None, self_term=False):
    """1D-periodic (x) Ewald splitting (static with a phase shift, or
    Helmholtz, any phase; not the neutral static case).

    Spatial part: sum_R phi_R S(|r - R|) as in 3D.  Spectral part
      (1/(4 pi Lx)) sum_m e^{-j kxm x} sum_{q>=0} ((-1)^q/q!) (rho E)^{2q} E_{q+1}(-krho_m^2/(4 E^2)),
    krho_m^2 = k0^2 - kxm^2, with E_{q+1} on the principal branch (the branch
    that matches Im krho_m <= 0) and E_{q+1}(z) = (e^{-z} - z E_q(z))/q.
    Valid at any rho, including rho = 0 (x not a lattice point)."""
    if lat.npsp:
        raise ValueError("the neutral static 1D case has no E1 spectral form (divergent m = 0 term)")
    r = np.atleast_2d(np.asarray(r, dtype=float))
    Lx = lat.L[0]
    k0 = lat.k0
    if E is None:
        E = max(math.sqrt(math.pi) / Lx, abs(k0) / 6.0)
    out = _spatial_part(r, lat, E, self_term)
    x = r[:, 0]
    t2 = (r[:, 1] ** 2 + r[:, 2] ** 2) * E * E
    kmax = 2 * E * math.sqrt(42.0 + max(0.0, (k0 * k0).real) / (4 * E * E)) + abs(lat.kt[0])
    mmax = int(math.ceil(kmax * Lx / (2 * math.pi))) + 1
    qmax = 0
    coef = 1.0
    tmax = float(t2.max()) if t2.size else 0.0
    while coef > 1e-19 and qmax < 200:
        qmax += 1
        coef *= tmax / qmax
    for m in range(-mmax, mmax + 1):
        kx = lat.kt[0] + 2 * math.pi * m / Lx
        z = -(k0 * k0 - kx * kx) / (4 * E * E)
        En = _expint1(z)
        ez = np.exp(-z)
        acc = np.full(x.size, En, dtype=complex)
        c = np.ones(x.size)
        for q in range(1, qmax + 1):
            En = (ez - z * En) / q
            c = c * (-t2) / q
            acc += c * En
        out += np.exp(-1j * kx * x) * acc / (4 * math.pi * Lx)
    return out


# ----------------------------------------------------------------------------
# dispatcher
# ----------------------------------------------------------------------------

def _pgf_reduced(r, lat, method):
    """G^p at points r already reduced into the cell (no Bloch factor)."""
    P = r.shape[0]
    out = np.empty(P, dtype=complex)
    L = lat.L
    d = lat.dims
    if d == 3:
        if lat.npsp:
            xrole = np.argmin(np.abs(r), axis=1)
            perm = np.stack([xrole, (xrole + 1) % 3, (xrole + 2) % 3], axis=1)
            rp = np.take_along_axis(r, perm, axis=1)
            rho = np.hypot(rp[:, 1], rp[:, 2])
            use_series = rho >= SERIES_MIN_FRACTION["npsp"] * L.min()
        else:
            zrole = np.argmax(np.abs(r), axis=1)
            perm = np.stack([(zrole + 1) % 3, (zrole + 2) % 3, zrole], axis=1)
            rp = np.take_along_axis(r, perm, axis=1)
            use_series = np.abs(rp[:, 2]) >= SERIES_MIN_FRACTION["dyn"] * L.min()
    elif d == 2:
        if lat.npsp:
            swap = np.abs(r[:, 1]) < np.abs(r[:, 0])
            perm = np.where(swap[:, None], np.array([1, 0, 2]), np.array([0, 1, 2]))
            rp = np.take_along_axis(r, perm, axis=1)
            rho = np.hypot(rp[:, 1], rp[:, 2])
            use_series = rho >= SERIES_MIN_FRACTION["npsp"] * L[:2].min()
        else:
            perm = np.tile(np.array([0, 1, 2]), (P, 1))
            rp = r
            use_series = np.abs(r[:, 2]) >= SERIES_MIN_FRACTION["dyn"] * L[:2].min()
    else:
        perm = np.tile(np.array([0, 1, 2]), (P, 1))
        rp = r
        rho = np.hypot(r[:, 1], r[:, 2])
        use_series = rho >= SERIES_MIN_FRACTION["npsp" if lat.npsp else "dyn"] * L[0]
    if method == "series":
        use_series = np.ones(P, dtype=bool)
    elif method == "ewald":
        use_series = np.zeros(P, dtype=bool)

    # series, grouped by axis permutation
    idx_s = np.nonzero(use_series)[0]
    if idx_s.size:
        keys = perm[idx_s, 0] * 9 + perm[idx_s, 1] * 3 + perm[idx_s, 2]
        for key in np.unique(keys):
            sel = idx_s[keys == key]
            p = perm[sel[0]]
            Lp = L[p]
            x, y, z = rp[sel, 0], rp[sel, 1], rp[sel, 2]
            if d == 3 and lat.npsp:
                out[sel] = lgf3_series(x, y, z, Lp[0], Lp[1], Lp[2])
            elif d == 3:
                out[sel] = pgf3_series(x, y, z, Lp, lat.k0, lat.kt[p])
            elif d == 2 and lat.npsp:
                out[sel] = lgf2_series(x, y, z, Lp[0], Lp[1])
            elif d == 2:
                out[sel] = pgf2_series(x, y, z, L[0], L[1], lat.k0, lat.kt[0], lat.kt[1])
            elif lat.npsp:
                out[sel] = lgf1_series(x, np.hypot(y, z), L[0])
            else:
                out[sel] = pgf1_series(x, np.hypot(y, z), L[0], lat.k0, lat.kt[0])
    idx_e = np.nonzero(~use_series)[0]
    if idx_e.size:
        re = r[idx_e]
        if d == 3:
            out[idx_e] = ewald3(re, lat)
        elif d == 2:
            out[idx_e] = ewald2(re, lat)
        elif lat.npsp:
            out[idx_e] = lgf1_realspace(re[:, 0], re[:, 1], re[:, 2], L[0])
        else:
            out[idx_e] = ewald1(re, lat)
    return out


def pgf(r, lat, method="auto", chunk=4096):
    """G^p(r) of Eq. (2) at an array of displacement vectors r (shape (..., 3)).

    method: "auto" (paper's series where they converge quickly, Ewald
    otherwise), "series" or "ewald" (forced, for cross-checks).
    Displacements equal to a lattice vector are singular and not allowed;
    use pgf_self for the regularized coincident limit.
    """
    r = np.asarray(r, dtype=float)
    shape = r.shape[:-1]
    rr = r.reshape(-1, 3)
    red, phase = reduce_to_cell(rr, lat)
    out = np.empty(rr.shape[0], dtype=complex)
    for s in range(0, rr.shape[0], chunk):
        out[s:s + chunk] = _pgf_reduced(red[s:s + chunk], lat, method)
    out *= phase
    return out.reshape(shape)


def pgf_self(lat):
    """lim_{r->0} [G^p(r) - G0(r)]: the images of a source seen at its own
    position, i.e. the n = m term of Eq. (1) with the singular i = 0 image
    removed."""
    z = np.zeros((1, 3))
    if lat.dims == 3:
        return complex(ewald3(z, lat, self_term=True)[0])
    if lat.dims == 2:
        return complex(ewald2(z, lat, self_term=True)[0])
    if lat.npsp:
        return (EULER_GAMMA - math.log(2 * lat.L[0])) / (2 * math.pi * lat.L[0])
    return complex(ewald1(z, lat, self_term=True)[0])


def g_near(r, lat, i_d):
    """Near-zone kernel of Eq. (4): Eq. (2) truncated to |i_c| <= i_d."""
    r = np.asarray(r, dtype=float)
    out = np.zeros(r.shape[:-1], dtype=complex)
    rng = [range(-i_d, i_d + 1) if c < lat.dims else range(0, 1) for c in range(3)]
    for ix in rng[0]:
        for iy in rng[1]:
            for iz in rng[2]:
                R = np.array([ix, iy, iz]) * lat.L
                out += np.exp(-1j * np.dot(lat.kt, R)) * g0(r - R, lat.k0)
    return out


def g_far(r, lat, i_d, method="auto"):
    """Far-zone kernel of Eq. (4): G^p - G^p_near."""
    return pgf(r, lat, method) - g_near(r, lat, i_d)
