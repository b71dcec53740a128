"""Position gradients (forces) of the periodic potential, in FP64 on the CPU.

Test infrastructure: only the test suite and the benchmark's CPU-baseline leg
use this module.

For amplitudes q, an upstream gradient g = dL/du (L real; for complex u the
convention dL = Re sum_m conj(g_m) du_m) and points that are both sources and
observers (Sec. 2), the gradient of L with respect to the position r_k is

    dL/dr_k = Re( conj(g_k) sum_n d/dr_k A[k, n] q_n )        (k as observer)
            + Re( sum_m conj(g_m) d/dr_k A[m, k] q_k )        (k as source),

summed over right-hand sides.  Two operators A are differentiated:

  * the exact one of Eq. (1), A[m, n] = G^p(r_m - r_n) (the n = m coefficient
    lim_{r->0}[G^p - G0] does not depend on the position): psp_grad;
  * the discrete FFT-PIM operator of Sec. 3 as oracle.steps builds it, whose
    entries depend on the positions through the Lagrange weights of the
    projections and interpolations (Eq. (projection), Eq. (interpolation))
    and through the correction entries of Eq. (er): steps_grad.
"""
import math

import numpy as np

from . import pgf as _pgf
from . import steps as _steps

FOUR_PI = 4.0 * math.pi


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def grad_g0(d, k0):
    """Gradient of G0(r) = exp(-j k0 |r|)/(4 pi |r|) at r = d (..., 3):
    (d / |d|) (-j k0 - 1/|d|) G0(|d|)."""
    d = np.asarray(d, dtype=float)
    R = np.sqrt(np.sum(d * d, axis=-1))
    g0 = np.exp(-1j * complex(k0) * R) / (FOUR_PI * R)
    f = (-1j * complex(k0) - 1.0 / R) * g0 / R
    return d * f[..., None]


def lagrange_stencil_deriv(x, origin, h, q, n):
    """Like oracle.steps.lagrange_stencil, also returning dw/dx: the
    derivative of each degree-q Lagrange basis value by the product rule,
    d l_k/du = sum_{j != k} (1/(k - j)) prod_{i != k, j} (u - i)/(k - i),
    divided by the spacing h (u = (x - origin)/h - s)."""
    s, w = _steps.lagrange_stencil(x, origin, h, q, n)
    t = (np.asarray(x, dtype=float) - origin) / h
    u = t - s
    dw = np.zeros_like(w)
    for k in range(q + 1):
        for j in range(q + 1):
            if j == k:
                continue
            term = np.full(u.shape, 1.0 / (k - j))
            for i in range(q + 1):
                if i != k and i != j:
                    term = term * (u - i) / (k - i)
            dw[:, k] += term
    return s, w, dw / h


class _DStencils:
    """Per-axis stencil starts, weights and weight derivatives."""

    def __init__(self, pts, origin, h, q, n):
        self.s = np.empty((pts.shape[0], 3), dtype=np.int64)
        self.w, self.dw = [], []
        for c in range(3):
            s, w, dw = lagrange_stencil_deriv(pts[:, c], origin[c], h[c], q, n[c])
            self.s[:, c] = s
            self.w.append(w)
            self.dw.append(dw)
        self.q = q
        self.n = n

    def lin(self, rows):
        k = np.arange(self.q + 1)
        ix = self.s[rows, 0][:, None] + k
        iy = self.s[rows, 1][:, None] + k
        iz = self.s[rows, 2][:, None] + k
        lin = (ix[:, :, None, None] * self.n[1] + iy[:, None, :, None]) * self.n[2] + iz[:, None, None, :]
        return lin.reshape(len(rows), -1)

    def tensor(self, rows, axis=None):
        """Tensor weights (P, (q+1)^3); with axis = c the factor of axis c is
        differentiated (the c-component of the weight gradient)."""
        f = [self.dw[c][rows] if c == axis else self.w[c][rows] for c in range(3)]
        return (f[0][:, :, None, None] * f[1][:, None, :, None] * f[2][:, None, None, :]).reshape(len(rows), -1)


def _grad_interp(st, grid_vals, rows):
    """d/dr_m of sum_g w_g(r_m) U[g] for each row: (nrhs, rows, 3)."""
    lin = st.lin(rows)
    out = np.zeros((grid_vals.shape[0], len(rows), 3), dtype=complex)
    for c in range(3):
        out[:, :, c] = np.einsum("pk,rpk->rp", st.tensor(rows, c), grid_vals[:, lin])
    return out


# ----------------------------------------------------------------------------
# the discrete operator of Sec. 3
# ----------------------------------------------------------------------------

def steps_grad(m, q, g, rows=None):
    """dL/dr_k (rows k, shape (len(rows), 3)) for the discrete operator of an
    oracle.steps.FFTPIM instance m (coinciding sources and observers), with
    L = Re sum_r g_r^H (A q_r), q and g of shape (nrhs, N) or (N,)."""
    if not m.coincide:
        raise ValueError("position gradients need coinciding sources and observers")
    qv = np.atleast_2d(np.asarray(q)).astype(complex)
    gv = np.atleast_2d(np.asarray(g)).astype(complex)
    N = m.src.shape[0]
    rows = np.arange(N) if rows is None else np.asarray(rows)
    out = np.zeros((len(rows), 3))

    # near grid (Sec. 3.3 Steps 1-3): interpolation weights differentiated on
    # the observer side (forward field of q) and on the source side (adjoint
    # field of g, the projection weights being the same)
    nst = _DStencils(m.src, m.origin, m.h, m.prm.near_q, m.prm.near_n)
    Vq = m._near_conv(_steps._spread(m.st_src, qv, m.Ng))
    Vg = m._near_conv(_steps._spread(m.st_obs, gv, m.Ng), adjoint=True)
    out += np.real(np.sum(np.conj(gv[:, rows])[..., None] * _grad_interp(nst, Vq, rows), axis=0))
    out += np.real(np.sum(np.conj(qv[:, rows])[..., None] * _grad_interp(nst, Vg, rows), axis=0))

    # far zone (Sec. 3.2): observer-grid weights on the forward grid sum,
    # source-grid weights on the conjugate-transposed one
    fo = _DStencils(m.obs, m.origin_fo, m.Df, m.prm.far_q, m.prm.far_n)
    fs = _DStencils(m.src, m.origin_fs, m.Df, m.prm.far_q, m.prm.far_n)
    Uq = m._far_grid_sum(_steps._spread(m.fst_src, qv, m.Ngf))
    Ug = m._far_grid_sum(_steps._spread(m.fst_obs, gv, m.Ngf), adjoint=True)
    out += np.real(np.sum(np.conj(gv[:, rows])[..., None] * _grad_interp(fo, Uq, rows), axis=0))
    out += np.real(np.sum(np.conj(qv[:, rows])[..., None] * _grad_interp(fs, Ug, rows), axis=0))

    # correction (Eq. (er)): d/dr of every entry C[k, n] (k observer) and
    # C[m, k] (k source), written out from the entry's definition
    for c in range(3):
        Dobs = correction_deriv(m, nst, rows, np.arange(N), c, side="obs")    # d C[k, n] / d r_k,c
        Dsrc = correction_deriv(m, nst, np.arange(N), rows, c, side="src")    # d C[m, k] / d r_k,c
        obs = np.einsum("kn,rn->rk", Dobs, qv)
        src = np.einsum("mk,rm->rk", Dsrc, np.conj(gv))
        out[:, c] += np.real(np.sum(np.conj(gv[:, rows]) * obs + src * qv[:, rows], axis=0))
    return out


def correction_deriv(m, dst, obs_rows, src_cols, c, side):
    """Derivative along axis c of the correction block C[obs_rows, src_cols]
    of Eq. (er), with respect to the observer position (side="obs") or the
    source position (side="src").  For each close triple (m, n, i):
        phi_i [ d/dr G0(r_m - r_n - R_i) - sum_a sum_b d/dr (w_a(r_m) w_b(r_n)) G0tab(a - b - i n_int) ],
    the G0 term dropped for the singular self pair (n = m, i = 0)."""
    lat = m.lat
    q = m.prm.near_q
    obs_rows = np.asarray(obs_rows)
    src_cols = np.asarray(src_cols)
    D = np.zeros((len(obs_rows), len(src_cols)), dtype=complex)
    k = np.arange(q + 1)
    ka = np.stack(np.meshgrid(k, k, k, indexing="ij"), axis=-1).reshape(-1, 3)
    kdiff = ka[:, None, :] - ka[None, :, :]
    so = m.st_obs.s[obs_rows]
    ss = m.st_src.s[src_cols]
    for img, ph in zip(m.images, m.img_phase):
        delta = so[:, None, :] - ss[None, :, :] - img * m.n_int
        jj, nn = np.nonzero(m._close(delta))
        if jj.size == 0:
            continue
        mm = obs_rows[jj]
        n = src_cols[nn]
        rv = m.obs[mm] - m.src[n] - img * lat.L
        with np.errstate(divide="ignore", invalid="ignore"):
            ex = grad_g0(rv, lat.k0)[:, c]
        if not np.any(img):
            ex = np.where(mm == n, 0.0, ex)
        if side == "src":
            ex = -ex
        dl = delta[jj, nn]
        keys, inv = np.unique(dl, axis=0, return_inverse=True)
        inv = inv.ravel()
        gg = np.empty(jj.size, dtype=complex)
        for kk in range(len(keys)):
            sel = np.nonzero(inv == kk)[0]
            M = m._g0_nodes(keys[kk][None, None, :] + kdiff)
            wm = dst.tensor(mm[sel], c if side == "obs" else None)
            wn = dst.tensor(n[sel], c if side == "src" else None)
            gg[sel] = np.sum((wm @ M) * wn, axis=1)
        np.add.at(D, (jj, nn), ph * (ex - gg))
    return D


# ----------------------------------------------------------------------------
# the exact sum of Eq. (1)
# ----------------------------------------------------------------------------

def grad_pgf(r, lat, i_d=1, h=None):
    """Gradient of G^p at displacements r (P, 3): the near images of Eq. (4)
    analytically, sum_{|i_c| <= i_d} phi_i grad G0(r - R_i), plus the smooth
    far part G^p - G^p_near by fourth-order central differences
    (f(-2h) - 8 f(-h) + 8 f(h) - f(2h)) / (12 h), whose nearest singularity is
    at least one period away."""
    r = np.atleast_2d(np.asarray(r, dtype=float))
    if h is None:
        h = 2e-3 * float(np.min(lat.L[:lat.dims]))
    out = np.zeros(r.shape, dtype=complex)
    rngs = [range(-i_d, i_d + 1) if c < lat.dims else range(0, 1) for c in range(3)]
    for ix in rngs[0]:
        for iy in rngs[1]:
            for iz in rngs[2]:
                R = np.array([ix, iy, iz]) * lat.L
                out += np.exp(-1j * np.dot(lat.kt, R)) * grad_g0(r - R, lat.k0)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        f = [_pgf.g_far(r + s * e, lat, i_d) for s in (-2, -1, 1, 2)]
        out[:, c] += (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
    return out


def psp_grad(lat, src, q, g, rows):
    """dL/dr_k at rows k for the exact operator of Eq. (1) (L as in the module
    docstring).  Direct sums over all points: O(N) per row."""
    src = np.asarray(src, dtype=float)
    qv = np.atleast_2d(np.asarray(q)).astype(complex)
    gv = np.atleast_2d(np.asarray(g)).astype(complex)
    N = src.shape[0]
    out = np.zeros((len(rows), 3))
    for t, k in enumerate(np.asarray(rows)):
        others = np.delete(np.arange(N), k)
        G = grad_pgf(src[k][None, :] - src[others], lat)          # grad G^p(r_k - r_n)
        obs = np.einsum("nc,rn->rc", G, qv[:, others])
        # d/dr_k G^p(r_m - r_k) = -grad G^p(r_m - r_k); G^p(r_m - r_k) is grad at -(r_k - r_m)
        Gm = grad_pgf(src[others] - src[k][None, :], lat)
        src_part = -np.einsum("mc,rm->rc", Gm, np.conj(gv[:, others]))
        out[t] = np.real(np.sum(np.conj(gv[:, k])[:, None] * obs + src_part * qv[:, k][:, None], axis=0))
    return out
