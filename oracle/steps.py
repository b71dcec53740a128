"""The FFT-PIM algorithm of Sec. 3, step by step, in FP64 on the CPU.

Test infrastructure: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module.  It is written from the paper's text and
shares nothing with the GPU library; it pins the GPU kernels to rounding
level, independently of the method's own approximation error (which the
direct pair sum in `psp` measures).

Order of operations (Sec. 3):
  far zone (Sec. 3.2): Step 1 projection onto the source grid, Eq. (projection);
      Step 2 grid sum with G^p_far, Eq. (8); Step 3 interpolation from the
      observer grid, Eq. (interpolation).
  near zone (Sec. 3.3): Step 1 projection onto the single near grid; Step 2
      zero-padded FFT convolution with tabulated G^p_near; Step 3
      interpolation; Step 4 error correction, Eq. (er), with only the close
      images kept (end of Sec. 3.3).
  u = u_near + u_far, Eq. (5).

Readings where the text is silent or garbled (each is also what the GPU
library implements):
  grids      Every grid carries a stencil halo.  A grid of n nodes with
             Lagrange order q on the domain [lo, hi] has n_int cells of width
             h = (hi - lo)/n_int, with n_int = n - q on periodic axes of the
             near grid and n_int = n - q - 1 otherwise, and node l at
             o + l h with o = lo - h (q-1)/2.  Eq. (gridc)'s linear index is
             read 0-based, x slowest.
  stencils   "q-th order" Lagrange = degree q, q+1 nodes per axis.  A point
             at x uses nodes s..s+q with s = floor((x - o)/h - (q-1)/2),
             clamped to [0, n-1-q]; its near-grid box is s.
  far grids  The observer grid is the source grid shifted by -Delta/2 (the
             paper shifts by +Delta/2; only the separation matters) so that
             both fit the same node count.
  near table G^p_near (Eq. (4)) sampled at node offsets, e h - R_i, with
             every term whose argument vanishes set to 0; the image shift on
             the near grid is exactly n_int nodes (L = n_int h).  "Doubling
             its size" means zero padding to 2n on every axis.
  correction The triple (observer m, source n, image i) is corrected when
             its box offset d = s_m - s_n - i n_int (in boxes) is close: the
             Chebyshev distance max_c |d_c| <= r_c (the cube), or, for the
             ball |r - r_m| <= D^ER of Eq. (er) with D^ER = corr_ball h_max,
             when sum_c (d_c h_c / h_max)^2 <= corr_ball^2 (a relative slack
             of 1e-9 settles offsets on the sphere).  Its entry is
             phi_i [G0(r_m - r_n - R_i) - G_grid,i(m, n)], the G0 term being
             dropped for the singular self pair (n = m, i = 0).  The weights in
             Eq. (er_2) are those of near Steps 1 and 3.
  self term  Default: the images of a source act on itself (the far zone and
             the near-image grid include them); self_mode="exclude" subtracts
             lim_{r->0}[G^p - G0] q_m as well (Eq. (5) literally).
"""
import itertools
import math

import numpy as np

from . import pgf as _pgf


class Params:
    """Method parameters: near grid nodes and order, correction radius (in
    boxes), far grid nodes and order, near image range i_d (Eq. (4)), and the
    correction region: the cube of Chebyshev box distance <= r_c
    (corr_ball = 0) or the ball of Eq. (er) over box offsets, of radius
    corr_ball h_max (corr_ball > 0; r_c is then unused)."""

    def __init__(self, near_n, near_q, r_c, far_n, far_q, i_d=1, corr_ball=0.0):
        self.near_n = np.broadcast_to(np.asarray(near_n, dtype=int), (3,)).copy()
        self.near_q = int(near_q)
        self.r_c = int(r_c)
        self.far_n = np.broadcast_to(np.asarray(far_n, dtype=int), (3,)).copy()
        self.far_q = int(far_q)
        self.i_d = int(i_d)
        self.corr_ball = float(corr_ball)


def domain_bounds(lat, pts):
    """Target region D (Sec. 3.2): the cell [0, L) on periodic axes, the
    bounding box of the points on the others (a zero extent is widened to
    [lo, lo + 1], the reading for a flat or single-point set)."""
    lo = pts.min(axis=0).astype(float)
    hi = pts.max(axis=0).astype(float)
    for c in range(3):
        if c < lat.dims:
            lo[c], hi[c] = 0.0, lat.L[c]
        elif not hi[c] > lo[c]:
            hi[c] = lo[c] + 1.0
    return lo, hi


def lagrange_stencil(x, origin, h, q, n):
    """Degree-q Lagrange weights of the nodes s..s+q for points x on the
    grid origin + l h (l = 0..n-1).  Returns (s, w) with w of shape (P, q+1)."""
    t = (np.asarray(x, dtype=float) - origin) / h
    s = np.floor(t - 0.5 * (q - 1)).astype(np.int64)
    s = np.clip(s, 0, n - 1 - q)
    u = t - s
    w = np.ones((t.size, q + 1))
    for k in range(q + 1):
        for j in range(q + 1):
            if j != k:
                w[:, k] *= (u - j) / (k - j)
    return s, w


class _Stencils:
    """Per-axis stencil starts and 1D weights of a point set on one grid."""

    def __init__(self, pts, origin, h, q, n):
        self.s = np.empty((pts.shape[0], 3), dtype=np.int64)
        self.w = []
        for c in range(3):
            s, w = lagrange_stencil(pts[:, c], origin[c], h[c], q, n[c])
            self.s[:, c] = s
            self.w.append(w)
        self.q = q
        self.n = n

    def taps(self, rows=None):
        """Linear node indices (x slowest) and tensor weights, (P, (q+1)^3)."""
        rows = np.arange(self.s.shape[0]) if rows is None else rows
        k = np.arange(self.q + 1)
        ix = self.s[rows, 0][:, None] + k
        iy = self.s[rows, 1][:, None] + k
        iz = self.s[rows, 2][:, None] + k
        lin = (ix[:, :, None, None] * self.n[1] + iy[:, None, :, None]) * self.n[2] + iz[:, None, None, :]
        w = (self.w[0][rows][:, :, None, None] * self.w[1][rows][:, None, :, None]
             * self.w[2][rows][:, None, None, :])
        P = len(rows)
        return lin.reshape(P, -1), w.reshape(P, -1)


def _spread(st, q_vals, ngrid):
    """Projection (Eq. (projection)): Q[g] = sum_n w_g(r_n) q_n; q_vals (nrhs, N)."""
    lin, w = st.taps()
    out = np.zeros((q_vals.shape[0], ngrid), dtype=complex)
    for r in range(q_vals.shape[0]):
        np.add.at(out[r], lin.ravel(), (w * q_vals[r][:, None]).ravel())
    return out


def _interp(st, grid_vals, rows):
    """Interpolation (Eq. (interpolation)): u_m = sum_g w_g(r_m) U[g]."""
    lin, w = st.taps(rows)
    return np.einsum("pk,rpk->rp", w, grid_vals[:, lin])


class FFTPIM:
    """The discrete FFT-PIM operator of Sec. 3 for one geometry.

    lat: oracle.pgf.Lattice; prm: Params; src: (N, 3); obs: (M, 3) or None
    (observers coincide with sources); lo, hi: target region (default
    domain_bounds over sources and observers).
    """

    def __init__(self, lat, prm, src, obs=None, lo=None, hi=None, self_mode="images",
                 far_method="auto"):
        self.lat, self.prm = lat, prm
        self.src = np.asarray(src, dtype=float)
        self.coincide = obs is None
        self.obs = self.src if obs is None else np.asarray(obs, dtype=float)
        allpts = self.src if self.coincide else np.vstack([self.src, self.obs])
        dlo, dhi = domain_bounds(lat, allpts)
        self.lo = dlo if lo is None else np.asarray(lo, float)
        self.hi = dhi if hi is None else np.asarray(hi, float)
        self.self_mode = self_mode
        periodic = np.arange(3) < lat.dims
        self.periodic = periodic

        # ---- near grid (Sec. 3.3: single grid, N_g comparable to N) ----
        q = prm.near_q
        n = prm.near_n
        self.n_int = np.where(periodic, n - q, n - q - 1)
        if np.any(self.n_int < 1):
            raise ValueError("near grid too small for the order")
        self.h = (self.hi - self.lo) / self.n_int
        self.origin = self.lo - self.h * 0.5 * (q - 1)
        self.st_src = _Stencils(self.src, self.origin, self.h, q, n)
        self.st_obs = self.st_src if self.coincide else _Stencils(self.obs, self.origin, self.h, q, n)
        self.Ng = int(np.prod(n))

        # near-zone images (Eq. (4)) and their phases
        rngs = [range(-prm.i_d, prm.i_d + 1) if periodic[c] else range(0, 1) for c in range(3)]
        self.images = np.array(list(itertools.product(*rngs)), dtype=np.int64)
        self.img_phase = np.exp(-1j * (self.images * lat.L) @ lat.kt)

        # ---- near Step 2 table: G^p_near at node offsets, zero padded ----
        self._near_spectrum()

        # ---- far grids (Sec. 3.2, Eq. (grid)) ----
        qf, nf = prm.far_q, prm.far_n
        nf_int = nf - qf - 1
        if np.any(nf_int < 1):
            raise ValueError("far grid too small for the order")
        self.Df = (self.hi - self.lo) / nf_int
        self.origin_fs = self.lo - self.Df * 0.5 * (qf - 1)
        self.origin_fo = self.origin_fs - 0.5 * self.Df
        self.fst_src = _Stencils(self.src, self.origin_fs, self.Df, qf, nf)
        self.fst_obs = _Stencils(self.obs, self.origin_fo, self.Df, qf, nf)
        self.Ngf = int(np.prod(nf))
        # G^p_far at the offsets between observer and source grid nodes
        d = [np.arange(-(nf[c] - 1), nf[c]) for c in range(3)]
        D = np.stack(np.meshgrid(*d, indexing="ij"), axis=-1)
        rvec = (D - 0.5) * self.Df
        self.far_table = _pgf.g_far(rvec.reshape(-1, 3), lat, prm.i_d, far_method).reshape(D.shape[:3])
        self.self_value = _pgf.pgf_self(lat) if self.coincide else 0.0

    # ------------------------------------------------------------------
    def _g0_nodes(self, e):
        """G0 at integer node offsets e (..., 3); 0 where the offset vanishes."""
        r = e * self.h
        R = np.sqrt(np.sum(r * r, axis=-1))
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.exp(-1j * self.lat.k0 * R) / (_pgf.FOUR_PI * R)
        return np.where(R == 0, 0.0, g)

    def _near_spectrum(self):
        n = self.prm.near_n
        N2 = 2 * n
        e = [np.arange(-(n[c] - 1), n[c]) for c in range(3)]
        E = np.stack(np.meshgrid(*e, indexing="ij"), axis=-1)
        T = np.zeros(E.shape[:3], dtype=complex)
        for img, ph in zip(self.images, self.img_phase):
            T += ph * self._g0_nodes(E - img * self.n_int)
        self.near_table = T
        # circular embedding of offsets -(n-1)..(n-1) into length 2n
        Tc = np.zeros(tuple(N2), dtype=complex)
        idx = [np.mod(np.arange(-(n[c] - 1), n[c]), N2[c]) for c in range(3)]
        Tc[np.ix_(*idx)] = T
        self.near_hat = np.fft.fftn(Tc)

    def _near_conv(self, Q, adjoint=False):
        n = self.prm.near_n
        N2 = tuple(2 * n)
        out = np.empty_like(Q)
        kern = np.conj(self.near_hat) if adjoint else self.near_hat
        for r in range(Q.shape[0]):
            grid = Q[r].reshape(tuple(n))
            V = np.fft.ifftn(np.fft.fftn(grid, s=N2, axes=(0, 1, 2)) * kern)
            out[r] = V[:n[0], :n[1], :n[2]].ravel()
        return out

    def _far_matrix(self, rows=None):
        """Dense K[m', n'] = G^p_far(x^o_m' - x^s_n') of Eq. (8) (rows m' only
        when given)."""
        nf = self.prm.far_n
        idx = np.stack(np.meshgrid(*[np.arange(nf[c]) for c in range(3)], indexing="ij"),
                       axis=-1).reshape(-1, 3)
        ri = idx if rows is None else idx[rows]
        dif = ri[:, None, :] - idx[None, :, :] + (nf - 1)
        return self.far_table[dif[..., 0], dif[..., 1], dif[..., 2]]

    def _far_grid_sum(self, Q, adjoint=False, block=1024):
        """Eq. (8), u_g = K q_g, or its conjugate transpose K^H q_g, computed
        one block of output grid nodes at a time.  Q: (nrhs, Ngf)."""
        nf = self.prm.far_n
        idx = np.stack(np.meshgrid(*[np.arange(nf[c]) for c in range(3)], indexing="ij"),
                       axis=-1).reshape(-1, 3)
        out = np.empty_like(Q)
        for s0 in range(0, self.Ngf, block):
            r = np.arange(s0, min(s0 + block, self.Ngf))
            if adjoint:
                # (K^H)[r, :] = conj(K[:, r])^T, K[m', n'] = table[m' - n']
                dif = idx[None, :, :] - idx[r][:, None, :] + (nf - 1)
                Kh = np.conj(self.far_table[dif[..., 0], dif[..., 1], dif[..., 2]])
            else:
                Kh = self._far_matrix(r)
            out[:, r] = (Kh @ Q.T).T
        return out

    # ------------------------------------------------------------------
    def correction_block(self, obs_rows, src_cols):
        """Dense block C[obs_rows, src_cols] of the near-zone error correction,
        Eq. (er), restricted to the close image triples (end of Sec. 3.3).

        For each close triple (m, n, i) the entry gains
        phi_i [G0(r_m - r_n - R_i) - sum_a sum_b w_a(r_m) G0tab(a - b - i n_int) w_b(r_n)]
        where a, b run over the two stencils.  Triples with the same box offset
        share the (q+1)^3 x (q+1)^3 matrix G0tab(a - b - i n_int), so they are
        evaluated together."""
        lat = self.lat
        q = self.prm.near_q
        obs_rows = np.asarray(obs_rows)
        src_cols = np.asarray(src_cols)
        C = np.zeros((len(obs_rows), len(src_cols)), dtype=complex)
        k = np.arange(q + 1)
        ka = np.stack(np.meshgrid(k, k, k, indexing="ij"), axis=-1).reshape(-1, 3)
        kdiff = ka[:, None, :] - ka[None, :, :]
        so = self.st_obs.s[obs_rows]
        ss = self.st_src.s[src_cols]
        for img, ph in zip(self.images, self.img_phase):
            delta = so[:, None, :] - ss[None, :, :] - img * self.n_int
            jj, nn = np.nonzero(self._close(delta))
            if jj.size == 0:
                continue
            m = obs_rows[jj]
            n = src_cols[nn]
            # exact part phi_i G0(r_m - r_n - R_i); the singular self pair is dropped
            rv = self.obs[m] - self.src[n] - img * lat.L
            R = np.sqrt(np.sum(rv * rv, axis=1))
            with np.errstate(divide="ignore", invalid="ignore"):
                ex = np.exp(-1j * lat.k0 * R) / (_pgf.FOUR_PI * R)
            if self.coincide and not np.any(img):
                ex = np.where(m == n, 0.0, ex)
            # grid part, grouped by box offset
            dl = delta[jj, nn]
            keys, inv = np.unique(dl, axis=0, return_inverse=True)
            inv = inv.ravel()
            order = np.argsort(inv, kind="stable")
            bounds = np.searchsorted(inv[order], np.arange(len(keys) + 1))
            gg = np.empty(jj.size, dtype=complex)
            for kk in range(len(keys)):
                sel = order[bounds[kk]:bounds[kk + 1]]
                M = self._g0_nodes(keys[kk][None, None, :] + kdiff)
                wm = self._tensor_w(self.st_obs, m[sel])
                wn = self._tensor_w(self.st_src, n[sel])
                gg[sel] = np.sum((wm @ M) * wn, axis=1)
            np.add.at(C, (jj, nn), ph * (ex - gg))
        return C

    def _close(self, delta):
        """Close box offsets (last axis: x, y, z) of the correction region."""
        if self.prm.corr_ball <= 0:
            return np.max(np.abs(delta), axis=-1) <= self.prm.r_c
        wgt = self.h / self.h.max()
        s = np.sum((delta * wgt) ** 2, axis=-1)
        return s <= self.prm.corr_ball ** 2 * (1.0 + 1e-9)

    @staticmethod
    def _tensor_w(st, idx):
        return (st.w[0][idx][:, :, None, None] * st.w[1][idx][:, None, :, None]
                * st.w[2][idx][:, None, None, :]).reshape(len(idx), -1)

    def correction_rows(self, rows):
        return self.correction_block(rows, np.arange(self.src.shape[0]))

    def correction_cols(self, cols):
        """Columns C[:, n] returned as rows (for the conjugate transpose)."""
        return self.correction_block(np.arange(self.obs.shape[0]), cols).T.copy()

    # ------------------------------------------------------------------
    def near_grid_part(self, qv, rows, adjoint=False):
        """Near Steps 1-3 (Sec. 3.3): projection, zero-padded FFT convolution
        with the tabulated G^p_near, interpolation.  The conjugate transpose
        projects with the observer weights, convolves with conj(G^p_near(-e))
        and interpolates at the sources."""
        st_in, st_out = (self.st_obs, self.st_src) if adjoint else (self.st_src, self.st_obs)
        Q = _spread(st_in, qv, self.Ng)
        V = self._near_conv(Q, adjoint=adjoint)
        return _interp(st_out, V, rows)

    def near_corr_part(self, qv, rows, adjoint=False):
        """Near Step 4 (Eq. (er))."""
        if adjoint:
            return (np.conj(self.correction_cols(rows)) @ qv.T).T
        return (self.correction_rows(rows) @ qv.T).T

    def far_part(self, qv, rows, adjoint=False):
        """Far Steps 1-3 (Sec. 3.2); the conjugate transpose projects onto the
        observer grid, applies K^H and interpolates from the source grid."""
        if adjoint:
            Qfo = _spread(self.fst_obs, qv, self.Ngf)
            return _interp(self.fst_src, self._far_grid_sum(Qfo, adjoint=True), rows)
        Qf = _spread(self.fst_src, qv, self.Ngf)
        return _interp(self.fst_obs, self._far_grid_sum(Qf), rows)

    @staticmethod
    def _vec(q):
        q = np.asarray(q)
        squeeze = q.ndim == 1
        return (q.reshape(1, -1) if squeeze else q).astype(complex), squeeze

    def apply(self, q, rows=None, parts=("near_grid", "near_corr", "far")):
        """u = (near Steps 1-4 + far Steps 1-3) q at observer indices rows."""
        qv, squeeze = self._vec(q)
        rows = np.arange(self.obs.shape[0]) if rows is None else np.asarray(rows)
        u = np.zeros((qv.shape[0], len(rows)), dtype=complex)
        if "near_grid" in parts:
            u += self.near_grid_part(qv, rows)
        if "near_corr" in parts:
            u += self.near_corr_part(qv, rows)
        if "far" in parts:
            u += self.far_part(qv, rows)
        if self.coincide and self.self_mode == "exclude":
            u -= self.self_value * qv[:, rows]
        return u[0] if squeeze else u

    def adjoint(self, v, rows=None, parts=("near_grid", "near_corr", "far")):
        """w = A^H v at source indices rows (exact conjugate transpose)."""
        vv, squeeze = self._vec(v)
        rows = np.arange(self.src.shape[0]) if rows is None else np.asarray(rows)
        w = np.zeros((vv.shape[0], len(rows)), dtype=complex)
        if "near_grid" in parts:
            w += self.near_grid_part(vv, rows, adjoint=True)
        if "near_corr" in parts:
            w += self.near_corr_part(vv, rows, adjoint=True)
        if "far" in parts:
            w += self.far_part(vv, rows, adjoint=True)
        if self.coincide and self.self_mode == "exclude":
            w -= np.conj(self.self_value) * vv[:, rows]
        return w[0] if squeeze else w
