// Position gradients of the discrete FFT-PIM operator (forces).
//
// For amplitudes q, an upstream gradient g = dL/du (L real, dL = Re sum_m
// conj(g_m) du_m) and coinciding sources and observers (Sec. 2):
//     dL/dr_k = Re( conj(g_k) sum_n dA[k, n]/dr_k q_n )     (k as observer)
//             + Re( sum_m conj(g_m) dA[m, k]/dr_k q_k )     (k as source),
// summed over the planes.  The operator depends on the positions only
// through the Lagrange weights of the projections and interpolations
// (Eq. (projection), Eq. (interpolation); Sec. 3.2 and 3.3) and through the
// correction entries of Eq. (er):
//   * grid parts (near grid, far zone): with U = (grid operator) W q and
//     V = (grid operator)^H W' g the forward and conjugate-transposed grid
//     fields, the gradient is Re(conj(g_k) grad_interp(U)(r_k)) +
//     Re(conj(q_k) grad_interp(V)(r_k)), grad_interp using the weights with
//     one factor differentiated (k_interp_grad);
//   * correction: k_corr_grad walks the close pairs of every point k (as the
//     plan's fill does) and differentiates each entry on the fly,
//       X'_j(k, m) = grad G0(r_k - r_m - R_j) - sum_ab grad w_a(r_k) w_b(r_m) G0tab(a - b + D_j),
//     adding Re(conj(g_k) phi_j X' q_m) + Re(conj(g_m) phi_{-j} X' q_k) (the
//     second is d C[m, k] / d r_k with the image -j, by the symmetry of G0
//     and of the correction region).
// Every kernel writes or adds to its own output in a fixed order: no atomics.
#include "kernels.h"

namespace fftpim {

// Lagrange basis values l_k(u) and derivatives dl_k/du on the nodes 0..Q
// (product rule: dl_k/du = sum_{j != k} (1/(k - j)) prod_{i != k, j} (u - i)/(k - i)).
template <int Q>
__device__ inline void lagrange_with_deriv(double u, double* w, double* dw) {
#pragma unroll
  for (int k = 0; k <= Q; ++k) {
    double val = 1.0, der = 0.0;
#pragma unroll
    for (int j = 0; j <= Q; ++j) {
      if (j == k) continue;
      // d/du of val * (u - j)/(k - j) = der * (u - j)/(k - j) + val / (k - j)
      const double f = (u - j) / static_cast<double>(k - j);
      der = der * f + val / static_cast<double>(k - j);
      val = val * f;
    }
    w[k] = val;
    dw[k] = der;
  }
}

// out[m][c] += sum over planes of Re(conj(coef[m][p]) d/dr_c interp(F)(r_m))
// for one grid (stencil starts s3 and positions u3 within the stencil, [3][N],
// spacing h).  One thread per point.
template <typename R, int Q>
__global__ void __launch_bounds__(256) k_interp_grad(GridArgs g, const double h0, const double h1, const double h2,
                                                     const int32_t* __restrict__ s3, const double* __restrict__ u3,
                                                     int64_t N, const cplx<R>* __restrict__ grid, int P,
                                                     const cplx<R>* __restrict__ coef, double* __restrict__ out) {
  const int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= N) return;
  double wx[Q + 1], wy[Q + 1], wz[Q + 1], dx[Q + 1], dy[Q + 1], dz[Q + 1];
  lagrange_with_deriv<Q>(u3[m], wx, dx);
  lagrange_with_deriv<Q>(u3[N + m], wy, dy);
  lagrange_with_deriv<Q>(u3[2 * N + m], wz, dz);
  for (int a = 0; a <= Q; ++a) {
    dx[a] /= h0;
    dy[a] /= h1;
    dz[a] /= h2;
  }
  const int sx = s3[m], sy = s3[N + m], sz = s3[2 * N + m];
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int p = 0; p < P; ++p) {
    const cplx<R> c = coef[m * P + p];
    const double cr = static_cast<double>(c.x), ci = static_cast<double>(c.y);
    double fx = 0.0, fy = 0.0, fz = 0.0;  // Re(conj(c) grad F) components
    for (int kx = 0; kx <= Q; ++kx) {
      for (int ky = 0; ky <= Q; ++ky) {
        const int64_t row = (static_cast<int64_t>(sx + kx) * g.n[1] + (sy + ky)) * g.n[2] + sz;
        double zr = 0.0, zi = 0.0, zdr = 0.0, zdi = 0.0;
#pragma unroll
        for (int kz = 0; kz <= Q; ++kz) {
          const cplx<R> v = grid[(row + kz) * P + p];
          const double vr = static_cast<double>(v.x), vi = static_cast<double>(v.y);
          zr += wz[kz] * vr;
          zi += wz[kz] * vi;
          zdr += dz[kz] * vr;
          zdi += dz[kz] * vi;
        }
        // Re(conj(c) v) = cr vr + ci vi
        const double t0 = cr * zr + ci * zi, td = cr * zdr + ci * zdi;
        fx += dx[kx] * wy[ky] * t0;
        fy += wx[kx] * dy[ky] * t0;
        fz += wx[kx] * wy[ky] * td;
      }
    }
    gx += fx;
    gy += fy;
    gz += fz;
  }
  out[3 * m] += gx;
  out[3 * m + 1] += gy;
  out[3 * m + 2] += gz;
}

// The correction part of the gradient, one thread per point k (plan order).
// CPLX: complex correction values (a Helmholtz kernel or a phase shift).
template <int Q, bool CPLX>
__global__ void __launch_bounds__(64) k_corr_grad(CorrArgs a, const int32_t* __restrict__ s3,
                                                  const double* __restrict__ u3, const double h0, const double h1,
                                                  const double h2, const double* __restrict__ pos3,
                                                  const int32_t* __restrict__ box_start,
                                                  const cplx<double>* __restrict__ g0tab, int P,
                                                  const void* __restrict__ q_v, const void* __restrict__ g_v,
                                                  int single, double* __restrict__ out) {
  const int32_t *loff0 = a.loff[0], *loff1 = a.loff[1], *loff2 = a.loff[2];
  const int32_t *lent0 = a.lent[0], *lent1 = a.lent[1], *lent2 = a.lent[2];
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= a.N) return;
  const int64_t N = a.N;
  // amplitudes: complex planes of FP64 (single = 0) or FP32 (single = 1)
  auto ampl = [&](const void* v, int64_t pt, int p, double& re, double& im) {
    if (single) {
      const cplx<float> x = static_cast<const cplx<float>*>(v)[pt * P + p];
      re = x.x;
      im = x.y;
    } else {
      const cplx<double> x = static_cast<const cplx<double>*>(v)[pt * P + p];
      re = x.x;
      im = x.y;
    }
  };
  const int S[3] = {s3[k], s3[N + k], s3[2 * N + k]};
  double wk[3][Q + 1], dk[3][Q + 1];
  lagrange_with_deriv<Q>(u3[k], wk[0], dk[0]);
  lagrange_with_deriv<Q>(u3[N + k], wk[1], dk[1]);
  lagrange_with_deriv<Q>(u3[2 * N + k], wk[2], dk[2]);
  const double hh[3] = {h0, h1, h2};
  for (int c = 0; c < 3; ++c)
    for (int t = 0; t <= Q; ++t) dk[c][t] /= hh[c];
  const double rk[3] = {pos3[k], pos3[N + k], pos3[2 * N + k]};
  int lo[3], hi[3];
  lo[0] = loff0[S[0]];
  hi[0] = loff0[S[0] + 1];
  lo[1] = loff1[S[1]];
  hi[1] = loff1[S[1] + 1];
  lo[2] = loff2[S[2]];
  hi[2] = loff2[S[2] + 1];
  const int A = a.nimg_axis, W = a.W, R = a.R;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int ix = lo[0]; ix < hi[0]; ++ix) {
    const int bx = lent0[ix] & 0xffff, mx = lent0[ix] >> 16;
    for (int iy = lo[1]; iy < hi[1]; ++iy) {
      const int by = lent1[iy] & 0xffff, my = lent1[iy] >> 16;
      for (int iz = lo[2]; iz < hi[2]; ++iz) {
        const int bz = lent2[iz] & 0xffff, mz = lent2[iz] >> 16;
        const int64_t b = (static_cast<int64_t>(bx) * a.nb[1] + by) * a.nb[2] + bz;
        const int n0 = box_start[b], n1 = box_start[b + 1];
        for (int n = n0; n < n1; ++n) {
          double wn[3][Q + 1];
          for (int c = 0; c < 3; ++c) lagrange_all<Q, double>(u3[c * N + n], wn[c]);
          // correlations C_c(d) = sum_a w_a(k) w_{a-d}(n) and their
          // derivatives along axis c (weights of k differentiated)
          double C[3][2 * Q + 1], Cd[3][2 * Q + 1];
          for (int c = 0; c < 3; ++c)
            for (int d = -Q; d <= Q; ++d) {
              double s = 0.0, sd = 0.0;
              for (int aa = max(0, d); aa <= min(Q, Q + d); ++aa) {
                s += wk[c][aa] * wn[c][aa - d];
                sd += dk[c][aa] * wn[c][aa - d];
              }
              C[c][d + Q] = s;
              Cd[c][d + Q] = sd;
            }
          // the pair's amplitude products over the planes:
          // s1 = sum_p conj(g_k) q_n (observer side), s2 = sum_p conj(g_n) q_k (source side)
          double s1r = 0.0, s1i = 0.0, s2r = 0.0, s2i = 0.0;
          for (int p = 0; p < P; ++p) {
            double gkr, gki, qnr, qni, gnr, gni, qkr, qki;
            ampl(g_v, k, p, gkr, gki);
            ampl(q_v, n, p, qnr, qni);
            ampl(g_v, n, p, gnr, gni);
            ampl(q_v, k, p, qkr, qki);
            s1r += gkr * qnr + gki * qni;
            s1i += gkr * qni - gki * qnr;
            s2r += gnr * qkr + gni * qki;
            s2i += gnr * qki - gni * qkr;
          }
          const double rn[3] = {pos3[n], pos3[N + n], pos3[2 * N + n]};
          for (int gxi = 0; gxi < A; ++gxi) {
            if (!((mx >> gxi) & 1)) continue;
            const int imx = gxi - a.id * a.per[0];
            for (int gyi = 0; gyi < A; ++gyi) {
              if (!((my >> gyi) & 1)) continue;
              const int imy = gyi - a.id * a.per[1];
              for (int gzi = 0; gzi < A; ++gzi) {
                if (!((mz >> gzi) & 1)) continue;
                const int imz = gzi - a.id * a.per[2];
                if (a.ball && !ball_close(a.bw, a.br2, S[0] - bx - imx * a.nint[0], S[1] - by - imy * a.nint[1],
                                          S[2] - bz - imz * a.nint[2]))
                  continue;
                const int D[3] = {S[0] - bx - imx * a.nint[0], S[1] - by - imy * a.nint[1],
                                  S[2] - bz - imz * a.nint[2]};
                // exact part: grad G0(d), d = r_k - r_n - R_j (dropped for the self pair)
                double ex[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
                if (!(n == k && imx == 0 && imy == 0 && imz == 0)) {
                  const double d0 = rk[0] - rn[0] - imx * a.L[0];
                  const double d1 = rk[1] - rn[1] - imy * a.L[1];
                  const double d2 = rk[2] - rn[2] - imz * a.L[2];
                  const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                  const double amp = (a.k0_im != 0.0 ? exp(a.k0_im * r) : 1.0) / (4.0 * M_PI * r);
                  double sn, cs;
                  sincos(a.k0 * r, &sn, &cs);
                  // G0 = amp (cos - j sin); dG0/dr = G0 (-j k0 - 1/r), k0 = k0 + j k0_im
                  const double g0r = amp * cs, g0i = -amp * sn;
                  const double fr = a.k0_im - 1.0 / r, fi = -a.k0;  // -j k0 - 1/r
                  const double dgr = g0r * fr - g0i * fi, dgi = g0r * fi + g0i * fr;
                  const double dd[3] = {d0, d1, d2};
                  for (int c = 0; c < 3; ++c) {
                    ex[c][0] = dgr * dd[c] / r;
                    ex[c][1] = CPLX ? dgi * dd[c] / r : 0.0;
                  }
                }
                // grid part: three components of sum_d C C C G0tab(D + d),
                // one factor differentiated
                double pyr = 0.0, pyi = 0.0, pzr = 0.0, pzi = 0.0;
                double gridx_r = 0.0, gridx_i = 0.0;
                for (int ddx = -Q; ddx <= Q; ++ddx) {
                  const int64_t rowx = static_cast<int64_t>(D[0] + ddx + R) * W;
                  double ar = 0.0, ai = 0.0, ayr = 0.0, ayi = 0.0, azr = 0.0, azi = 0.0;
                  for (int ddy = -Q; ddy <= Q; ++ddy) {
                    const cplx<double>* tab = g0tab + (rowx + D[1] + ddy + R) * W + (D[2] + R);
                    double sr = 0.0, si = 0.0, sdr = 0.0, sdi = 0.0;
#pragma unroll
                    for (int ddz = -Q; ddz <= Q; ++ddz) {
                      const cplx<double> t = tab[ddz];
                      sr += C[2][ddz + Q] * t.x;
                      sdr += Cd[2][ddz + Q] * t.x;
                      if (CPLX) {
                        si += C[2][ddz + Q] * t.y;
                        sdi += Cd[2][ddz + Q] * t.y;
                      }
                    }
                    const double cy = C[1][ddy + Q], cdy = Cd[1][ddy + Q];
                    ar += cy * sr;
                    ai += cy * si;
                    ayr += cdy * sr;
                    ayi += cdy * si;
                    azr += cy * sdr;
                    azi += cy * sdi;
                  }
                  const double cx = C[0][ddx + Q], cdx = Cd[0][ddx + Q];
                  gridx_r += cdx * ar;
                  gridx_i += cdx * ai;
                  pyr += cx * ayr;
                  pyi += cx * ayi;
                  pzr += cx * azr;
                  pzi += cx * azi;
                }
                const double xr_[3] = {ex[0][0] - gridx_r, ex[1][0] - pyr, ex[2][0] - pzr};
                const double xi_[3] = {ex[0][1] - gridx_i, ex[1][1] - pyi, ex[2][1] - pzi};
                // phases of image j and of image -j
                const int pidx = (gxi * A + gyi) * A + gzi;
                const int nidx = ((a.per[0] ? A - 1 - gxi : gxi) * A + (a.per[1] ? A - 1 - gyi : gyi)) * A +
                                 (a.per[2] ? A - 1 - gzi : gzi);
                double fjr = 1.0, fji = 0.0, fnr = 1.0, fni = 0.0;
                if (CPLX) {
                  fjr = a.phase[2 * pidx];
                  fji = a.phase[2 * pidx + 1];
                  fnr = a.phase[2 * nidx];
                  fni = a.phase[2 * nidx + 1];
                }
                // Re(phi_j X s1) + Re(phi_{-j} X s2) per component
                const double a1r = fjr * s1r - fji * s1i, a1i = fjr * s1i + fji * s1r;
                const double a2r = fnr * s2r - fni * s2i, a2i = fnr * s2i + fni * s2r;
                const double cr = a1r + a2r, ci = a1i + a2i;
                gx += xr_[0] * cr - xi_[0] * ci;
                gy += xr_[1] * cr - xi_[1] * ci;
                gz += xr_[2] * cr - xi_[2] * ci;
              }
            }
          }
        }
      }
    }
  }
  out[3 * k] += gx;
  out[3 * k + 1] += gy;
  out[3 * k + 2] += gz;
}

__global__ void k_unpermute3(const double* __restrict__ in, const int32_t* __restrict__ perm, int64_t N, int use_perm,
                             double* __restrict__ out) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int64_t d = use_perm ? perm[j] : j;
  out[3 * d] = in[3 * j];
  out[3 * d + 1] = in[3 * j + 1];
  out[3 * d + 2] = in[3 * j + 2];
}

void launch_unpermute3(const double* in, const int32_t* perm, int64_t N, bool use_perm, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_unpermute3, dim3(static_cast<unsigned>((N + 255) / 256)), dim3(256), 0, st, in, perm, N,
                     use_perm ? 1 : 0, out);
}

template <typename R>
int launch_interp_grad(int q, const GridArgs& g, const double h[3], const int32_t* s3, const double* u3, int64_t N,
                       const void* grid, int P, const void* coef, double* out, hipStream_t st) {
  const dim3 gr(static_cast<unsigned>((N + 255) / 256));
#define FFTPIM_IG(QV)                                                                                        \
  hipLaunchKernelGGL((k_interp_grad<R, QV>), gr, dim3(256), 0, st, g, h[0], h[1], h[2], s3, u3, N,           \
                     static_cast<const cplx<R>*>(grid), P, static_cast<const cplx<R>*>(coef), out)
  switch (q) {
    case 1: FFTPIM_IG(1); break;
    case 2: FFTPIM_IG(2); break;
    case 3: FFTPIM_IG(3); break;
    case 4: FFTPIM_IG(4); break;
    case 5: FFTPIM_IG(5); break;
    case 6: FFTPIM_IG(6); break;
    case 7: FFTPIM_IG(7); break;
    case 8: FFTPIM_IG(8); break;
    case 9: FFTPIM_IG(9); break;
    default: return FFTPIM_ERR_UNSUPPORTED;
  }
#undef FFTPIM_IG
  return FFTPIM_OK;
}

int launch_corr_grad(int q, bool cplx_vals, const CorrArgs& a, const int32_t* s3, const double* u3, const double h[3],
                     const double* pos3, const int32_t* box_start, const void* g0tab, int P, const void* qint,
                     const void* gint, bool single, double* out, hipStream_t st) {
  const dim3 gr(static_cast<unsigned>((a.N + 63) / 64));
  const cplx<double>* tab = static_cast<const cplx<double>*>(g0tab);
#define FFTPIM_CG(QV)                                                                                           \
  do {                                                                                                          \
    if (cplx_vals)                                                                                              \
      hipLaunchKernelGGL((k_corr_grad<QV, true>), gr, dim3(64), 0, st, a, s3, u3, h[0], h[1], h[2], pos3,        \
                         box_start, tab, P, qint, gint, single ? 1 : 0, out);                                   \
    else                                                                                                        \
      hipLaunchKernelGGL((k_corr_grad<QV, false>), gr, dim3(64), 0, st, a, s3, u3, h[0], h[1], h[2], pos3,       \
                         box_start, tab, P, qint, gint, single ? 1 : 0, out);                                   \
  } while (0)
  switch (q) {
    case 1: FFTPIM_CG(1); break;
    case 2: FFTPIM_CG(2); break;
    case 3: FFTPIM_CG(3); break;
    case 4: FFTPIM_CG(4); break;
    case 5: FFTPIM_CG(5); break;
    case 6: FFTPIM_CG(6); break;
    case 7: FFTPIM_CG(7); break;
    case 8: FFTPIM_CG(8); break;
    default: return FFTPIM_ERR_UNSUPPORTED;
  }
#undef FFTPIM_CG
  return FFTPIM_OK;
}

template int launch_interp_grad<double>(int, const GridArgs&, const double*, const int32_t*, const double*, int64_t,
                                        const void*, int, const void*, double*, hipStream_t);
template int launch_interp_grad<float>(int, const GridArgs&, const double*, const int32_t*, const double*, int64_t,
                                       const void*, int, const void*, double*, hipStream_t);

}  // namespace fftpim
