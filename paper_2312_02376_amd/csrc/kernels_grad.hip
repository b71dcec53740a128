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

constexpr int kGradWaves = 4;             // wavefronts per workgroup
constexpr int kGradPPW = 8;               // observer points per wavefront
constexpr int kGradListInts = kPairListInts;
constexpr int kGradWDoubles = 6 * 16;           // per-wave LDS weights of k: w[3][Q+1], dw[3][Q+1], Q < 16

inline size_t grad_list_bytes() {
  return static_cast<size_t>(kGradWaves) * (kGradListInts * sizeof(int) + kGradWDoubles * sizeof(double));
}

// The correction part of the gradient.  One wavefront per point k (plan
// order; kGradPPW points in turn); wave_pairs hands its close pairs to the
// lanes 64 at a time, so the lanes stay busy whatever the box occupancy.
// The G0 table is read from LDS when LT.
template <int Q, bool CPLX, bool LT>
__global__ void __launch_bounds__(64 * kGradWaves) k_corr_grad(
    CorrArgs a, const int32_t* __restrict__ s3, const double* __restrict__ u3, const double h0, const double h1,
    const double h2, const double* __restrict__ pos3, const int32_t* __restrict__ box_start,
    const cplx<double>* __restrict__ g0tab, int P, const void* __restrict__ q_v, const void* __restrict__ g_v,
    int single, double* __restrict__ out) {
  extern __shared__ __align__(16) double lt[];
  const int64_t tabn = static_cast<int64_t>(a.W) * a.W * a.W;
  if (LT) tab_stage<CPLX>(g0tab, lt, tabn);
  double* wlds = lt + (LT ? tabn * (CPLX ? 2 : 1) : 0);
  int* lists = reinterpret_cast<int*>(wlds + kGradWaves * kGradWDoubles);
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int lane = static_cast<int>(threadIdx.x) & 63;
  // the weights of k and their derivatives (the same for every lane) live in
  // LDS, read as broadcasts, to keep registers for the per-pair arrays
  double* wk = wlds + wave * kGradWDoubles;  // [3][Q + 1]
  double* dk = wk + 3 * (Q + 1);             // [3][Q + 1]
  int* pre = lists + wave * kGradListInts;  // the wave's pair-enumeration lists
  const int64_t N = a.N;
  const int A = a.nimg_axis, W = a.W, R = a.R;
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
  for (int pp = 0; pp < kGradPPW; ++pp) {
    const int64_t k = (static_cast<int64_t>(blockIdx.x) * kGradWaves + wave) * kGradPPW + pp;
    if (k >= N) break;
    const int S[3] = {s3[k], s3[N + k], s3[2 * N + k]};
    if (lane < 3) {
      double w[Q + 1], dw[Q + 1];
      lagrange_with_deriv<Q>(u3[lane * N + k], w, dw);
      const double hc = lane == 0 ? h0 : (lane == 1 ? h1 : h2);
#pragma unroll
      for (int t = 0; t <= Q; ++t) {
        wk[lane * (Q + 1) + t] = w[t];
        dk[lane * (Q + 1) + t] = dw[t] / hc;
      }
    }
    wave_lds_sync();
    const double rk[3] = {pos3[k], pos3[N + k], pos3[2 * N + k]};
    int lo[3], hi[3];
    axis_range(a.loff[0], S[0], lo[0], hi[0]);
    axis_range(a.loff[1], S[1], lo[1], hi[1]);
    axis_range(a.loff[2], S[2], lo[2], hi[2]);
    double gx = 0.0, gy = 0.0, gz = 0.0;
    wave_pairs(a, S, lo, hi, box_start, pre, lane, [&](int64_t, int n, int bx, int by, int bz, int mx, int my, int mz) {
          double wn[3][Q + 1];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) lagrange_all<Q, double>(u3[cc * N + n], wn[cc]);
          // correlations C_c(d) = sum_a w_a(k) w_{a-d}(n) and their
          // derivatives along axis c (weights of k differentiated); every
          // loop over these small arrays is unrolled so they stay in registers
          double C[3][2 * Q + 1], Cd[3][2 * Q + 1];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
#pragma unroll
            for (int d = -Q; d <= Q; ++d) {
              double sw = 0.0, sd = 0.0;
#pragma unroll
              for (int aa = 0; aa <= Q; ++aa) {
                if (aa - d < 0 || aa - d > Q) continue;
                sw += wk[cc * (Q + 1) + aa] * wn[cc][aa - d];
                sd += dk[cc * (Q + 1) + aa] * wn[cc][aa - d];
              }
              C[cc][d + Q] = sw;
              Cd[cc][d + Q] = sd;
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
                if (!image_close(a, S, bx, by, bz, imx, imy, imz)) continue;
                const int D[3] = {S[0] - bx - imx * a.nint[0], S[1] - by - imy * a.nint[1],
                                  S[2] - bz - imz * a.nint[2]};
                // exact part: grad G0(d), d = r_k - r_n - R_j (dropped for the self pair)
                double ex3[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
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
#pragma unroll
                  for (int cc = 0; cc < 3; ++cc) {
                    ex3[cc][0] = dgr * dd[cc] / r;
                    ex3[cc][1] = CPLX ? dgi * dd[cc] / r : 0.0;
                  }
                }
                // grid part: three components of sum_d C C C G0tab(D + d),
                // one factor differentiated
                double pyr = 0.0, pyi = 0.0, pzr = 0.0, pzi = 0.0;
                double gridx_r = 0.0, gridx_i = 0.0;
                // x stays a loop (bounding the loads in flight, hence the
                // registers); its two weights are picked by selects, not by
                // a run-time index, so C and Cd stay in registers
#pragma nounroll
                for (int ddx = -Q; ddx <= Q; ++ddx) {
                  const int64_t rowx = static_cast<int64_t>(D[0] + ddx + R) * W;
                  double ar = 0.0, ai = 0.0, ayr = 0.0, ayi = 0.0, azr = 0.0, azi = 0.0;
#pragma unroll
                  for (int ddy = -Q; ddy <= Q; ++ddy) {
                    const int64_t toff = (rowx + D[1] + ddy + R) * W + (D[2] + R);
                    double sr = 0.0, si = 0.0, sdr = 0.0, sdi = 0.0;
#pragma unroll
                    for (int ddz = -Q; ddz <= Q; ++ddz) {
                      double tx, ty;
                      tab_get<CPLX, LT>(g0tab, lt, toff + ddz, tx, ty);
                      sr += C[2][ddz + Q] * tx;
                      sdr += Cd[2][ddz + Q] * tx;
                      if (CPLX) {
                        si += C[2][ddz + Q] * ty;
                        sdi += Cd[2][ddz + Q] * ty;
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
                  double cx = 0.0, cdx = 0.0;
#pragma unroll
                  for (int t = 0; t <= 2 * Q; ++t) {
                    cx = (t == ddx + Q) ? C[0][t] : cx;
                    cdx = (t == ddx + Q) ? Cd[0][t] : cdx;
                  }
                  gridx_r += cdx * ar;
                  gridx_i += cdx * ai;
                  pyr += cx * ayr;
                  pyi += cx * ayi;
                  pzr += cx * azr;
                  pzi += cx * azi;
                }
                const double xr_[3] = {ex3[0][0] - gridx_r, ex3[1][0] - pyr, ex3[2][0] - pzr};
                const double xi_[3] = {ex3[0][1] - gridx_i, ex3[1][1] - pyi, ex3[2][1] - pzi};
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
    });
    gx = wave_sum(gx);
    gy = wave_sum(gy);
    gz = wave_sum(gz);
    if (lane == 0) {
      out[3 * k] += gx;
      out[3 * k + 1] += gy;
      out[3 * k + 2] += gz;
    }
    wave_lds_sync();
  }
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
  // the table in LDS beside the wave lists when both fit, else read from
  // global memory
  const size_t tab = tab_lds_bytes(a.W, cplx_vals);
  const bool lt = tab + grad_list_bytes() <= kTabLdsBytes;
  const size_t lds = (lt ? tab : 0) + grad_list_bytes();
  const int64_t per_block = static_cast<int64_t>(kGradWaves) * kGradPPW;
  const dim3 gr(static_cast<unsigned>((a.N + per_block - 1) / per_block));
  const cplx<double>* tab_d = static_cast<const cplx<double>*>(g0tab);
#define FFTPIM_CG1(QV, CV, LV)                                                                                  \
  hipLaunchKernelGGL((k_corr_grad<QV, CV, LV>), gr, dim3(64 * kGradWaves), lds, st, a, s3, u3, h[0], h[1], h[2], \
                     pos3, box_start, tab_d, P, qint, gint, single ? 1 : 0, out)
#define FFTPIM_CG(QV)                                  \
  do {                                                 \
    if (cplx_vals) {                                   \
      if (lt) FFTPIM_CG1(QV, true, true);              \
      else FFTPIM_CG1(QV, true, false);                \
    } else {                                           \
      if (lt) FFTPIM_CG1(QV, false, true);             \
      else FFTPIM_CG1(QV, false, false);               \
    }                                                  \
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
#undef FFTPIM_CG1
  return FFTPIM_OK;
}

template int launch_interp_grad<double>(int, const GridArgs&, const double*, const int32_t*, const double*, int64_t,
                                        const void*, int, const void*, double*, hipStream_t);
template int launch_interp_grad<float>(int, const GridArgs&, const double*, const int32_t*, const double*, int64_t,
                                       const void*, int, const void*, double*, hipStream_t);

}  // namespace fftpim
