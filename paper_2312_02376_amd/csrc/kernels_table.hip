// Plan time, on the device: the far-zone kernel table of Sec. 3.2 for every
// lattice class except 2D periodicity with k0 or a phase shift (that one has
// its own kernel in kernels_far.hip).  Entry e is
//     G^p_far(r) = G^p(r) - sum_{|i_c| <= i_d} phi_i G0(r - R_i)
// at the offset r between the shifted observer and source grids, with G^p from
// the paper's rapidly converging series:
//   3D, neutral static:  Eq. (lgf_3) plus Lz/(12 Lx Ly) (zero cell mean), the
//                        x role on the axis with the smallest |r_c|;
//   3D, k0 or a phase:   Eq. (pgf_3) with the z images summed in closed form,
//                        the z role on the axis with the largest |r_c| whose
//                        lateral Floquet wavenumbers have no 0/0 term;
//   2D, neutral static:  Eq. (lgf_2), the x role on the periodic axis with the
//                        smaller |r_c|;
//   1D, neutral static:  Eq. (lgf_1);
//   1D, k0 or a phase:   Eq. (pgf_1) as (1/(2 pi Lx)) sum_m e^{-j k_xm x}
//                        K0(j k_rho,m rho) (H0^(2)(z) = (2j/pi) K0(j z)).
// The grids are shifted by half a cell on every axis, so no offset has a
// vanishing transverse distance.  One block per entry; its threads split the
// outer Floquet / lattice index and add their partial sums in a fixed tree
// order.  Wavenumbers may be complex (Sec. 2); square roots take Im <= 0.
#include "kernels.h"

namespace fftpim {

namespace {

constexpr double kPiD = 3.14159265358979323846;
constexpr double kGammaD = 0.57721566490153286061;
constexpr double kDecayD = 41.0;  // terms below e^-41 are dropped
constexpr int kTabThreads = 256;

// K0(x), real x > 0: DLMF 10.31.2 for x <= 2, else DLMF 10.32.9 by the
// trapezoidal rule (step min(1/4, 1/(2 sqrt x))).
__device__ double k0_real(double x) {
  if (x <= 2.0) {
    const double t = 0.25 * x * x;
    double term = 1.0, i0 = 1.0, s = 0.0, hk = 0.0;
    for (int k = 1; k < 40; ++k) {
      term *= t / (static_cast<double>(k) * k);
      hk += 1.0 / k;
      i0 += term;
      s += term * hk;
      if (term < 1e-18 * i0) break;
    }
    return -(log(0.5 * x) + kGammaD) * i0 + s;
  }
  const double tau = fmin(0.25, 0.5 / sqrt(x));
  double acc = 0.5;
  for (int j = 1; j < 10000; ++j) {
    const double e = -x * (cosh(j * tau) - 1.0);
    if (e < -kDecayD) break;
    acc += exp(e);
  }
  return tau * acc * exp(-x);
}

__device__ inline cplx<double> cmul_d(cplx<double> a, cplx<double> b) { return cmul(a, b); }

__device__ inline cplx<double> clog_d(cplx<double> z) {
  return cmake<double>(log(hypot(z.x, z.y)), atan2(z.y, z.x));
}

__device__ inline cplx<double> csqrt_d(cplx<double> w) {  // principal branch
  const double a = hypot(w.x, w.y);
  if (a == 0.0) return cmake<double>(0.0, 0.0);
  if (w.x >= 0.0) {
    const double re = sqrt(0.5 * (a + w.x));
    return cmake<double>(re, w.y / (2.0 * re));
  }
  const double im = copysign(sqrt(0.5 * (a - w.x)), w.y);
  return cmake<double>(w.y / (2.0 * im), im);
}

// H0^(2)(z) = J0 - j Y0 for moderate |z| and small |Im z|: Miller's backward
// recurrence for J_n normalised by J0 + 2 sum J_2k = 1 (DLMF 10.6.1, 10.12.4)
// and Neumann's expansion Y0 = (2/pi)(ln(z/2) + gamma) J0 - (4/pi) sum (-1)^k J_2k / k.
__device__ cplx<double> hankel2_0_d(cplx<double> z) {
  const double az = hypot(z.x, z.y);
  const int start = 2 * static_cast<int>(0.5 * (1.5 * az + 40.0));
  cplx<double> f_up = cmake<double>(0.0, 0.0), f = cmake<double>(1e-30, 0.0);
  cplx<double> S = cmake<double>(0.0, 0.0), T = cmake<double>(0.0, 0.0);
  const cplx<double> zinv = cdiv_d(cmake<double>(1.0, 0.0), z);
  for (int k = start; k >= 1; --k) {
    if ((k & 1) == 0) {
      const int h = k / 2;
      S = cadd(S, cscale(f, 2.0));
      T = cadd(T, cscale(f, ((h & 1) ? -1.0 : 1.0) / static_cast<double>(h)));
    }
    const cplx<double> f_down = csub(cscale(cmul(zinv, f), 2.0 * k), f_up);
    f_up = f;
    f = f_down;
    if (hypot(f.x, f.y) > 1e250) {
      f = cscale(f, 1e-250);
      f_up = cscale(f_up, 1e-250);
      S = cscale(S, 1e-250);
      T = cscale(T, 1e-250);
    }
  }
  S = cadd(S, f);
  const cplx<double> j0 = cdiv_d(f, S);
  const cplx<double> lz = cadd(clog_d(cscale(z, 0.5)), cmake<double>(kGammaD, 0.0));
  const cplx<double> y0 = csub(cscale(cmul(lz, j0), 2.0 / kPiD), cscale(cdiv_d(T, S), 4.0 / kPiD));
  return cmake<double>(j0.x + y0.y, j0.y - y0.x);  // j0 - j y0
}

// K0(w) for complex w with Re w >= 0 (the same four regimes as the host
// evaluator: DLMF 10.31.2 series for |w| <= 2, DLMF 10.40.2 asymptotic series
// for |w| >= 18, DLMF 10.32.9 by the trapezoidal rule for Re w >= 1.5, and
// K0(w) = -(j pi/2) H0^(2)(-j w) next to the imaginary axis).
__device__ cplx<double> k0_cplx(cplx<double> w) {
  if (w.y == 0.0 && w.x > 0.0) return cmake<double>(k0_real(w.x), 0.0);
  const double aw = hypot(w.x, w.y);
  if (aw <= 2.0) {
    const cplx<double> t = cscale(cmul(w, w), 0.25);
    cplx<double> term = cmake<double>(1.0, 0.0), i0 = cmake<double>(1.0, 0.0), s = cmake<double>(0.0, 0.0);
    double hk = 0.0;
    for (int k = 1; k < 60; ++k) {
      term = cscale(cmul(term, t), 1.0 / (static_cast<double>(k) * k));
      hk += 1.0 / k;
      i0 = cadd(i0, term);
      s = cadd(s, cscale(term, hk));
      if (hypot(term.x, term.y) < 1e-18 * hypot(i0.x, i0.y)) break;
    }
    const cplx<double> lw = cadd(clog_d(cscale(w, 0.5)), cmake<double>(kGammaD, 0.0));
    return csub(s, cmul(lw, i0));
  }
  if (aw >= 18.0) {
    cplx<double> sum = cmake<double>(1.0, 0.0), term = cmake<double>(1.0, 0.0);
    const cplx<double> winv = cdiv_d(cmake<double>(1.0, 0.0), w);
    for (int k = 1; k < 100; ++k) {
      const double a = 2.0 * k - 1.0;
      const cplx<double> next = cscale(cmul(term, winv), -(a * a) / (8.0 * k));
      if (hypot(next.x, next.y) >= hypot(term.x, term.y)) break;
      term = next;
      sum = cadd(sum, term);
      if (hypot(term.x, term.y) < 1e-17 * hypot(sum.x, sum.y)) break;
    }
    const cplx<double> pre = csqrt_d(cdiv_d(cmake<double>(kPiD / 2.0, 0.0), w));
    return cmul(cmul(pre, cexp_d(cmake<double>(-w.x, -w.y))), sum);
  }
  if (w.x >= 1.5) {
    const double theta = fabs(atan2(w.y, w.x));
    const double d = fmin(0.25 * kPiD, 0.5 * (0.5 * kPiD - theta));
    const double tau = fmin(0.25, 2.0 * kPiD * d / 40.0);
    cplx<double> acc = cmake<double>(0.5, 0.0);
    for (int j = 1; j < 1000000; ++j) {
      const double c1 = cosh(j * tau) - 1.0;
      if (w.x * c1 > kDecayD + 4.0) break;
      acc = cadd(acc, cexp_d(cmake<double>(-w.x * c1, -w.y * c1)));
    }
    return cscale(cmul(acc, cexp_d(cmake<double>(-w.x, -w.y))), tau);
  }
  const cplx<double> h = hankel2_0_d(cmake<double>(w.y, -w.x));
  return cmake<double>(0.5 * kPiD * h.y, -0.5 * kPiD * h.x);  // -(j pi/2) h
}

// ln(1 - 2 e^{-a} cos(theta) + e^{-2a}) without cancellation
__device__ inline double log_layer_d(double a, double theta) {
  const double e = expm1(-a);
  const double s = sin(0.5 * theta);
  return log(e * e + 4.0 * exp(-a) * s * s);
}

// A 3D axis pair (a, b) is usable as the lateral axes of Eq. (pgf_3) unless
// the kernel is static and both phase shifts are whole multiples of 2 pi / L.
__device__ inline bool lateral_ok_d(const FarTableArgs& t, int a, int b) {
  if (t.k0 != 0.0 || t.k0_im != 0.0) return true;
  auto on_grid = [&](int c) {
    if (t.kt_im[c] != 0.0) return false;
    const double q = t.kt[c] * t.L[c] / (2.0 * kPiD);
    return fabs(q - rint(q)) < 1e-12;
  };
  return !(on_grid(a) && on_grid(b));
}

}  // namespace

// The lattice classes of the kernel below.
enum { kTab3Static = 0, kTab3Dyn = 1, kTab2Static = 2, kTab1Static = 3, kTab1Dyn = 4 };

__global__ void __launch_bounds__(kTabThreads) k_far_table(FarTableArgs a, int cls, cplx<double>* __restrict__ table) {
  __shared__ double shr[kTabThreads], shi[kTabThreads];
  __shared__ int roles[3];
  const int t = threadIdx.x;
  const int sy = 2 * a.nf[1] - 1, sz = 2 * a.nf[2] - 1;
  const int64_t e = blockIdx.x;
  const int dz = static_cast<int>(e % sz), dy = static_cast<int>((e / sz) % sy),
            dx = static_cast<int>(e / (static_cast<int64_t>(sz) * sy));
  const double r0[3] = {(dx - (a.nf[0] - 1) - 0.5) * a.delta[0], (dy - (a.nf[1] - 1) - 0.5) * a.delta[1],
                        (dz - (a.nf[2] - 1) - 0.5) * a.delta[2]};
  const cplx<double> k0 = cmake<double>(a.k0, a.k0_im);
  cplx<double> kt[3];
  for (int c = 0; c < 3; ++c) kt[c] = cmake<double>(a.kt[c], a.kt_im[c]);
  // reduce into the cell on the periodic axes; Bloch phase exp(-j sum kt_c n_c L_c)
  double r[3] = {r0[0], r0[1], r0[2]};
  cplx<double> barg = cmake<double>(0.0, 0.0);
  for (int c = 0; c < a.dims; ++c) {
    const double n = rint(r[c] / a.L[c]);
    r[c] -= n * a.L[c];
    barg = cadd(barg, cscale(kt[c], n * a.L[c]));
  }
  // axis roles
  if (t == 0) {
    int xr = 0, yr = 1, zr = 2;
    if (cls == kTab3Static) {
      for (int c = 1; c < 3; ++c)
        if (fabs(r[c]) < fabs(r[xr])) xr = c;
      yr = (xr + 1) % 3;
      zr = (xr + 2) % 3;
    } else if (cls == kTab3Dyn) {
      int order[3] = {0, 1, 2};
      for (int i = 0; i < 3; ++i)  // stable sort by decreasing |r_c|
        for (int j = 2; j > i; --j)
          if (fabs(r[order[j]]) > fabs(r[order[j - 1]])) {
            const int tmp = order[j];
            order[j] = order[j - 1];
            order[j - 1] = tmp;
          }
      zr = -1;
      for (int i = 0; i < 3 && zr < 0; ++i) {
        const int z = order[i];
        if (lateral_ok_d(a, (z + 1) % 3, (z + 2) % 3)) zr = z;
      }
      if (zr < 0) zr = order[0];  // unsupported classes are refused before planning
      xr = (zr + 1) % 3;
      yr = (zr + 2) % 3;
    } else if (cls == kTab2Static) {
      if (fabs(r[1]) < fabs(r[0])) {
        xr = 1;
        yr = 0;
      }
    }
    roles[0] = xr;
    roles[1] = yr;
    roles[2] = zr;
  }
  __syncthreads();
  const int xr = roles[0], yr = roles[1], zr = roles[2];
  const double x = r[xr], y = r[yr], z = r[zr];
  const double Lx = a.L[xr], Ly = a.L[yr], Lz = a.L[zr];
  double sr = 0.0, si = 0.0;
  if (cls == kTab3Static || cls == kTab2Static) {
    // (1/(pi Lx)) sum_{m>=1} sum_{n, k} K0(2 pi m rho_nk / Lx) cos(2 pi m x / Lx),
    // rho_nk = sqrt((n Ly + y)^2 + (k Lz + z)^2) (k = 0 only in 2D); a pair
    // (m, k) per thread iteration
    const bool kz = cls == kTab3Static;
    const double rho0 = sqrt(y * y + z * z);
    const int mmax = static_cast<int>(kDecayD * Lx / (2.0 * kPiD * rho0)) + 1;
    const int kmax = kz ? static_cast<int>(ceil(kDecayD * Lx / (2.0 * kPiD * Lz))) + 1 : 0;
    const int nk = 2 * kmax + 1;
    for (int it = t; it < mmax * nk; it += kTabThreads) {
      const int m = it / nk + 1, k = it % nk - kmax;
      const double cutoff = kDecayD * Lx / (2.0 * kPiD * m);
      const double zz = kz ? k * Lz + z : z;
      if (fabs(zz) > cutoff) continue;
      const int nmax = static_cast<int>(ceil(cutoff / Ly)) + 1;
      const double cx = cos(2.0 * m * kPiD * x / Lx);
      double acc = 0.0;
      for (int n = -nmax; n <= nmax; ++n) {
        const double yy = n * Ly + y;
        const double rho = sqrt(yy * yy + zz * zz);
        if (rho > cutoff) continue;
        acc += k0_real(2.0 * m * kPiD * rho / Lx);
      }
      sr += acc * cx;
    }
  } else if (cls == kTab1Static) {
    const double rho = sqrt(y * y + z * z);
    const int mmax = static_cast<int>(kDecayD * Lx / (2.0 * kPiD * rho)) + 1;
    for (int m = 1 + t; m <= mmax; m += kTabThreads) sr += k0_real(2.0 * m * kPiD * rho / Lx) * cos(2.0 * m * kPiD * x / Lx);
  } else if (cls == kTab1Dyn) {
    const double rho = sqrt(y * y + z * z);
    const double kreach = kDecayD / rho + hypot(k0.x, k0.y) + hypot(kt[0].x, kt[0].y);
    const int mmax = static_cast<int>(ceil(kreach * Lx / (2.0 * kPiD))) + 1;
    for (int m = -mmax + t; m <= mmax; m += kTabThreads) {
      const cplx<double> kx = cadd(kt[0], cmake<double>(2.0 * kPiD * m / Lx, 0.0));
      const cplx<double> krho = csqrt_im_nonpos_d(csub(cmul(k0, k0), cmul(kx, kx)));
      const cplx<double> kk = k0_cplx(cmake<double>(-krho.y * rho, krho.x * rho));  // K0(j krho rho)
      const cplx<double> v = cmul(cexp_d(cmake<double>(kx.y * x, -kx.x * x)), kk);
      sr += v.x;
      si += v.y;
    }
  } else {  // kTab3Dyn: Eq. (pgf_3) with the z images in closed form
    const cplx<double> ktx = kt[xr], kty = kt[yr], ktz = kt[zr];
    const double az = fabs(z);
    const double kreach = kDecayD / az + hypot(k0.x, k0.y) + hypot(ktx.x, ktx.y) + hypot(kty.x, kty.y);
    const int mmax = static_cast<int>(ceil(kreach * Lx / (2.0 * kPiD))) + 1;
    const int nmax = static_cast<int>(ceil(kreach * Ly / (2.0 * kPiD))) + 1;
    const cplx<double> k02 = cmul(k0, k0);
    for (int m = -mmax + t; m <= mmax; m += kTabThreads) {
      const cplx<double> kx = cadd(ktx, cmake<double>(2.0 * kPiD * m / Lx, 0.0));
      const cplx<double> kx2 = cmul(kx, kx);
      for (int n = -nmax; n <= nmax; ++n) {
        const cplx<double> ky = cadd(kty, cmake<double>(2.0 * kPiD * n / Ly, 0.0));
        const cplx<double> kz = csqrt_im_nonpos_d(csub(csub(k02, kx2), cmul(ky, ky)));
        // am = exp(-j (kz - kz0) Lz), ap = exp(-j (kz + kz0) Lz)
        const cplx<double> dm = cscale(csub(kz, ktz), Lz), dp = cscale(cadd(kz, ktz), Lz);
        const cplx<double> am = cexp_d(cmake<double>(dm.y, -dm.x)), ap = cexp_d(cmake<double>(dp.y, -dp.x));
        const cplx<double> e1 = cexp_d(cmake<double>(kz.y * az, -kz.x * az));     // exp(-j kz |z|)
        const cplx<double> e2 = cexp_d(cmake<double>(kz.y * z, -kz.x * z));       // exp(-j kz z)
        const cplx<double> e3 = cexp_d(cmake<double>(-kz.y * z, kz.x * z));       // exp(+j kz z)
        const cplx<double> one = cmake<double>(1.0, 0.0);
        cplx<double> zp = cadd(e1, cdiv_d(cmul(am, e2), csub(one, am)));
        zp = cadd(zp, cdiv_d(cmul(ap, e3), csub(one, ap)));
        const cplx<double> lat = cadd(cscale(kx, x), cscale(ky, y));
        const cplx<double> v = cdiv_d(cmul(cexp_d(cmake<double>(lat.y, -lat.x)), zp), kz);
        sr += v.x;
        si += v.y;
      }
    }
  }
  shr[t] = sr;
  shi[t] = si;
  __syncthreads();
  for (int h = kTabThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      shr[t] += shr[t + h];
      shi[t] += shi[t + h];
    }
    __syncthreads();
  }
  if (t != 0) return;
  cplx<double> g;
  if (cls == kTab3Static) {
    double out = (z * z - fabs(z) * Lz) / (2.0 * Lx * Ly * Lz);
    const int kmax = static_cast<int>(ceil(kDecayD * Ly / (2.0 * kPiD * Lz))) + 2;
    for (int k = -kmax; k <= kmax; ++k)
      out -= log_layer_d(2.0 * kPiD * fabs(k * Lz + z) / Ly, 2.0 * kPiD * y / Ly) / (4.0 * kPiD * Lx);
    out += shr[0] / (kPiD * Lx) + Lz / (12.0 * Lx * Ly);
    g = cmake<double>(out, 0.0);
  } else if (cls == kTab2Static) {
    const double az = fabs(z);
    double out = -az / (2.0 * Lx * Ly) - log_layer_d(2.0 * kPiD * az / Ly, 2.0 * kPiD * y / Ly) / (4.0 * kPiD * Lx);
    g = cmake<double>(out + shr[0] / (kPiD * Lx), 0.0);
  } else if (cls == kTab1Static) {
    const double rho = sqrt(y * y + z * z);
    g = cmake<double>(-log(rho) / (2.0 * kPiD * Lx) + shr[0] / (kPiD * Lx), 0.0);
  } else if (cls == kTab1Dyn) {
    g = cmake<double>(shr[0] / (2.0 * kPiD * Lx), shi[0] / (2.0 * kPiD * Lx));
  } else {
    // divide by 2 j Lx Ly
    const double inv = 1.0 / (2.0 * Lx * Ly);
    g = cmake<double>(shi[0] * inv, -shr[0] * inv);
  }
  cplx<double> out = cmul(cexp_d(cmake<double>(barg.y, -barg.x)), g);
  // minus the near-zone images (unreduced offset)
  int lim[3];
  for (int c = 0; c < 3; ++c) lim[c] = c < a.dims ? a.id : 0;
  for (int ix = -lim[0]; ix <= lim[0]; ++ix)
    for (int iy = -lim[1]; iy <= lim[1]; ++iy)
      for (int iz = -lim[2]; iz <= lim[2]; ++iz) {
        const double R[3] = {ix * a.L[0], iy * a.L[1], iz * a.L[2]};
        const double ddx = r0[0] - R[0], ddy = r0[1] - R[1], ddz = r0[2] - R[2];
        const double dist = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
        // phase exp(-j kt . R) times exp(-j k0 dist) / (4 pi dist)
        cplx<double> ph = cscale(k0, dist);
        for (int c = 0; c < a.dims; ++c) ph = cadd(ph, cscale(kt[c], R[c]));
        out = csub(out, cscale(cexp_d(cmake<double>(ph.y, -ph.x)), 1.0 / (4.0 * kPiD * dist)));
      }
  table[e] = out;
}

int launch_far_table(const FarTableArgs& a, bool npsp, void* table, hipStream_t st) {
  int cls;
  if (a.dims == 3)
    cls = npsp ? kTab3Static : kTab3Dyn;
  else if (a.dims == 2)
    cls = kTab2Static;  // 2D with k0 or a phase: launch_far_table_pgf2
  else
    cls = npsp ? kTab1Static : kTab1Dyn;
  if (a.dims == 2 && !npsp) return FFTPIM_ERR_INVALID_ARG;
  const int64_t total = static_cast<int64_t>(2 * a.nf[0] - 1) * (2 * a.nf[1] - 1) * (2 * a.nf[2] - 1);
  hipLaunchKernelGGL(k_far_table, dim3(static_cast<unsigned>(total)), dim3(kTabThreads), 0, st, a, cls,
                     static_cast<cplx<double>*>(table));
  return FFTPIM_OK;
}

__global__ void k_far_circulant(const cplx<double>* __restrict__ table, int nf0, int nf1, int nf2, int M0, int M1,
                                int M2, cplx<double>* __restrict__ out) {
  const int64_t total = static_cast<int64_t>(M0) * M1 * M2;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int i2 = static_cast<int>(idx % M2);
  const int i1 = static_cast<int>((idx / M2) % M1);
  const int i0 = static_cast<int>(idx / (static_cast<int64_t>(M1) * M2));
  // index i holds offset i (i < nf) or i - M (the negative offsets)
  const int e0 = i0 < nf0 ? i0 : i0 - M0, e1 = i1 < nf1 ? i1 : i1 - M1, e2 = i2 < nf2 ? i2 : i2 - M2;
  cplx<double> v = cmake<double>(0.0, 0.0);
  if (e0 > -nf0 && e1 > -nf1 && e2 > -nf2)
    v = table[((static_cast<int64_t>(e0 + nf0 - 1) * (2 * nf1 - 1)) + e1 + nf1 - 1) * (2 * nf2 - 1) + e2 + nf2 - 1];
  out[idx] = v;
}

void launch_far_circulant(const void* table, const int nf[3], const int Mf[3], void* out, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(Mf[0]) * Mf[1] * Mf[2];
  hipLaunchKernelGGL(k_far_circulant, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, st,
                     static_cast<const cplx<double>*>(table), nf[0], nf[1], nf[2], Mf[0], Mf[1], Mf[2],
                     static_cast<cplx<double>*>(out));
}

}  // namespace fftpim
