// Host FP64 evaluation of the periodic Green's function G^p (Sec. 2) with the
// rapidly converging series of Eq. (pgf) and Eq. (lgf) (valid away from the
// periodic axes / planes), the Rayleigh-Wood checks of a plan and the self
// coefficient lim_{r->0}[G^p - G0].  The far-zone table itself is evaluated on
// the device (kernels_table.hip, kernels_far.hip) with the same series; this
// evaluator is the library's reference for them and is exposed through
// fftpim_eval_pgf.
//
// Wavenumbers may be complex (a lossy k0, a complex phase shift; Sec. 2): the
// series are then their analytic continuation, with every square root taken
// with Im <= 0.
#include "pgf_host.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace fftpim {

namespace {
constexpr double kPi = 3.14159265358979323846;
constexpr double kFourPi = 4.0 * kPi;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kDecay = 41.0;  // terms below e^-41 ~ 1.6e-18 are dropped

cd csqrt_im_nonpos(cd w) {
  cd s = std::sqrt(w);  // principal branch: Re >= 0
  if (s.imag() > 0) s = -s;
  return s;
}

double log_layer(double a, double theta) {
  // ln(1 - 2 e^{-a} cos(theta) + e^{-2a}) without cancellation
  double e = std::expm1(-a);
  double s = std::sin(0.5 * theta);
  return std::log(e * e + 4.0 * std::exp(-a) * s * s);
}

// (1/(pi Lx)) sum_{m>=1} sum_{n, k} K0(2 m pi rho_nk / Lx) cos(2 m pi x / Lx),
// rho_nk = sqrt((n Ly + y)^2 + (k Lz + z)^2); k = 0 only when kz_images is false.
double k0_lattice_sum(double x, double y, double z, double Lx, double Ly, double Lz,
                      bool kz_images) {
  double out = 0.0;
  for (int m = 1;; ++m) {
    double cutoff = kDecay * Lx / (2.0 * kPi * m);
    bool any = false;
    double cx = std::cos(2.0 * m * kPi * x / Lx);
    int kmax = kz_images ? static_cast<int>(std::ceil(cutoff / Lz)) + 1 : 0;
    int nmax = static_cast<int>(std::ceil(cutoff / Ly)) + 1;
    for (int k = -kmax; k <= kmax; ++k) {
      double zz = kz_images ? k * Lz + z : z;
      if (std::fabs(zz) > cutoff) continue;
      for (int n = -nmax; n <= nmax; ++n) {
        double yy = n * Ly + y;
        double rho = std::sqrt(yy * yy + zz * zz);
        if (rho > cutoff) continue;
        any = true;
        out += bessel_k0(2.0 * m * kPi * rho / Lx) * cx;
      }
    }
    if (!any) break;
  }
  return out / (kPi * Lx);
}

}  // namespace

// K0 for real x > 0.  For x <= 2 the ascending series of DLMF 10.31.2,
//   K0(x) = -(ln(x/2) + gamma) I0(x) + sum_{k>=1} (x^2/4)^k / (k!)^2 H_k,
// with H_k the harmonic numbers; for x > 2 the integral DLMF 10.32.9,
//   K0(x) = int_0^inf exp(-x cosh t) dt,
// by the trapezoidal rule, which converges geometrically for this entire,
// rapidly decaying integrand (step min(1/4, 1/(2 sqrt x))).
double bessel_k0(double x) {
  if (x <= 2.0) {
    double t = 0.25 * x * x;
    double term = 1.0, i0 = 1.0, s = 0.0, hk = 0.0;
    for (int k = 1; k < 40; ++k) {
      term *= t / (static_cast<double>(k) * k);
      hk += 1.0 / k;
      i0 += term;
      s += term * hk;
      if (term < 1e-18 * i0) break;
    }
    return -(std::log(0.5 * x) + kEulerGamma) * i0 + s;
  }
  double tau = std::min(0.25, 0.5 / std::sqrt(x));
  double acc = 0.5;  // e^{-x cosh 0} scaled by e^{x}
  for (int j = 1; j < 10000; ++j) {
    double e = -x * (std::cosh(j * tau) - 1.0);
    if (e < -kDecay) break;
    acc += std::exp(e);
  }
  return tau * acc * std::exp(-x);
}

namespace {

// H0^(2)(z) = J0(z) - j Y0(z) for moderate |z| and small |Im z| (the Floquet
// terms of Eq. (pgf_1) next to the propagating modes).  J_n(z) comes from the
// backward recurrence J_{n-1} = (2n/z) J_n - J_{n+1} started well above |z|
// and normalised with J0 + 2 sum_k J_2k = 1 (Miller's algorithm; DLMF 10.6.1,
// 10.12.4); Y0 from Neumann's expansion
//   Y0(z) = (2/pi)(ln(z/2) + gamma) J0(z) - (4/pi) sum_{k>=1} (-1)^k J_2k(z)/k.
cd hankel2_0(cd z) {
  const double az = std::abs(z);
  const int start = 2 * static_cast<int>(0.5 * (1.5 * az + 40.0));
  cd f_up = 0.0, f = 1e-30;  // f_{k+1}, f_k
  cd S = 0.0, T = 0.0;
  for (int k = start; k >= 1; --k) {
    if ((k & 1) == 0) {
      const int h = k / 2;
      S += 2.0 * f;
      T += ((h & 1) ? -1.0 : 1.0) * f / static_cast<double>(h);
    }
    const cd f_down = (2.0 * k) / z * f - f_up;
    f_up = f;
    f = f_down;
    if (std::abs(f) > 1e250) {  // rescale; only ratios matter
      f *= 1e-250;
      f_up *= 1e-250;
      S *= 1e-250;
      T *= 1e-250;
    }
  }
  S += f;
  const cd j0 = f / S;
  const cd y0 = (2.0 / kPi) * (std::log(0.5 * z) + kEulerGamma) * j0 - (4.0 / kPi) * T / S;
  return j0 - cd(0.0, 1.0) * y0;
}

}  // namespace

// K0(w) for complex w, Re w >= 0, w != 0 (H0^(2)(z) = (2j/pi) K0(j z) turns
// the Hankel terms of Eq. (pgf_1) into K0 terms, DLMF 10.27.8):
//   |w| <= 2:   ascending series DLMF 10.31.2;
//   |w| >= 18:  Hankel's asymptotic expansion DLMF 10.40.2 (the smallest term
//               is about e^{-2|w|});
//   Re w >= 1.5: the integral DLMF 10.32.9 by the trapezoidal rule, with the
//               step set by the width pi/2 - |arg w| of the strip in which the
//               integrand stays bounded;
//   otherwise (close to the imaginary axis): K0(w) = -(j pi/2) H0^(2)(-j w)
//               with the Miller/Neumann Hankel function above.
cd bessel_k0c(cd w) {
  if (w.imag() == 0.0 && w.real() > 0.0) return bessel_k0(w.real());
  const double aw = std::abs(w);
  if (aw <= 2.0) {
    const cd t = 0.25 * w * w;
    cd term = 1.0, i0 = 1.0, s = 0.0;
    double hk = 0.0;
    for (int k = 1; k < 60; ++k) {
      term *= t / (static_cast<double>(k) * k);
      hk += 1.0 / k;
      i0 += term;
      s += term * hk;
      if (std::abs(term) < 1e-18 * std::abs(i0)) break;
    }
    return -(std::log(0.5 * w) + kEulerGamma) * i0 + s;
  }
  if (aw >= 18.0) {
    cd sum = 1.0, term = 1.0;
    for (int k = 1; k < 100; ++k) {
      const double a = 2.0 * k - 1.0;
      const cd next = term * (-(a * a) / (8.0 * k)) / w;
      if (std::abs(next) >= std::abs(term)) break;
      term = next;
      sum += term;
      if (std::abs(term) < 1e-17 * std::abs(sum)) break;
    }
    return std::sqrt(kPi / (2.0 * w)) * std::exp(-w) * sum;
  }
  if (w.real() >= 1.5) {
    const double theta = std::fabs(std::arg(w));
    const double d = std::min(0.25 * kPi, 0.5 * (0.5 * kPi - theta));
    const double tau = std::min(0.25, 2.0 * kPi * d / 40.0);
    cd acc = 0.5;  // e^{-w cosh t} scaled by e^{w}
    for (int j = 1; j < 1000000; ++j) {
      const double c1 = std::cosh(j * tau) - 1.0;
      if (w.real() * c1 > kDecay + 4.0) break;
      acc += std::exp(-w * c1);
    }
    return tau * acc * std::exp(-w);
  }
  return cd(0.0, -0.5 * kPi) * hankel2_0(cd(w.imag(), -w.real()));
}

cd g0(double r, cd k0) { return std::exp(cd(0.0, -1.0) * k0 * r) / (kFourPi * r); }

cd Lattice::phase(int ix, int iy, int iz) const {
  const cd a = kt[0] * (ix * L[0]) + kt[1] * (iy * L[1]) + kt[2] * (iz * L[2]);
  return std::exp(cd(0.0, -1.0) * a);
}

// Eq. (lgf_3) plus Lz/(12 Lx Ly) (zero cell mean); |z| <= Lz, y^2 + z^2 > 0.
double lgf3(double x, double y, double z, double Lx, double Ly, double Lz) {
  double out = (z * z - std::fabs(z) * Lz) / (2.0 * Lx * Ly * Lz);
  int kmax = static_cast<int>(std::ceil(kDecay * Ly / (2.0 * kPi * Lz))) + 2;
  for (int k = -kmax; k <= kmax; ++k) {
    double a = 2.0 * kPi * std::fabs(k * Lz + z) / Ly;
    out -= log_layer(a, 2.0 * kPi * y / Ly) / (4.0 * kPi * Lx);
  }
  out += k0_lattice_sum(x, y, z, Lx, Ly, Lz, true);
  return out + Lz / (12.0 * Lx * Ly);
}

// Eq. (lgf_2); y^2 + z^2 > 0.
double lgf2(double x, double y, double z, double Lx, double Ly) {
  double az = std::fabs(z);
  double out = -az / (2.0 * Lx * Ly);
  out -= log_layer(2.0 * kPi * az / Ly, 2.0 * kPi * y / Ly) / (4.0 * kPi * Lx);
  return out + k0_lattice_sum(x, y, z, Lx, Ly, 1.0, false);
}

// Eq. (lgf_1); rho > 0.
double lgf1(double x, double rho, double Lx) {
  double out = -std::log(rho) / (2.0 * kPi * Lx);
  for (int m = 1;; ++m) {
    double a = 2.0 * m * kPi * rho / Lx;
    if (a > kDecay) break;
    out += bessel_k0(a) * std::cos(2.0 * m * kPi * x / Lx) / (kPi * Lx);
  }
  return out;
}

// Eq. (pgf_1), with H0^(2)(z) = (2j/pi) K0(j z):
//   G = (1/(2 pi Lx)) sum_m e^{-j k_xm x} K0(j k_rho,m rho),
// k_rho,m = (k0^2 - k_xm^2)^{1/2} with Im <= 0, so Re(j k_rho,m rho) >= 0;
// rho > 0.  Terms beyond |k_xm| rho > 41 are below e^-41 and dropped.
cd pgf1(double x, double rho, double Lx, cd k0, cd kx0) {
  const double kreach = kDecay / rho + std::abs(k0) + std::abs(kx0);
  const int mmax = static_cast<int>(std::ceil(kreach * Lx / (2.0 * kPi))) + 1;
  cd sum = 0.0;
  for (int m = -mmax; m <= mmax; ++m) {
    const cd kx = kx0 + 2.0 * kPi * m / Lx;
    const cd krho = csqrt_im_nonpos(k0 * k0 - kx * kx);
    sum += std::exp(cd(0.0, -1.0) * kx * x) * bessel_k0c(cd(0.0, 1.0) * krho * rho);
  }
  return sum / (2.0 * kPi * Lx);
}

// Eq. (pgf_2), summed over the square |m|, |n| <= M with M set by the decay
// exp(-|k_t,mn| |z|) of the evanescent modes; |z| > 0.
cd pgf2(double x, double y, double z, double Lx, double Ly, cd k0, cd kx0, cd ky0) {
  double az = std::fabs(z);
  double kreach = kDecay / az + std::abs(k0) + std::abs(kx0) + std::abs(ky0);
  int mmax = static_cast<int>(std::ceil(kreach * Lx / (2.0 * kPi))) + 1;
  int nmax = static_cast<int>(std::ceil(kreach * Ly / (2.0 * kPi))) + 1;
  cd sum = 0.0;
  double A = Lx * Ly;
  const cd mj(0.0, -1.0);
  for (int m = -mmax; m <= mmax; ++m) {
    cd kx = kx0 + 2.0 * kPi * m / Lx;
    cd ex = std::exp(mj * kx * x);
    cd part = 0.0;
    for (int n = -nmax; n <= nmax; ++n) {
      cd ky = ky0 + 2.0 * kPi * n / Ly;
      cd kz = csqrt_im_nonpos(k0 * k0 - kx * kx - ky * ky);
      part += std::exp(mj * (ky * y + kz * az)) / kz;
    }
    sum += ex * part;
  }
  return sum / (cd(0.0, 2.0) * A);
}

// Eq. (pgf_3) with the z images summed in closed form; |z| <= Lz, |z| > 0.
cd pgf3(double x, double y, double z, const double L[3], cd k0, const cd kt[3]) {
  double az = std::fabs(z);
  double kreach = kDecay / az + std::abs(k0) + std::abs(kt[0]) + std::abs(kt[1]);
  int mmax = static_cast<int>(std::ceil(kreach * L[0] / (2.0 * kPi))) + 1;
  int nmax = static_cast<int>(std::ceil(kreach * L[1] / (2.0 * kPi))) + 1;
  cd sum = 0.0;
  const cd mj(0.0, -1.0);
  for (int m = -mmax; m <= mmax; ++m) {
    cd kx = kt[0] + 2.0 * kPi * m / L[0];
    for (int n = -nmax; n <= nmax; ++n) {
      cd ky = kt[1] + 2.0 * kPi * n / L[1];
      cd kz = csqrt_im_nonpos(k0 * k0 - kx * kx - ky * ky);
      cd am = std::exp(mj * (kz - kt[2]) * L[2]);
      cd ap = std::exp(mj * (kz + kt[2]) * L[2]);
      cd zpart = std::exp(mj * kz * az) + am * std::exp(mj * kz * z) / (1.0 - am) +
                 ap * std::exp(-mj * kz * z) / (1.0 - ap);
      sum += std::exp(mj * (kx * x + ky * y)) * zpart / kz;
    }
  }
  return sum / (cd(0.0, 2.0) * L[0] * L[1]);
}

namespace {

// A 3D axis permutation is usable for Eq. (pgf_3) when no lateral Floquet
// wavenumber vanishes together with k0 (static case), which would make a
// 0/0 term.
bool lateral_ok(const Lattice& lat, int a, int b) {
  if (lat.k0 != 0.0) return true;
  auto on_grid = [&](int c) {
    if (lat.kt[c].imag() != 0.0) return false;
    double t = lat.kt[c].real() * lat.L[c] / (2.0 * kPi);
    return std::fabs(t - std::round(t)) < 1e-12;
  };
  return !(on_grid(a) && on_grid(b));
}

}  // namespace

// G^p at a displacement already reduced into [-L/2, L/2] on the periodic axes.
cd pgf_reduced(const Lattice& lat, const double r[3]) {
  const double* L = lat.L;
  if (lat.dims == 3) {
    if (lat.npsp()) {
      int xr = 0;
      for (int c = 1; c < 3; ++c)
        if (std::fabs(r[c]) < std::fabs(r[xr])) xr = c;
      int yr = (xr + 1) % 3, zr = (xr + 2) % 3;
      return lgf3(r[xr], r[yr], r[zr], L[xr], L[yr], L[zr]);
    }
    int order[3] = {0, 1, 2};
    std::sort(order, order + 3, [&](int a, int b) { return std::fabs(r[a]) > std::fabs(r[b]); });
    for (int t = 0; t < 3; ++t) {
      int zr = order[t];
      int xr = (zr + 1) % 3, yr = (zr + 2) % 3;
      if (!lateral_ok(lat, xr, yr)) continue;
      double Lp[3] = {L[xr], L[yr], L[zr]};
      cd kp[3] = {lat.kt[xr], lat.kt[yr], lat.kt[zr]};
      return pgf3(r[xr], r[yr], r[zr], Lp, lat.k0, kp);
    }
    return cd(NAN, NAN);
  }
  if (lat.dims == 2) {
    if (lat.npsp()) {
      if (std::fabs(r[1]) < std::fabs(r[0])) return lgf2(r[1], r[0], r[2], L[1], L[0]);
      return lgf2(r[0], r[1], r[2], L[0], L[1]);
    }
    return pgf2(r[0], r[1], r[2], L[0], L[1], lat.k0, lat.kt[0], lat.kt[1]);
  }
  if (lat.npsp()) return lgf1(r[0], std::hypot(r[1], r[2]), L[0]);
  return pgf1(r[0], std::hypot(r[1], r[2]), L[0], lat.k0, lat.kt[0]);
}

cd pgf(const Lattice& lat, const double r_in[3]) {
  double r[3] = {r_in[0], r_in[1], r_in[2]};
  int n[3] = {0, 0, 0};
  for (int c = 0; c < lat.dims; ++c) {
    n[c] = static_cast<int>(std::round(r[c] / lat.L[c]));
    r[c] -= n[c] * lat.L[c];
  }
  return lat.phase(n[0], n[1], n[2]) * pgf_reduced(lat, r);
}

cd g_near(const Lattice& lat, const double r[3], int i_d) {
  cd out = 0.0;
  int lim[3];
  for (int c = 0; c < 3; ++c) lim[c] = c < lat.dims ? i_d : 0;
  for (int ix = -lim[0]; ix <= lim[0]; ++ix)
    for (int iy = -lim[1]; iy <= lim[1]; ++iy)
      for (int iz = -lim[2]; iz <= lim[2]; ++iz) {
        double R[3] = {ix * lat.L[0], iy * lat.L[1], iz * lat.L[2]};
        double d[3] = {r[0] - R[0], r[1] - R[1], r[2] - R[2]};
        double dist = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        out += lat.phase(ix, iy, iz) * g0(dist, lat.k0);
      }
  return out;
}

int check_supported(const Lattice& lat) {
  if (lat.dims == 3 && !lat.npsp()) {
    bool any = false;
    for (int z = 0; z < 3; ++z)
      if (lateral_ok(lat, (z + 1) % 3, (z + 2) % 3)) any = true;
    if (!any) return 1;
  }
  return 0;
}

// Rayleigh-Wood anomalies (Sec. 2): a vanishing k_zmn (2D, 3D) or k_rho,m
// (1D) with k0 != 0, or for 3D a resonant z-image sum,
// 1 - exp(-j (k_zmn -+ k_z0) L_z) = 0 (checked for every axis role the
// evaluator may use).
bool wood_anomaly(const Lattice& lat) {
  if (lat.npsp()) return false;
  const double Lmax = *std::max_element(lat.L, lat.L + lat.dims);
  double scale = std::max(std::abs(lat.k0), 2.0 * kPi / Lmax);
  double tol = 1e-3 * scale;
  double kmax = std::abs(lat.k0);
  for (int c = 0; c < lat.dims; ++c) kmax = std::max(kmax, std::abs(lat.kt[c]));
  int reach = 2 + static_cast<int>(std::ceil((kmax + 10.0) * *std::max_element(lat.L, lat.L + 3) / (2 * kPi)));
  const bool dyn = lat.k0 != 0.0;
  if (lat.dims == 1) {
    if (!dyn) return false;
    for (int m = -reach; m <= reach; ++m) {
      cd kx = lat.kt[0] + 2 * kPi * m / lat.L[0];
      if (std::sqrt(std::abs(lat.k0 * lat.k0 - kx * kx)) < tol) return true;
    }
    return false;
  }
  for (int z = (lat.dims == 3 ? 0 : 2); z < 3; ++z) {
    int a = (z + 1) % 3, b = (z + 2) % 3;
    if (lat.dims == 3 && !lateral_ok(lat, a, b)) continue;
    for (int m = -reach; m <= reach; ++m)
      for (int n = -reach; n <= reach; ++n) {
        cd kx = lat.kt[a] + 2 * kPi * m / lat.L[a];
        cd ky = lat.kt[b] + 2 * kPi * n / lat.L[b];
        cd kz2 = lat.k0 * lat.k0 - kx * kx - ky * ky;
        if (dyn && std::sqrt(std::abs(kz2)) < tol) return true;
        if (lat.dims == 3 && std::abs(kz2) > 0.0) {
          cd kz = csqrt_im_nonpos(kz2);
          for (int s = -1; s <= 1; s += 2) {
            cd e = std::exp(cd(0.0, -1.0) * (kz + static_cast<double>(s) * lat.kt[z]) * lat.L[z]);
            if (std::abs(1.0 - e) < 1e-3) return true;
          }
        }
      }
  }
  return false;
}

namespace {

// erfc(z) for Re z >= 0.  |z| <= 3 (or close to the imaginary axis): the
// Maclaurin series of erf (DLMF 7.6.1) in extended precision, whose terms
// grow to about e^{|z|^2}; otherwise Laplace's continued fraction
// (DLMF 7.9.2), evaluated from depth 120 upwards.
cd erfc_c(cd z) {
  const double az = std::abs(z);
  if (az <= 3.0 || z.real() < 0.5) {
    using cl = std::complex<long double>;
    const cl zz(z.real(), z.imag());
    const cl z2 = zz * zz;
    cl term = zz, sum = zz;
    for (int n = 1; n < 400; ++n) {
      term *= -z2 / static_cast<long double>(n);
      const cl t = term / static_cast<long double>(2 * n + 1);
      sum += t;
      if (n > 4 && std::abs(t) < 1e-22L * std::max<long double>(1.0L, std::abs(sum))) break;
    }
    const cl r = 1.0L - sum * (2.0L / std::sqrt(3.14159265358979323846264338327950288L));
    return cd(static_cast<double>(r.real()), static_cast<double>(r.imag()));
  }
  cd t = z;
  for (int k = 120; k >= 1; --k) t = z + (0.5 * k) / t;
  return std::exp(-z * z) / (std::sqrt(kPi) * t);
}

// E1(z) on the principal branch; on the negative real axis the value reached
// from above.  |z| <= 4 or Re z < 0: the series DLMF 6.6.2,
//   E1(z) = -gamma - ln z - sum_{k>=1} (-z)^k / (k k!),
// in extended precision; otherwise the continued fraction DLMF 6.9.1,
//   E1(z) = e^{-z} / (z + 1 - 1/(z + 3 - 4/(z + 5 - 9/(z + 7 - ...)))).
cd expint1_c(cd z) {
  if (std::abs(z) <= 4.0 || z.real() < 0.0) {
    using cl = std::complex<long double>;
    const cl zz(z.real(), z.imag());
    cl term = 1.0L, sum = 0.0L;
    for (int k = 1; k < 400; ++k) {
      term *= -zz / static_cast<long double>(k);
      const cl t = term / static_cast<long double>(k);
      sum += t;
      if (k > 4 && std::abs(t) < 1e-22L * std::max<long double>(1.0L, std::abs(sum))) break;
    }
    cd lnz = (z.imag() == 0.0 && z.real() < 0.0) ? cd(std::log(-z.real()), kPi) : std::log(z);
    const cd s2(static_cast<double>(sum.real()), static_cast<double>(sum.imag()));
    return -kEulerGamma - lnz - s2;
  }
  cd t = z + 241.0;
  for (int i = 120; i >= 1; --i) t = z + (2.0 * i - 1.0) - static_cast<double>(i) * i / t;
  return std::exp(-z) / t;
}

}  // namespace

// lim_{r -> 0} [G^p(r) - G0(r)]: the images of a source seen at its own
// position (the n = m coefficient of Eq. (1) without the singular image).
// The paper's series do not converge at r = 0; this uses the Ewald splitting
// of G^p at r = 0 with a splitting parameter E large enough (E L_min >= 6.8)
// that every real-space term but the regularised zeroth one is below e^-46:
//   C = S_0 + (spectral part at r = 0),
//   S_0 = [2 j k0 erfc(j k0 / 2E) - (4E/sqrt(pi)) e^{k0^2/4E^2}] / (8 pi),
//   3D: (1/V) sum_G e^{-(kG.kG - k0^2)/4E^2} / (kG.kG - k0^2);
//       neutral static: G = 0 dropped and -1/(4 E^2 V) added (zero cell mean);
//   2D: sum_mn erfc(j kz / 2E) / (2 j A kz), kz with Im <= 0;
//       neutral static: the (0,0) term is -1/(2 A sqrt(pi) E) (the gauge of
//       Eq. (lgf_2));
//   1D: (1/(4 pi L)) sum_m E1(-k_rho,m^2 / 4E^2);
//       neutral static: (gamma - ln 2L)/(2 pi L) in the gauge of Eq. (lgf_1).
cd pgf_self(const Lattice& lat) {
  const int d = lat.dims;
  const double* L = lat.L;
  if (lat.npsp() && d == 1) return (kEulerGamma - std::log(2.0 * L[0])) / (2.0 * kPi * L[0]);
  double Lmin = L[0], Lmax = L[0];
  for (int c = 1; c < d; ++c) {
    Lmin = std::min(Lmin, L[c]);
    Lmax = std::max(Lmax, L[c]);
  }
  double grow = std::fabs(lat.k0.imag());
  for (int c = 0; c < d; ++c) grow += std::fabs(lat.kt[c].imag());
  double E = std::sqrt(46.0 + grow * Lmax) / Lmin;
  E = std::max(E, std::abs(lat.k0) / 6.0);
  const cd j(0.0, 1.0);
  const cd k0 = lat.k0, k02 = k0 * k0;
  const double e2 = 4.0 * E * E;
  cd out = (2.0 * j * k0 * erfc_c(j * k0 / (2.0 * E)) - (4.0 * E / std::sqrt(kPi)) * std::exp(k02 / e2)) /
           (8.0 * kPi);
  double kt_abs = 0.0;
  for (int c = 0; c < d; ++c) kt_abs = std::max(kt_abs, std::abs(lat.kt[c]));
  const double kmax = std::sqrt(e2 * 46.0 + std::max(0.0, k02.real())) + kt_abs;
  int mm[3] = {0, 0, 0};
  for (int c = 0; c < d; ++c) mm[c] = static_cast<int>(std::ceil(kmax * L[c] / (2.0 * kPi))) + 1;
  if (d == 3) {
    const double V = L[0] * L[1] * L[2];
    cd acc = 0.0;
    for (int m = -mm[0]; m <= mm[0]; ++m)
      for (int n = -mm[1]; n <= mm[1]; ++n)
        for (int q = -mm[2]; q <= mm[2]; ++q) {
          if (lat.npsp() && m == 0 && n == 0 && q == 0) continue;
          const cd kx = lat.kt[0] + 2.0 * kPi * m / L[0];
          const cd ky = lat.kt[1] + 2.0 * kPi * n / L[1];
          const cd kz = lat.kt[2] + 2.0 * kPi * q / L[2];
          const cd den = kx * kx + ky * ky + kz * kz - k02;
          acc += std::exp(-den / e2) / den;
        }
    out += acc / V;
    if (lat.npsp()) out -= 1.0 / (e2 * V);
  } else if (d == 2) {
    const double A = L[0] * L[1];
    cd acc = 0.0;
    for (int m = -mm[0]; m <= mm[0]; ++m)
      for (int n = -mm[1]; n <= mm[1]; ++n) {
        if (lat.npsp() && m == 0 && n == 0) {
          out -= 1.0 / (2.0 * A * std::sqrt(kPi) * E);
          continue;
        }
        const cd kx = lat.kt[0] + 2.0 * kPi * m / L[0];
        const cd ky = lat.kt[1] + 2.0 * kPi * n / L[1];
        const cd kz = csqrt_im_nonpos(k02 - kx * kx - ky * ky);
        acc += erfc_c(j * kz / (2.0 * E)) / kz;
      }
    out += acc / (2.0 * j * A);
  } else {
    cd acc = 0.0;
    for (int m = -mm[0]; m <= mm[0]; ++m) {
      const cd kx = lat.kt[0] + 2.0 * kPi * m / L[0];
      acc += expint1_c(-(k02 - kx * kx) / e2);
    }
    out += acc / (4.0 * kPi * L[0]);
  }
  return out;
}

}  // namespace fftpim
