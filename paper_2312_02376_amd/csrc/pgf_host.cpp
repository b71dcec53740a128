// Host FP64 evaluation of the periodic Green's function G^p (Sec. 2) for the
// far-zone kernel table (Sec. 3.2: the table of G^p_far at the offsets between
// the shifted observer and source grids, evaluated with the rapidly converging
// series of Eq. (pgf) and Eq. (lgf)).
//
// The far-grid offsets never vanish on any axis (the two grids are shifted by
// half a cell), so the series always have a non-vanishing transverse distance.
#include "pgf_host.h"

#include <algorithm>
#include <cmath>
#include <system_error>
#include <thread>
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

cd g0(double r, double k0) { return std::exp(cd(0.0, -k0 * r)) / (kFourPi * r); }

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

// Eq. (pgf_2), summed over the square |m|, |n| <= M with M set by the decay
// exp(-|k_t,mn| |z|) of the evanescent modes; |z| > 0.
cd pgf2(double x, double y, double z, double Lx, double Ly, double k0, double kx0, double ky0) {
  double az = std::fabs(z);
  double kreach = kDecay / az + std::fabs(k0) + std::fabs(kx0) + std::fabs(ky0);
  int mmax = static_cast<int>(std::ceil(kreach * Lx / (2.0 * kPi))) + 1;
  int nmax = static_cast<int>(std::ceil(kreach * Ly / (2.0 * kPi))) + 1;
  cd sum = 0.0;
  double A = Lx * Ly;
  for (int m = -mmax; m <= mmax; ++m) {
    double kx = kx0 + 2.0 * kPi * m / Lx;
    cd ex = std::exp(cd(0.0, -kx * x));
    cd part = 0.0;
    for (int n = -nmax; n <= nmax; ++n) {
      double ky = ky0 + 2.0 * kPi * n / Ly;
      cd kz = csqrt_im_nonpos(cd(k0 * k0 - kx * kx - ky * ky, 0.0));
      part += std::exp(cd(0.0, -1.0) * (ky * y + kz * az)) / kz;
    }
    sum += ex * part;
  }
  return sum / (cd(0.0, 2.0) * A);
}

// Eq. (pgf_3) with the z images summed in closed form; |z| <= Lz, |z| > 0.
cd pgf3(double x, double y, double z, const double L[3], double k0, const double kt[3]) {
  double az = std::fabs(z);
  double kreach = kDecay / az + std::fabs(k0) + std::fabs(kt[0]) + std::fabs(kt[1]);
  int mmax = static_cast<int>(std::ceil(kreach * L[0] / (2.0 * kPi))) + 1;
  int nmax = static_cast<int>(std::ceil(kreach * L[1] / (2.0 * kPi))) + 1;
  cd sum = 0.0;
  const cd mj(0.0, -1.0);
  for (int m = -mmax; m <= mmax; ++m) {
    double kx = kt[0] + 2.0 * kPi * m / L[0];
    for (int n = -nmax; n <= nmax; ++n) {
      double ky = kt[1] + 2.0 * kPi * n / L[1];
      cd kz = csqrt_im_nonpos(cd(k0 * k0 - kx * kx - ky * ky, 0.0));
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
    double t = lat.kt[c] * lat.L[c] / (2.0 * kPi);
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
      double kp[3] = {lat.kt[xr], lat.kt[yr], lat.kt[zr]};
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
  return cd(NAN, NAN);  // 1D Helmholtz is not provided by this evaluator
}

cd pgf(const Lattice& lat, const double r_in[3]) {
  double r[3] = {r_in[0], r_in[1], r_in[2]};
  double arg = 0.0;
  for (int c = 0; c < lat.dims; ++c) {
    double n = std::round(r[c] / lat.L[c]);
    r[c] -= n * lat.L[c];
    arg += lat.kt[c] * n * lat.L[c];
  }
  return std::exp(cd(0.0, -arg)) * pgf_reduced(lat, r);
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
        double ph = lat.kt[0] * R[0] + lat.kt[1] * R[1] + lat.kt[2] * R[2];
        out += std::exp(cd(0.0, -ph)) * g0(dist, lat.k0);
      }
  return out;
}

int check_supported(const Lattice& lat) {
  if (lat.dims == 1 && !lat.npsp()) return 1;
  if (lat.dims == 3 && !lat.npsp()) {
    bool any = false;
    for (int z = 0; z < 3; ++z)
      if (lateral_ok(lat, (z + 1) % 3, (z + 2) % 3)) any = true;
    if (!any) return 1;
  }
  return 0;
}

// Rayleigh-Wood anomalies (Sec. 2): a vanishing k_zmn (2D, 3D) or k_rho,m
// (1D), or for 3D a resonant z-image sum, 1 - exp(-j (k_zmn -+ k_z0) L_z) = 0.
bool wood_anomaly(const Lattice& lat) {
  if (lat.npsp() || lat.k0 == 0.0) return false;
  double scale = std::max(std::fabs(lat.k0), 2.0 * kPi / *std::max_element(lat.L, lat.L + lat.dims));
  double tol = 1e-3 * scale;
  int reach = 2 + static_cast<int>(std::ceil((std::fabs(lat.k0) + 10.0) *
                                             *std::max_element(lat.L, lat.L + 3) / (2 * kPi)));
  if (lat.dims == 1) {
    for (int m = -reach; m <= reach; ++m) {
      double kx = lat.kt[0] + 2 * kPi * m / lat.L[0];
      if (std::sqrt(std::fabs(lat.k0 * lat.k0 - kx * kx)) < tol) return true;
    }
    return false;
  }
  for (int z = (lat.dims == 3 ? 0 : 2); z < 3; ++z) {
    int a = (z + 1) % 3, b = (z + 2) % 3;
    for (int m = -reach; m <= reach; ++m)
      for (int n = -reach; n <= reach; ++n) {
        double kx = lat.kt[a] + 2 * kPi * m / lat.L[a];
        double ky = lat.kt[b] + 2 * kPi * n / lat.L[b];
        double kz2 = lat.k0 * lat.k0 - kx * kx - ky * ky;
        if (std::sqrt(std::fabs(kz2)) < tol) return true;
        if (lat.dims == 3 && kz2 > 0) {
          double kz = std::sqrt(kz2);
          for (int s = -1; s <= 1; s += 2) {
            double ph = (kz + s * lat.kt[z]) * lat.L[z] / (2 * kPi);
            if (std::fabs(ph - std::round(ph)) * 2 * kPi < 1e-3) return true;
          }
        }
      }
  }
  return false;
}

void far_table(const Lattice& lat, int i_d, const int nf[3], const double delta[3],
               std::vector<cd>& table) {
  const int sx = 2 * nf[0] - 1, sy = 2 * nf[1] - 1, sz = 2 * nf[2] - 1;
  const int64_t total = static_cast<int64_t>(sx) * sy * sz;
  table.assign(total, cd(0.0, 0.0));
  const unsigned nthreads = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
  auto work = [&](unsigned t) {
    for (int64_t e = t; e < total; e += nthreads) {
      int dz = static_cast<int>(e % sz);
      int dy = static_cast<int>((e / sz) % sy);
      int dx = static_cast<int>(e / (static_cast<int64_t>(sz) * sy));
      double r[3] = {(dx - (nf[0] - 1) - 0.5) * delta[0], (dy - (nf[1] - 1) - 0.5) * delta[1],
                     (dz - (nf[2] - 1) - 0.5) * delta[2]};
      table[e] = pgf(lat, r) - g_near(lat, r, i_d);
    }
  };
  std::vector<std::thread> pool;
  pool.reserve(nthreads);
  unsigned started = 0;
  for (; started < nthreads; ++started) {
    try {
      pool.emplace_back(work, started);
    } catch (const std::system_error&) {
      break;  // no more host threads: the calling thread takes the rest
    }
  }
  for (unsigned t = started; t < nthreads; ++t) work(t);
  for (auto& th : pool) th.join();
}

}  // namespace fftpim
