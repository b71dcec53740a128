// Host FP64 periodic Green's function (Sec. 2, Eq. (pgf) and Eq. (lgf)): the
// library's own evaluator of G^p (exposed through fftpim_eval_pgf), the
// Rayleigh-Wood checks of a plan, and the self coefficient of Eq. (5).
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace fftpim {

using cd = std::complex<double>;

struct Lattice {
  int dims;       // periodic axes: x (1), x,y (2), x,y,z (3)
  double L[3];    // periods
  cd k0;          // free-space wavenumber (Im <= 0)
  cd kt[3];       // phase-shift wavenumbers (possibly complex, Sec. 2)
  bool npsp() const { return k0 == 0.0 && kt[0] == 0.0 && kt[1] == 0.0 && kt[2] == 0.0; }
  // the correction operator is Hermitian only for a real static kernel with
  // a real phase shift
  bool hermitian() const {
    return k0 == 0.0 && kt[0].imag() == 0.0 && kt[1].imag() == 0.0 && kt[2].imag() == 0.0;
  }
  // phase exp(-j k_t . R) of the image i (integer offsets on the periodic axes)
  cd phase(int ix, int iy, int iz) const;
};

double bessel_k0(double x);
// K0(w) for complex w with Re w >= 0, w != 0.
cd bessel_k0c(cd w);
cd g0(double r, cd k0);
double lgf3(double x, double y, double z, double Lx, double Ly, double Lz);
double lgf2(double x, double y, double z, double Lx, double Ly);
double lgf1(double x, double rho, double Lx);
cd pgf1(double x, double rho, double Lx, cd k0, cd kx0);
cd pgf2(double x, double y, double z, double Lx, double Ly, cd k0, cd kx0, cd ky0);
cd pgf3(double x, double y, double z, const double L[3], cd k0, const cd kt[3]);
cd pgf_reduced(const Lattice& lat, const double r[3]);
// Full G^p (Bloch factor included); r must not be a lattice vector.
cd pgf(const Lattice& lat, const double r[3]);
// lim_{r->0} [G^p(r) - G0(r)] (the images of a point acting on itself).
cd pgf_self(const Lattice& lat);
// Eq. (4): images |i_c| <= i_d on the periodic axes.
cd g_near(const Lattice& lat, const double r[3], int i_d);
// Nonzero when this evaluator does not cover the problem class.
int check_supported(const Lattice& lat);
bool wood_anomaly(const Lattice& lat);
}  // namespace fftpim
