// FP64 table arithmetic for the translation operator of Eqs. (4)-(5).
#include <cmath>

#include "pie_internal.h"

namespace pie {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    // Newton iteration on P_n from the Tricomi-type initial guess
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pnm1 = (n == 1) ? 1.0 : p0;
      dp = n * (z * pn - pnm1) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pn = (n == 1) ? z : p1;
    double pnm1 = (n == 1) ? 1.0 : p0;
    dp = n * (z * pn - pnm1) / (z * z - 1.0);
    x[n - 1 - i] = z;  // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// k s^t h_t(z), z = k w, t = 0..tau.  Imaginary parts (from y_t) by the
// upward recurrence written for the scaled quantity, which stays finite as
// k -> 0 with s proportional to k:
//   u_{t+1} = (2t+1)(s/z) u_t - s^2 u_{t-1},  u_t = k s^t y_t(z).
// Real parts k s^t j_t(z): power series for z < 1, downward (Miller)
// recurrence otherwise, normalised by whichever of j_0 = sin z / z and
// j_1 = sin z / z^2 - cos z / z is larger in magnitude (their zeros
// interlace, so the normalisation never divides by a vanishing value:
// at z = n pi, where j_0 vanishes, j_1 = -cos z / z).
void scaled_hankel(double k, double s, double w, int tau, std::vector<double>& out) {
  out.assign(2 * (tau + 1), 0.0);
  const double z = k * w;
  const double r = s / (k * w);
  const double cz = std::cos(z), sz = std::sin(z);
  // imaginary parts
  double um = -cz / w;                          // k y_0
  double u = -r * cz / w - s * sz / w;          // k s y_1
  out[1] = um;
  if (tau >= 1) out[3] = u;
  for (int t = 1; t < tau; ++t) {
    double un = (2.0 * t + 1.0) * r * u - s * s * um;
    um = u;
    u = un;
    out[2 * (t + 1) + 1] = u;
  }
  // real parts
  if (z < 1.0) {
    double szt = 1.0;  // (s z)^t / (2t+1)!!
    for (int t = 0; t <= tau; ++t) {
      if (t > 0) szt *= (s * z) / (2.0 * t + 1.0);
      double term = 1.0, sum = 1.0;
      for (int m = 1; m < 40; ++m) {
        term *= -(z * z / 2.0) / (m * (2.0 * t + 2.0 * m + 1.0));
        sum += term;
        if (std::fabs(term) < 1e-18 * std::fabs(sum)) break;
      }
      out[2 * t] = k * szt * sum;
    }
  } else {
    int nstart = tau + 40 + (int)z;
    std::vector<double> j(nstart + 2, 0.0);
    j[nstart + 1] = 0.0;
    j[nstart] = 1e-300;
    for (int t = nstart; t >= 1; --t) {
      j[t - 1] = (2.0 * t + 1.0) / z * j[t] - j[t + 1];
      if (std::fabs(j[t - 1]) > 1e250) {  // rescale to avoid overflow
        for (int q = t - 1; q <= nstart + 1; ++q) j[q] *= 1e-250;
      }
    }
    const double j0 = sz / z, j1 = sz / (z * z) - cz / z;
    const double scale = std::fabs(j0) >= std::fabs(j1) ? j0 / j[0] : j1 / j[1];
    double st = 1.0;
    for (int t = 0; t <= tau; ++t) {
      out[2 * t] = k * st * j[t] * scale;
      st *= s;
    }
  }
}

}  // namespace pie
