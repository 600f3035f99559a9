// Host-side check of the near-field regularization (Section 3.1): the even
// polynomial K_R(r) = sum_j c_j (r/eI)^(2j) returned by nfs::nearfield_poly
// must match the kernel and its first derivatives at r = eI, for
// K = exp(-r^rho/e) (rho = 1 and real rho) and for the primal cost's kernel
// r^rho exp(-r^rho/e).  Prints one line per case: value and derivative
// mismatches relative to the kernel's scale, by finite differences.
#include <cmath>
#include <cstdio>

#include "host_math.h"

int main() {
  const double e = 0.002, eI = 0.03;
  const int p = 8;
  const double rhos[] = {1.0, 1.5, 2.5, 3.0};
  for (double rho : rhos) {
    for (int cost = 0; cost < 2; ++cost) {
      const std::vector<double> cf = nfs::nearfield_poly(e, eI, p, rho, cost != 0);
      auto f = [&](double r) {
        const double k = std::exp(-std::pow(r, rho) / e);
        return cost ? std::pow(r, rho) * k : k;
      };
      auto P = [&](double r) {
        const double u2 = (r / eI) * (r / eI);
        double v = 0.0;
        for (int j = p - 1; j >= 0; --j) v = v * u2 + cf[j];
        return v;
      };
      const double h = 1e-4 * eI;
      const double scale = std::fabs(f(eI)) + 1e-300;
      const double d0 = std::fabs(P(eI) - f(eI)) / scale;
      const double d1 = std::fabs((P(eI + h) - P(eI - h)) - (f(eI + h) - f(eI - h))) / (2 * h) * eI / scale;
      const double d2 = std::fabs((P(eI + h) - 2 * P(eI) + P(eI - h)) - (f(eI + h) - 2 * f(eI) + f(eI - h))) /
                        (h * h) * eI * eI / scale;
      // evenness: P(-r) = P(r) by construction; smooth at 0 means finite P(0)
      std::printf("rho=%.2f cost=%d d0=%.3e d1=%.3e d2=%.3e p0=%.6e\n", rho, cost, d0, d1, d2, P(0.0));
    }
  }
  return 0;
}
