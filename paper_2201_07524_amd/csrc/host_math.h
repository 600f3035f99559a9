// Host-side FP64 setup of fast summation: the Kaiser-Bessel window and its
// Fourier transform, the torus scaling of the point clouds, the Fourier
// coefficients b_k of the regularized kernel and the fused diagonal tables.
#pragma once

#include <cmath>
#include <vector>

#include "common.h"

namespace nfs {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Modified Bessel function I_0 by its power series sum_j ((x/2)^j / j!)^2
// (all terms positive, so the partial sums are accurate in FP64).
inline double bessel_i0(double x) {
  const double h = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int j = 1; j < 500; ++j) {
    term *= h / (double(j) * double(j));
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

// Window shape parameter b = pi (2 - 1/sigma_eff) for oversampling sigma_eff = g/N.
inline WindowConst make_window(int m, int g, int N) {
  WindowConst w;
  const double sig = double(g) / double(N);
  w.b = kPi * (2.0 - 1.0 / sig);
  w.m2 = double(m) * double(m);
  w.bm = w.b * m;
  w.cnorm = w.bm / (1.0 - std::exp(-2.0 * w.bm));
  return w;
}

// Phi(k) = sum_l psi(l - u) exp(-2 pi i k l / g) exp(2 pi i k u / g) up to aliasing,
// i.e. the continuous Fourier transform of the cell-unit window psi at frequency k/g:
//   Phi(k) = pi m I_0(m sqrt(b^2 - (2 pi k / g)^2)) / sinh(b m).
inline double window_hat(int k, int m, int g, const WindowConst& w) {
  const double om = 2.0 * kPi * double(k) / double(g);
  const double arg = w.b * w.b - om * om;
  const double i0 = arg > 0.0 ? bessel_i0(double(m) * std::sqrt(arg)) : 1.0;
  // pi m / sinh(bm) computed as 2 pi m exp(-bm) / (1 - exp(-2bm))
  return 2.0 * kPi * m * std::exp(-w.bm) / (1.0 - std::exp(-2.0 * w.bm)) * i0;
}

// Torus mapping: torus coordinate = scale * (x - center), chosen so that for
// r = 2 both the periodization error exp(-(1 - 2 R s)^2 / (eps s^2)) and the
// truncation of the Gaussian's Fourier series at |k| = N/2,
// exp(-pi^2 eps s^2 N^2 / 4), stay below exp(-40) when possible (otherwise
// they are balanced).  R is the half extent of the common bounding box.
struct Scaling {
  double center[3];
  double scale;
  double eps_t;       // temperature in torus units (eps * scale^r)
  double kernel_err;  // a-priori kernel approximation error estimate
};

inline Scaling choose_scaling(int d, int r, double eps, int N, const double* lo, const double* hi) {
  Scaling s{};
  double R = 0.0;
  for (int c = 0; c < 3; ++c) s.center[c] = 0.0;
  for (int c = 0; c < d; ++c) {
    s.center[c] = 0.5 * (lo[c] + hi[c]);
    R = std::max(R, 0.5 * (hi[c] - lo[c]));
  }
  const double L = 40.0;
  if (r == 2) {
    double sc = 1.0 / (2.0 * R + std::sqrt(L * eps));
    const double trunc = kPi * kPi * eps * sc * sc * double(N) * N / 4.0;
    if (trunc < L) {
      const double a = kPi * eps * N / 2.0;
      sc = (-2.0 * R + std::sqrt(4.0 * R * R + 4.0 * a)) / (2.0 * a);
    }
    s.scale = sc;
    s.eps_t = eps * sc * sc;
    const double per = (1.0 - 2.0 * R * sc) * (1.0 - 2.0 * R * sc) / s.eps_t;
    const double tr = kPi * kPi * s.eps_t * double(N) * N / 4.0;
    s.kernel_err = std::exp(-std::min(per, tr));
  } else {
    s.scale = 0.0;  // r = 1 is set up by the near-field planner
  }
  return s;
}

// Tables of the fused diagonal over |k_c| = 0..N/2 per axis (extent H = N/2+1,
// row-major).  With the periodized Gaussian of temperature eps_t (period 1),
// whose Fourier coefficient is prod_c sqrt(pi eps_t) exp(-pi^2 eps_t k_c^2)
// (Poisson summation), and the window transform Phi:
//   kernel: D(k) = prod_c f(k_c),  f(k) = sqrt(pi eps_t) exp(-pi^2 eps_t k^2) hw(k) / Phi(k)^2
//   cost:   C(k) = D(k) (d eps_t / 2 - pi^2 eps_t^2 |k|^2) / scale^2
//           (the coefficients of |z|^2 exp(-|z|^2/eps_t), back in the caller's units)
// hw = 1/2 on |k_c| = N/2: the symmetric form of the real part of the sum over I_N.
struct DiagTables {
  std::vector<double> kernel, cost;
};

inline std::vector<double> window_hat_table(int N, int m, int g, const WindowConst& w) {
  const int H = N / 2 + 1;
  std::vector<double> phi(H);
  for (int k = 0; k < H; ++k) phi[k] = window_hat(k, m, g, w);
  return phi;
}

inline DiagTables gauss_tables(int d, int N, double eps_t, double scale, const std::vector<double>& phi) {
  const int H = N / 2 + 1;
  std::vector<double> f(H);
  for (int k = 0; k < H; ++k) {
    f[k] = std::sqrt(kPi * eps_t) * std::exp(-kPi * kPi * eps_t * double(k) * k) / (phi[k] * phi[k]);
    if (k == N / 2) f[k] *= 0.5;
  }
  long total = 1;
  for (int c = 0; c < d; ++c) total *= H;
  DiagTables t;
  t.kernel.resize(total);
  t.cost.resize(total);
  const double inv_s2 = 1.0 / (scale * scale);
  for (long i = 0; i < total; ++i) {
    long rem = i;
    double prod = 1.0, k2 = 0.0;
    for (int c = d - 1; c >= 0; --c) {
      const int kc = int(rem % H);
      rem /= H;
      prod *= f[kc];
      k2 += double(kc) * kc;
    }
    t.kernel[i] = prod;
    t.cost[i] = prod * (0.5 * d * eps_t - kPi * kPi * eps_t * eps_t * k2) * inv_s2;
  }
  return t;
}

}  // namespace nfs
