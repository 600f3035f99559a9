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
  w.edge = 2.0 * w.cnorm * std::exp(-w.bm);
  return w;
}

// The window in cell units, FP64 (same normalization as the device forms).
inline double window_value(double z, const WindowConst& w) {
  const double t = w.m2 - z * z;
  if (t <= 0.0) return 0.0;
  const double a = w.b * std::sqrt(t);
  if (a < 1e-6) return w.edge;
  return w.cnorm * (std::exp(a - w.bm) - std::exp(-a - w.bm)) / a;
}

// Per-tap polynomials of the window (see WindowPoly, WindowPoly64): for tap
// j the function x -> psi(j - m + (x + 1)/2) on [-1, 1] is interpolated at K
// Chebyshev points, and the Chebyshev series is converted to monomial
// coefficients (in double, then rounded to T).  Rows j >= 2m stay zero.
template <typename T, int STRIDE>
inline void fit_window_poly(int m, int K, const WindowConst& w, T (&c)[2 * kMaxM + 1][STRIDE]) {
  constexpr int KM = 16;
  for (int j = 0; j < 2 * m; ++j) {
    double f[KM], a[KM];
    for (int i = 0; i < K; ++i) {
      const double xi = std::cos(kPi * (i + 0.5) / K);
      f[i] = window_value(double(j - m) + 0.5 * (xi + 1.0), w);
    }
    for (int k = 0; k < K; ++k) {  // Chebyshev coefficients
      double sum = 0.0;
      for (int i = 0; i < K; ++i) sum += f[i] * std::cos(kPi * k * (i + 0.5) / K);
      a[k] = (k == 0 ? 1.0 : 2.0) * sum / K;
    }
    // monomial coefficients: accumulate a_k T_k(x) with T_{k+1} = 2x T_k - T_{k-1}
    double mono[KM] = {0.0}, tkm1[KM] = {0.0}, tk[KM] = {0.0}, tkp1[KM];
    tkm1[0] = 1.0;  // T_0
    tk[1] = 1.0;    // T_1
    for (int q = 0; q < K; ++q) mono[q] += a[0] * tkm1[q];
    for (int q = 0; q < K; ++q) mono[q] += a[1] * tk[q];
    for (int k = 2; k < K; ++k) {
      for (int q = 0; q < K; ++q) tkp1[q] = (q > 0 ? 2.0 * tk[q - 1] : 0.0) - tkm1[q];
      for (int q = 0; q < K; ++q) mono[q] += a[k] * tkp1[q];
      for (int q = 0; q < K; ++q) {
        tkm1[q] = tk[q];
        tk[q] = tkp1[q];
      }
    }
    for (int q = 0; q < K; ++q) c[j][q] = T(mono[q]);  // entries K.. stay zero
  }
}

inline WindowPoly make_window_poly(int m, const WindowConst& w) {
  WindowPoly P{};
  fit_window_poly(m, poly_coef(m), w, P.c);
  return P;
}

inline WindowPoly64 make_window_poly64(int m, const WindowConst& w) {
  WindowPoly64 P{};
  fit_window_poly(m, kPolyCoef64, w, P.c);
  return P;
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
  // Centred form (r = 2): the x cloud is mapped as x + shift, the y cloud as
  // y - shift, with shift = (mean_nu y - mean_mu x)/2, so both clouds have the
  // same weighted mean; zero otherwise.
  double shift[3];
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
    s.scale = 0.0;  // r = 1: see choose_scaling_r1
  }
  return s;
}

// r = 1 (kernel exp(-|z|/eps)): the periodization error is exp(-(1 - 2 R s)/(eps s));
// keep it below exp(-L) (L = 20 for FP32 grids, 36 for FP64).
inline Scaling choose_scaling_r1(int d, double eps, double L, const double* lo, const double* hi) {
  Scaling s{};
  double R = 0.0;
  for (int c = 0; c < d; ++c) {
    s.center[c] = 0.5 * (lo[c] + hi[c]);
    R = std::max(R, 0.5 * (hi[c] - lo[c]));
  }
  s.scale = 1.0 / (2.0 * R + L * eps);
  s.eps_t = eps * s.scale;
  s.kernel_err = std::exp(-(1.0 - 2.0 * R * s.scale) / s.eps_t);
  return s;
}

// Real exponent rho in (1, 4] (kernel exp(-|z|^rho/eps)): the torus mapping as
// for r = 1 with the periodization error exp(-((1 - 2 R s)/s)^rho / eps) below
// exp(-L), so s = 1 / (2R + (L eps)^(1/rho)); eps_t = eps s^rho.
inline Scaling choose_scaling_rho(int d, double eps, double rho, double L, const double* lo, const double* hi) {
  Scaling s{};
  double R = 0.0;
  for (int c = 0; c < d; ++c) {
    s.center[c] = 0.5 * (lo[c] + hi[c]);
    R = std::max(R, 0.5 * (hi[c] - lo[c]));
  }
  s.scale = 1.0 / (2.0 * R + std::pow(L * eps, 1.0 / rho));
  s.eps_t = eps * std::pow(s.scale, rho);
  s.kernel_err = std::exp(-std::pow(1.0 - 2.0 * R * s.scale, rho) / s.eps_t);
  return s;
}

// Near-field regularization of K(r) = exp(-r/e) (r = |z| on the torus): inside
// r < eI the kernel is replaced by the even polynomial
//   K_R(r) = sum_{j<p} c_j (r/eI)^{2j},
// whose first p-1 derivatives match K at r = eI, so K_R is smooth at the origin
// and p-1 times differentiable at eI.  The difference K - K_R on r < eI is the
// near-field correction.  The p x p system is solved in long double.
// With a real exponent rho, K(r) = exp(-r^rho/e): its derivatives in u = r/eI at
// u = 1 come from the Taylor series of exp(h(t)), h(t) = -(eI^rho/e) (1 + t)^rho
// = -(eI^rho/e) sum_j binom(rho, j) t^j, truncated at degree p - 1.
// cost: the same for the cost-weighted kernel r^rho exp(-r^rho/e) (the primal
// cost's kernel), whose series is that of exp(h(t)) times eI^rho (1 + t)^rho.
inline std::vector<double> nearfield_poly(double e, double eI, int p, double rho = 1.0, bool cost = false) {
  std::vector<long double> A(size_t(p) * p, 0.0L), b(p);
  std::vector<long double> dk(p);  // d^q/du^q K at u = 1
  if (rho == 1.0 && !cost) {
    for (int q = 0; q < p; ++q) dk[q] = std::pow(-(long double)(eI / e), (long double)q) * std::exp(-(long double)(eI / e));
  } else {
    const long double a = std::pow((long double)eI, (long double)rho) / (long double)e;
    std::vector<long double> h(p, 0.0L), ex(p, 0.0L), term(p, 0.0L);
    long double bin = 1.0L;  // binom(rho, j)
    for (int j = 0; j < p; ++j) {
      h[j] = -a * bin;
      bin *= ((long double)rho - j) / (long double)(j + 1);
    }
    // exp(h0 + H(t)), H = h without its constant: exp(h0) sum_k H^k / k!
    term[0] = 1.0L;
    ex[0] = 1.0L;
    for (int k = 1; k < p; ++k) {
      std::vector<long double> nt(p, 0.0L);
      for (int i = 0; i < p; ++i)
        for (int j = 1; i + j < p; ++j) nt[i + j] += term[i] * h[j];
      for (int i = 0; i < p; ++i) {
        term[i] = nt[i] / (long double)k;
        ex[i] += term[i];
      }
    }
    if (cost) {  // times eI^rho (1 + t)^rho = -(e) h(t)
      std::vector<long double> prod(p, 0.0L);
      for (int i = 0; i < p; ++i)
        for (int j = 0; i + j < p; ++j) prod[i + j] += ex[i] * (-(long double)e * h[j]);
      ex = prod;
    }
    long double fact = 1.0L;
    for (int q = 0; q < p; ++q) {
      if (q > 0) fact *= q;
      dk[q] = std::exp(h[0]) * ex[q] * fact;
    }
  }
  for (int q = 0; q < p; ++q) {
    for (int j = 0; j < p; ++j) {
      if (2 * j >= q) {
        long double f = 1.0L;
        for (int t = 0; t < q; ++t) f *= (long double)(2 * j - t);
        A[size_t(q) * p + j] = f;
      }
    }
    b[q] = dk[q];
  }
  for (int c = 0; c < p; ++c) {  // Gaussian elimination with partial pivoting
    int piv = c;
    for (int r = c + 1; r < p; ++r)
      if (std::fabs(A[size_t(r) * p + c]) > std::fabs(A[size_t(piv) * p + c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < p; ++k) std::swap(A[size_t(c) * p + k], A[size_t(piv) * p + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < p; ++r) {
      const long double f = A[size_t(r) * p + c] / A[size_t(c) * p + c];
      for (int k = c; k < p; ++k) A[size_t(r) * p + k] -= f * A[size_t(c) * p + k];
      b[r] -= f * b[c];
    }
  }
  std::vector<double> cf(p);
  for (int r = p - 1; r >= 0; --r) {
    long double acc = b[r];
    for (int k = r + 1; k < p; ++k) acc -= A[size_t(r) * p + k] * (long double)cf[k];
    cf[r] = double(acc / A[size_t(r) * p + r]);
  }
  return cf;
}

inline std::vector<double> window_hat_table(int N, int m, int g, const WindowConst& w) {
  const int H = N / 2 + 1;
  std::vector<double> phi(H);
  for (int k = 0; k < H; ++k) phi[k] = window_hat(k, m, g, w);
  return phi;
}

}  // namespace nfs
