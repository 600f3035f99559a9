/*
 * Matrix-free FP64 kernel sums for the oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Plain C with OpenMP.  For clouds too large for a dense Gibbs kernel this
 * evaluates, for selected targets i, the sums of the Sinkhorn matrix-vector
 * product (Section 3.1, eqs. (matexp)/(matexpt)):
 *
 *     out_i = sum_j w_j exp(-|x_i - y_j|^r / eps)
 *
 * and the position-gradient sums of the transport plan, sum_j w_j k_ij
 * grad_x c(x_i, y_j), straight from their definitions, one exp per pair, in
 * double precision with plain sequential summation over j.
 * Points are point-major: x[i*d + c].
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

static double pair_cost(const double* a, const double* b, int d, int r) {
  double s = 0.0;
  for (int c = 0; c < d; ++c) {
    double t = a[c] - b[c];
    s += t * t;
  }
  return r == 2 ? s : sqrt(s);
}

/* out[q] = sum_j w[j] exp(-c(tgt[rows[q]], src[j]) / eps), q < nrows.
 * rows == NULL selects targets 0..nrows-1. */
void oracle_kv_rows(int d, int r, double eps,
                    const double* tgt, const int64_t* rows, int64_t nrows,
                    const double* src, int64_t ns, const double* w,
                    double* out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < nrows; ++q) {
    const int64_t i = rows ? rows[q] : q;
    const double* xi = tgt + i * d;
    double acc = 0.0;
    for (int64_t j = 0; j < ns; ++j) acc += w[j] * exp(-pair_cost(xi, src + j * d, d, r) / eps);
    out[q] = acc;
  }
}

/* The same sums for a real exponent rho of the distance (Definition 2.1 with
 * the cost |x - y|^rho): out[q] = sum_j w[j] exp(-|x_i - y_j|^rho / eps). */
void oracle_kv_rows_real(int d, double rho, double eps,
                         const double* tgt, const int64_t* rows, int64_t nrows,
                         const double* src, int64_t ns, const double* w,
                         double* out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < nrows; ++q) {
    const int64_t i = rows ? rows[q] : q;
    const double* xi = tgt + i * d;
    double acc = 0.0;
    for (int64_t j = 0; j < ns; ++j) acc += w[j] * exp(-pow(pair_cost(xi, src + j * d, d, 1), rho) / eps);
    out[q] = acc;
  }
}

/* g[q*d + c] = sum_j w[j] k(x_i, y_j) d c(x_i, y_j)/d x_i[c] for i = rows[q]:
 * r = 2: 2 (x_i - y_j); r = 1: (x_i - y_j)/|x_i - y_j| (zero when equal). */
void oracle_grad_rows(int d, int r, double eps,
                      const double* tgt, const int64_t* rows, int64_t nrows,
                      const double* src, int64_t ns, const double* w,
                      double* g) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < nrows; ++q) {
    const int64_t i = rows ? rows[q] : q;
    const double* xi = tgt + i * d;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < ns; ++j) {
      const double* yj = src + j * d;
      double c2 = 0.0;
      for (int c = 0; c < d; ++c) c2 += (xi[c] - yj[c]) * (xi[c] - yj[c]);
      const double dist = sqrt(c2);
      const double cost = r == 2 ? c2 : dist;
      const double kw = w[j] * exp(-cost / eps);
      for (int c = 0; c < d; ++c) {
        double gc;
        if (r == 2) gc = 2.0 * (xi[c] - yj[c]);
        else gc = dist > 0.0 ? (xi[c] - yj[c]) / dist : 0.0;
        acc[c] += kw * gc;
      }
    }
    for (int c = 0; c < d; ++c) g[q * d + c] = acc[c];
  }
}

int oracle_num_threads(void) {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
}
