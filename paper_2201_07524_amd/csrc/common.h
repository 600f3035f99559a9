// Shared device/host definitions of the NFFT-boosted Sinkhorn kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nfs {

constexpr int kBlock = 256;       // threads per workgroup for every kernel here
constexpr int kMaxDim = 3;

template <typename R>
struct cplx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return {a.x, -a.y}; }

// Kaiser-Bessel window in grid-cell units, normalized to psi(0) = 1:
//   psi(z) = (b m / sinh(b m)) * sinh(b sqrt(m^2 - z^2)) / (b sqrt(m^2 - z^2)),  |z| <= m,
// evaluated as cnorm * (exp(a - bm) - exp(-a - bm)) / a with a = b sqrt(m^2 - z^2)
// and cnorm = bm / (1 - exp(-2 bm)), so no intermediate exceeds 1.
struct WindowConst {
  double m2;     // m^2
  double b;      // pi (2 - 1/sigma)
  double bm;     // b m
  double cnorm;  // bm / (1 - exp(-2 bm))
  double edge;   // 2 cnorm exp(-bm): psi at the support edge
};

// Per-tap polynomial form of the FP32 window.  A point whose first tap lies at
// distance z0 = t - M (t in [0, 1)) from it has, at tap j, the window value
//   psi(z0 + j) = sum_k c[j][k] x^k,   x = 2 t - 1,
// a Chebyshev interpolant built on the host with poly_coef(m) coefficients:
// degree 7 for m >= 4 and degree 9 below (absolute error 4e-8 to 8e-8 for
// m = 2..8, the FP32 rounding level; degree 9 gains nothing measurable for
// m >= 4 and costs two more FMAs per window value).  Tap 2M lies outside
// the support except at t = 0 and is zero.  Rows hold kPolyCoef entries,
// zero past poly_coef(m).
constexpr int kMaxM = 8;
constexpr int kPolyCoef = 10;
__host__ __device__ constexpr int poly_coef(int m) { return m >= 4 ? 8 : kPolyCoef; }
struct WindowPoly {
  float c[2 * kMaxM + 1][kPolyCoef];
};
// FP64 grids: the same per-tap interpolants with kPolyCoef64 coefficients
// (degree 14; absolute error at most 1.6e-14 for m = 2..8 in FP64 Horner,
// the rounding level of the closed form).
constexpr int kPolyCoef64 = 15;
struct WindowPoly64 {
  double c[2 * kMaxM + 1][kPolyCoef64];
};

// Longest run of same-cell points that spreading and interpolation handle
// together (window values of a run stay in registers: G x d x (2m+1)).
template <typename R>
__host__ __device__ constexpr int run_length(int) {
  return sizeof(R) == 8 ? 2 : 4;
}

// Geometry of the oversampled grid and its bins (tiles).
struct Geom {
  int d;        // dimension
  int g;        // grid points per dimension (even)
  int N;        // bandwidth
  int M;        // window cutoff m
  int T;        // cells per tile side
  int E;        // LDS tile extent per side = T + 2M + 1
  int nt[3];    // tiles per dimension (nt[c] = ceil(g / T)), unused dims = 1
};

// Workgroups are dealt to the 8 XCDs round robin (workgroup b runs on XCD
// b mod 8), each XCD with its own L2.  xcd_block numbers the work items of a
// launch of G workgroups so that each XCD takes one contiguous block of them
// (the first G mod 8 blocks one longer): workgroup b gets item
// block(b mod 8) + b / 8.  Neighbouring items (adjacent pencils of a strided
// FFT pass, chunks of adjacent tiles) then share lines in one L2 instead of
// each XCD fetching every line.
constexpr int kXcds = 8;
__device__ __forceinline__ long xcd_block(long b, long G) {
  const long x = b % kXcds, k = b / kXcds, q = G / kXcds, r = G % kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// A chunk is a run of at most `chunk` sorted points of one problem that share
// one tile of that problem's grid.
struct Chunk {
  int tile;     // linear tile id within the problem's grid
  int start;    // first sorted point (index into the packed arrays)
  int count;    // points in the chunk
  int prob;     // problem index (0 for a single problem)
};

}  // namespace nfs
