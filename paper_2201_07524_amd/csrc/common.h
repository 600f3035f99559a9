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
};

template <typename R>
__device__ __forceinline__ R kb_psi(R z, R m2, R b, R bm, R cnorm) {
  const R t = m2 - z * z;
  if (t <= R(0)) return R(0);
  const R a = b * sqrt(t);
  if (a < R(1e-4)) return cnorm * R(2) * exp(-bm);
  return cnorm * (exp(a - bm) - exp(-a - bm)) / a;
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

// A chunk is a run of at most `chunk` sorted points of one problem that share
// one tile of that problem's grid.
struct Chunk {
  int tile;     // linear tile id within the problem's grid
  int start;    // first sorted point (index into the packed arrays)
  int count;    // points in the chunk
  int prob;     // problem index (0 for a single problem)
};

}  // namespace nfs
