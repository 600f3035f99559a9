// Spreading (adjoint NFFT, first step) and interpolation (NFFT, last step) of
// fast summation (Section 3.1, eq. (fastsum)) on gfx950.
//
// Points arrive sorted by tile (a T^d block of grid cells) and are processed
// in chunks of at most `chunk` points per workgroup.  Each workgroup works on
// an LDS copy of its tile plus a halo of m+1 / m cells per side:
//   spread:  accumulate w_j * psi(l - u_j) into LDS with ds_add, then flush the
//            tile to the global grid with global float atomics;
//   interp:  load the tile from the grid once (coalesced), then gather
//            t_i = sum_l grid_l psi(u_i - l) from LDS, and run the epilogue
//            (plain output, Sinkhorn scaling update, or residual evaluation)
//            with FP64 block reductions.
// One lane handles one point; its 2m+1 window values per dimension stay in
// registers.
#include "common.h"
#include "kernels.h"

namespace nfs {

template <typename R, int D, int M>
struct Taps {
  static constexpr int W = 2 * M + 1;
  R psi[D][W];
  int off[D];

  __device__ __forceinline__ void compute(const R* u, const WindowConst& wc) {
    const R m2 = R(wc.m2), b = R(wc.b), bm = R(wc.bm), cn = R(wc.cnorm);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const R s = ceil(u[c] - R(M));
      off[c] = int(s) + M;
      const R z0 = s - u[c];
#pragma unroll
      for (int j = 0; j < W; ++j) psi[c][j] = kb_psi(z0 + R(j), m2, b, bm, cn);
    }
  }
};

__device__ __forceinline__ int wrap(int v, int g) {
  v %= g;
  return v < 0 ? v + g : v;
}

// --------------------------------------------------------------------------- spread
template <typename R, int D, int M>
__global__ __launch_bounds__(kBlock) void spread_kernel(SpreadArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* tile = reinterpret_cast<R*>(smem_raw);
  constexpr int W = 2 * M + 1;
  const Geom geo = a.geo;
  const int E = geo.E;
  const int ncell = D == 1 ? E : (D == 2 ? E * E : E * E * E);
  const Chunk ch = a.chunks[blockIdx.x];

  for (int i = threadIdx.x; i < ncell; i += kBlock) tile[i] = R(0);
  __syncthreads();

  const double wm = a.wconst * (a.wmul ? *a.wmul : 1.0);
  for (int q = ch.start + threadIdx.x; q < ch.start + ch.count; q += kBlock) {
    const R w = R(a.w[q] * wm);
    if (w == R(0)) continue;
    R u[D];
#pragma unroll
    for (int c = 0; c < D; ++c) u[c] = a.coords[size_t(q) * D + c];
    Taps<R, D, M> tp;
    tp.compute(u, a.win);
    if constexpr (D == 1) {
#pragma unroll
      for (int j = 0; j < W; ++j) atomicAdd(&tile[tp.off[0] + j], w * tp.psi[0][j]);
    } else if constexpr (D == 2) {
#pragma unroll
      for (int j0 = 0; j0 < W; ++j0) {
        const R v0 = w * tp.psi[0][j0];
        R* row = tile + (tp.off[0] + j0) * E + tp.off[1];
#pragma unroll
        for (int j1 = 0; j1 < W; ++j1) atomicAdd(&row[j1], v0 * tp.psi[1][j1]);
      }
    } else {
      for (int j0 = 0; j0 < W; ++j0) {
        const R v0 = w * tp.psi[0][j0];
#pragma unroll 1
        for (int j1 = 0; j1 < W; ++j1) {
          const R v1 = v0 * tp.psi[1][j1];
          R* row = tile + ((tp.off[0] + j0) * E + tp.off[1] + j1) * E + tp.off[2];
#pragma unroll
          for (int j2 = 0; j2 < W; ++j2) atomicAdd(&row[j2], v1 * tp.psi[2][j2]);
        }
      }
    }
  }
  __syncthreads();

  // flush the tile (with halo) into the periodic global grid
  int org[3] = {0, 0, 0};
  {
    int t = ch.tile;
    for (int c = D - 1; c >= 0; --c) {
      org[c] = (t % geo.nt[c]) * geo.T - M;
      t /= geo.nt[c];
    }
  }
  const int g = geo.g;
  for (int i = threadIdx.x; i < ncell; i += kBlock) {
    const R v = tile[i];
    if (v == R(0)) continue;
    size_t lin;
    if constexpr (D == 1) {
      lin = wrap(org[0] + i, g);
    } else if constexpr (D == 2) {
      const int e0 = i / E, e1 = i - e0 * E;
      lin = size_t(wrap(org[0] + e0, g)) * g + wrap(org[1] + e1, g);
    } else {
      const int e0 = i / (E * E), rem = i - e0 * E * E, e1 = rem / E, e2 = rem - e1 * E;
      lin = (size_t(wrap(org[0] + e0, g)) * g + wrap(org[1] + e1, g)) * g + wrap(org[2] + e2, g);
    }
    atomicAdd(&a.grid[lin], v);
  }
}

// --------------------------------------------------------------------------- block reduction
struct Red4 {
  double s0, s1, mx;
  double cnt;
};

__device__ __forceinline__ Red4 red_combine(Red4 a, Red4 b) {
  return {a.s0 + b.s0, a.s1 + b.s1, fmax(a.mx, b.mx), a.cnt + b.cnt};
}

__device__ Red4 block_reduce(Red4 v, Red4* sh) {
  // wave64 butterfly, then across the 4 waves in fixed order
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    Red4 w;
    w.s0 = __shfl_xor(v.s0, o, 64);
    w.s1 = __shfl_xor(v.s1, o, 64);
    w.mx = __shfl_xor(v.mx, o, 64);
    w.cnt = __shfl_xor(v.cnt, o, 64);
    v = red_combine(v, w);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  Red4 r = sh[0];
  for (int k = 1; k < kBlock / 64; ++k) r = red_combine(r, sh[k]);
  return r;
}

// Final reduction by the last workgroup to finish (ticket counter).  Writes
// stats[0..3] = {sum s0, sum s1, max, count}, adds count to stats[4], and, if wmul_next is set,
// wmul_next = 1/max (the normalization of the next spread's weights).
__device__ void finish_reduce(Red4 mine, Red4* sh, double* partials, unsigned* counter, double* stats,
                              double* wmul_next) {
  __shared__ bool last;
  if (threadIdx.x == 0) {
    partials[4 * blockIdx.x + 0] = mine.s0;
    partials[4 * blockIdx.x + 1] = mine.s1;
    partials[4 * blockIdx.x + 2] = mine.mx;
    partials[4 * blockIdx.x + 3] = mine.cnt;
    __threadfence();
    const unsigned ticket = atomicAdd(counter, 1u);
    last = (ticket == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  Red4 v{0.0, 0.0, 0.0, 0.0};
  const volatile double* pv = partials;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) {
    Red4 w{pv[4 * b + 0], pv[4 * b + 1], pv[4 * b + 2], pv[4 * b + 3]};
    v = red_combine(v, w);
  }
  __syncthreads();
  const Red4 r = block_reduce(v, sh);
  if (threadIdx.x == 0) {
    stats[0] = r.s0;
    stats[1] = r.s1;
    stats[2] = r.mx;
    stats[3] = r.cnt;
    stats[4] += r.cnt;  // running count over all launches into this slot
    if (wmul_next) *wmul_next = (r.mx > 0.0 && r.mx < 1e300) ? 1.0 / r.mx : 1.0;
    *counter = 0u;
  }
}

// --------------------------------------------------------------------------- interp
template <typename R, int D, int M>
__global__ __launch_bounds__(kBlock) void interp_kernel(InterpArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* tile = reinterpret_cast<R*>(smem_raw);
  __shared__ Red4 red_sh[kBlock / 64];
  constexpr int W = 2 * M + 1;
  const Geom geo = a.geo;
  const int E = geo.E;
  const int g = geo.g;
  const int ncell = D == 1 ? E : (D == 2 ? E * E : E * E * E);
  const Chunk ch = a.chunks[blockIdx.x];

  int org[3] = {0, 0, 0};
  {
    int t = ch.tile;
    for (int c = D - 1; c >= 0; --c) {
      org[c] = (t % geo.nt[c]) * geo.T - M;
      t /= geo.nt[c];
    }
  }
  for (int i = threadIdx.x; i < ncell; i += kBlock) {
    size_t lin;
    if constexpr (D == 1) {
      lin = wrap(org[0] + i, g);
    } else if constexpr (D == 2) {
      const int e0 = i / E, e1 = i - e0 * E;
      lin = size_t(wrap(org[0] + e0, g)) * g + wrap(org[1] + e1, g);
    } else {
      const int e0 = i / (E * E), rem = i - e0 * E * E, e1 = rem / E, e2 = rem - e1 * E;
      lin = (size_t(wrap(org[0] + e0, g)) * g + wrap(org[1] + e1, g)) * g + wrap(org[2] + e2, g);
    }
    tile[i] = a.grid[lin];
  }
  __syncthreads();

  const double outmul = a.norm / (a.wmul_src ? *a.wmul_src : 1.0);
  Red4 acc_red{0.0, 0.0, 0.0, 0.0};
  for (int q = ch.start + threadIdx.x; q < ch.start + ch.count; q += kBlock) {
    R u[D];
#pragma unroll
    for (int c = 0; c < D; ++c) u[c] = a.coords[size_t(q) * D + c];
    Taps<R, D, M> tp;
    tp.compute(u, a.win);
    R acc = R(0);
    if constexpr (D == 1) {
#pragma unroll
      for (int j = 0; j < W; ++j) acc += tile[tp.off[0] + j] * tp.psi[0][j];
    } else if constexpr (D == 2) {
#pragma unroll
      for (int j0 = 0; j0 < W; ++j0) {
        const R* row = tile + (tp.off[0] + j0) * E + tp.off[1];
        R racc = R(0);
#pragma unroll
        for (int j1 = 0; j1 < W; ++j1) racc += row[j1] * tp.psi[1][j1];
        acc += racc * tp.psi[0][j0];
      }
    } else {
      for (int j0 = 0; j0 < W; ++j0) {
        R pacc = R(0);
#pragma unroll 1
        for (int j1 = 0; j1 < W; ++j1) {
          const R* row = tile + ((tp.off[0] + j0) * E + tp.off[1] + j1) * E + tp.off[2];
          R racc = R(0);
#pragma unroll
          for (int j2 = 0; j2 < W; ++j2) racc += row[j2] * tp.psi[2][j2];
          pacc += racc * tp.psi[1][j1];
        }
        acc += pacc * tp.psi[0][j0];
      }
    }
    const double t = double(acc) * outmul;
    if (a.epi == EPI_OUT) {
      const double sc = a.scale_vec ? a.scale_vec[q] : 1.0;
      a.out[size_t(a.perm[q]) * a.out_stride + a.out_comp] = t * sc;
    } else {
      const double p = a.p[q];
      const double aold = a.alpha[q];
      const double res = aold * t - p;
      acc_red.s0 += res * res;
      if (p > 0.0) {
        if (!(t > 0.0) || !isfinite(t)) acc_red.cnt += 1.0;
        if (a.epi == EPI_SINK) {
          const double anew = p / t;
          a.alpha[q] = anew;
          acc_red.s1 += anew * t;
          acc_red.mx = fmax(acc_red.mx, anew);
        } else {
          acc_red.s1 += aold * t;
          acc_red.mx = fmax(acc_red.mx, aold);
        }
      } else if (a.epi == EPI_SINK) {
        a.alpha[q] = 0.0;
      }
    }
  }
  if (a.epi != EPI_OUT) {
    const Red4 r = block_reduce(acc_red, red_sh);
    finish_reduce(r, red_sh, a.partials, a.counter, a.stats, a.wmul_next);
  }
}

// --------------------------------------------------------------------------- launchers
template <typename R>
size_t tile_bytes(const Geom& geo) {
  size_t n = geo.E;
  for (int c = 1; c < geo.d; ++c) n *= geo.E;
  return n * sizeof(R);
}

#define NFS_DISPATCH_M(D_, R_, KERNEL, ARGS, NBLK, SHM, STREAM)                                          \
  switch (geo.M) {                                                                                        \
    case 2: hipLaunchKernelGGL((KERNEL<R_, D_, 2>), dim3(NBLK), dim3(kBlock), SHM, STREAM, ARGS); break; \
    case 3: hipLaunchKernelGGL((KERNEL<R_, D_, 3>), dim3(NBLK), dim3(kBlock), SHM, STREAM, ARGS); break; \
    case 4: hipLaunchKernelGGL((KERNEL<R_, D_, 4>), dim3(NBLK), dim3(kBlock), SHM, STREAM, ARGS); break; \
    case 5: hipLaunchKernelGGL((KERNEL<R_, D_, 5>), dim3(NBLK), dim3(kBlock), SHM, STREAM, ARGS); break; \
    case 6: hipLaunchKernelGGL((KERNEL<R_, D_, 6>), dim3(NBLK), dim3(kBlock), SHM, STREAM, ARGS); break; \
    case 7: hipLaunchKernelGGL((KERNEL<R_, D_, 7>), dim3(NBLK), dim3(kBlock), SHM, STREAM, ARGS); break; \
    case 8: hipLaunchKernelGGL((KERNEL<R_, D_, 8>), dim3(NBLK), dim3(kBlock), SHM, STREAM, ARGS); break; \
    default: return hipErrorInvalidValue;                                                                 \
  }

template <typename R>
hipError_t launch_spread(const SpreadArgs<R>& a, int nchunks, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  const Geom& geo = a.geo;
  const size_t shm = tile_bytes<R>(geo);
  if (geo.d == 1) {
    NFS_DISPATCH_M(1, R, spread_kernel, a, nchunks, shm, st)
  } else if (geo.d == 2) {
    NFS_DISPATCH_M(2, R, spread_kernel, a, nchunks, shm, st)
  } else {
    NFS_DISPATCH_M(3, R, spread_kernel, a, nchunks, shm, st)
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_interp(const InterpArgs<R>& a, int nchunks, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  const Geom& geo = a.geo;
  const size_t shm = tile_bytes<R>(geo);
  if (geo.d == 1) {
    NFS_DISPATCH_M(1, R, interp_kernel, a, nchunks, shm, st)
  } else if (geo.d == 2) {
    NFS_DISPATCH_M(2, R, interp_kernel, a, nchunks, shm, st)
  } else {
    NFS_DISPATCH_M(3, R, interp_kernel, a, nchunks, shm, st)
  }
  return hipGetLastError();
}

template hipError_t launch_spread<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread<double>(const SpreadArgs<double>&, int, hipStream_t);
template hipError_t launch_interp<float>(const InterpArgs<float>&, int, hipStream_t);
template hipError_t launch_interp<double>(const InterpArgs<double>&, int, hipStream_t);

}  // namespace nfs
