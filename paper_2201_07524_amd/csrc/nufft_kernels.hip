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
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace nfs {

// Window evaluation.  arg() maps the distance z0 in [-M, -M + 1) from a point
// to its first tap to the per-point argument, and tap(j, x) is the window
// at tap j.  Both precisions evaluate per-tap polynomials by Horner, their
// coefficients read from a small workspace table through scalar loads.
template <typename R>
struct WinEval;

template <>
struct WinEval<float> {
  const float* __restrict__ P;  // (2 kMaxM + 1) x kPolyCoef, uniform across the wave
  float shift;                  // 2M - 1
  __device__ __forceinline__ WinEval(const WindowConst&, const void* p, int M)
      : P(static_cast<const float*>(p)), shift(float(2 * M - 1)) {}
  __device__ __forceinline__ float arg(float z0) const { return fmaf(2.0f, z0, shift); }
  // NC = poly_coef(m): the coefficients the host fitted for this half-width
  template <int NC>
  __device__ __forceinline__ float tap(int j, float x) const {
    const float* c = P + j * kPolyCoef;
    float v = c[NC - 1];
#pragma unroll
    for (int k = NC - 2; k >= 0; --k) v = fmaf(v, x, c[k]);
    return v;
  }
};

// FP64: degree-14 per-tap polynomials (WindowPoly64), 14 FMAs per window
// value instead of a square root, two exponentials and a division.
template <>
struct WinEval<double> {
  const double* __restrict__ P;  // (2 kMaxM + 1) x kPolyCoef64, uniform across the wave
  double shift;                  // 2M - 1
  __device__ __forceinline__ WinEval(const WindowConst&, const void* p, int M)
      : P(static_cast<const double*>(p)), shift(double(2 * M - 1)) {}
  __device__ __forceinline__ double arg(double z0) const { return fma(2.0, z0, shift); }
  template <int NC>
  __device__ __forceinline__ double tap(int j, double x) const {
    const double* c = P + j * kPolyCoef64;
    double v = c[kPolyCoef64 - 1];
#pragma unroll
    for (int k = kPolyCoef64 - 2; k >= 0; --k) v = fma(v, x, c[k]);
    return v;
  }
};

// Window taps of one point: the first tap offset per axis (off), the window
// argument per axis (x), and the 2m+1 window values of every axis c >= FROM
// (axes below FROM are evaluated on the fly by the caller, one value per row,
// so that loops over them can stay rolled with static register indices).
template <typename R, int D, int M, int FROM>
struct Taps {
  static constexpr int W = 2 * M + 1;
  R psi[D][W];
  R x[D];
  int off[D];

  __device__ __forceinline__ void compute(const R* u, const WinEval<R>& ev) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const R s = ceil(u[c] - R(M));
      off[c] = int(s) + M;
      x[c] = ev.arg(s - u[c]);
      if (c >= FROM) {
#pragma unroll
        for (int j = 0; j < W; ++j) psi[c][j] = ev.template tap<poly_coef(M)>(j, x[c]);
      }
    }
  }
};

// Range [lo, hi) of LDS tile cells (linear, axis 0 slowest) that a chunk's
// taps can touch.  In cell order the first axis is the most significant part
// of the sort key, so the chunk's first and last points bound its axis-0
// cells c0; a point in cell c0 has taps on E-rows c0 .. c0 + 2M + 1.
template <typename R, int D, int M>
__device__ __forceinline__ void chunk_rows(const R* coords, const Chunk& ch, const Geom& geo, bool cell_order,
                                           int& lo, int& hi) {
  const int E = geo.E;
  const int inner = D == 1 ? 1 : (D == 2 ? E : E * E);
  if (!cell_order) {
    lo = 0;
    hi = E * inner;
    return;
  }
  const int T = geo.T;
  const int c_first = min(max(int(coords[size_t(ch.start) * D]), 0), T - 1);
  const int c_last = min(max(int(coords[size_t(ch.start + ch.count - 1) * D]), 0), T - 1);
  lo = c_first * inner;
  hi = min(c_last + 2 * M + 2, E) * inner;
}

// a[0..W) <- a[1], ..., a[W-1], a[0] (register moves)
template <typename R, int W>
__device__ __forceinline__ void rotate_left(R (&v)[W]) {
  const R first = v[0];
#pragma unroll
  for (int j = 0; j + 1 < W; ++j) v[j] = v[j + 1];
  v[W - 1] = first;
}

// Lanes of one wave take runs spread over the whole chunk (lane l of slot row
// r gets run l * rows + r), so that the 64 lanes of a wave work in different
// cells of the cell-sorted chunk rather than on the same few LDS words.
constexpr int kWave = 64;
__device__ __forceinline__ int run_of_slot(int slot, int rows) {
  return (slot % kWave) * rows + slot / kWave;
}

__device__ __forceinline__ int wrap(int v, int g) {
  v %= g;
  return v < 0 ? v + g : v;
}

// --------------------------------------------------------------------------- spread
// LDS accumulation modes.  Float atomics in LDS (ds_add_f32/f64) are slow on
// gfx950 (about one lane per three clocks per CU) while 64-bit integer LDS
// atomics run an order of magnitude faster, so contributions v (|v| <= G after
// the weights are normalized by their maximum) are accumulated in fixed point:
//   FIX64  (FP32 path): q = round(v 2^32) in one int64 word;
//   FIX128 (FP64 path): hi = round(v 2^30), lo = round((v 2^30 - hi) 2^30) in
//                       two int64 words (resolution 2^-60 of the largest weight).
// The integer is formed in two FP64 instructions: with M = 1.5 2^52,
// fma(v, 2^s, M) rounds v 2^s to an integer q (|q| < 2^51) and its bit pattern
// is bits(M) + q.  The atomics add these patterns directly.  bits(M) has 48
// zero low bits, so the low 48 bits of a word hold the exact sum of its q's
// whatever the number of adds, as long as |sum q| < 2^47; that bounds the sum
// of |v| landing on one cell of one chunk by 2^15 (FIX64) and 2^17 (FIX128),
// which chunks of at most 32768 points respect.  Integer sums are exact and
// order independent, so the LDS tile is deterministic; its words are flushed
// as exact integers into an int64 grid (GRID_FIX64 / GRID_FIX128), so the
// spread grid is too.  ACC_FLOAT keeps native float atomics (LDS and grid)
// for tiles too large for the fixed-point LDS footprint.
enum AccMode : int { ACC_FLOAT = 0, ACC_FIX64 = 1, ACC_FIX128 = 2 };

constexpr double kFixMagic = 6755399441055744.0;  // 1.5 * 2^52

__device__ __forceinline__ unsigned long long fix_bits(double y) {
  return (unsigned long long)__double_as_longlong(y);
}
// exact sum of the q's held in a word (low 48 bits, sign-extended)
__device__ __forceinline__ long long fix_sum(long long a) {
  return (long long)((unsigned long long)a << 16) >> 16;
}

template <typename R, int ACC>
struct Acc;

template <typename R>
struct Acc<R, ACC_FLOAT> {
  static constexpr int kWords = 0;
  R* t;
  __device__ Acc(unsigned char* raw, int) : t(reinterpret_cast<R*>(raw)) {}
  __device__ __forceinline__ void zero(int i) { t[i] = R(0); }
  __device__ __forceinline__ void add(int i, R v) { atomicAdd(&t[i], v); }
  __device__ __forceinline__ R get(int i) const { return t[i]; }
};

template <>
struct Acc<float, ACC_FIX64> {
  long long* t;
  __device__ Acc(unsigned char* raw, int) : t(reinterpret_cast<long long*>(raw)) {}
  __device__ __forceinline__ void zero(int i) { t[i] = 0; }
  __device__ __forceinline__ void add(int i, float v) {
    const double y = fma(double(v), 4294967296.0, kFixMagic);  // M + round(v 2^32)
    atomicAdd(reinterpret_cast<unsigned long long*>(&t[i]), fix_bits(y));
  }
  __device__ __forceinline__ float get(int i) const { return float(double(fix_sum(t[i])) * 2.3283064365386963e-10); }
  __device__ __forceinline__ long long word(int i) const { return fix_sum(t[i]); }  // units of 2^-32
};

template <>
struct Acc<double, ACC_FIX128> {
  long long* hi_;
  long long* lo_;
  __device__ Acc(unsigned char* raw, int ncell)
      : hi_(reinterpret_cast<long long*>(raw)), lo_(reinterpret_cast<long long*>(raw) + ncell) {}
  __device__ __forceinline__ void zero(int i) {
    hi_[i] = 0;
    lo_[i] = 0;
  }
  __device__ __forceinline__ void add(int i, double v) {
    const double yh = fma(v, 1073741824.0, kFixMagic);  // M + round(v 2^30)
    const double h = yh - kFixMagic;                      // exact
    const double r = fma(v, 1073741824.0, -h);            // exact, |r| <= 1/2
    const double yl = fma(r, 1073741824.0, kFixMagic);
    atomicAdd(reinterpret_cast<unsigned long long*>(&hi_[i]), fix_bits(yh));
    atomicAdd(reinterpret_cast<unsigned long long*>(&lo_[i]), fix_bits(yl));
  }
  __device__ __forceinline__ double get(int i) const {
    return double(fix_sum(hi_[i])) * 9.313225746154785e-10 + double(fix_sum(lo_[i])) * 8.673617379884035e-19;
  }
  __device__ __forceinline__ long long word_hi(int i) const { return fix_sum(hi_[i]); }  // units of 2^-30
  __device__ __forceinline__ long long word_lo(int i) const { return fix_sum(lo_[i]); }  // units of 2^-60
};

// Lane exchanges inside a DPP quad: CTRL 0xB1 = quad permutation [1,0,3,2]
// (the value of lane ^ 1), 0x4E = [2,3,0,1] (lane ^ 2).
template <int CTRL>
__device__ __forceinline__ float quad_swap(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
// Sum over the GROUP lanes (1, 2 or 4 aligned lanes) of a group, in every lane of it.
template <int GROUP, typename R>
__device__ __forceinline__ R group_sum(R v) {
  if constexpr (GROUP >= 2) v += quad_swap<0xB1>(v);
  if constexpr (GROUP >= 4) v += quad_swap<0x4E>(v);
  return v;
}

// Adds the W taps of one tile row.  tap(j) gives this lane's value of tap j.
// GROUP = 2 or 4: the group's lanes hold runs of the same cell (same tap
// offsets).  Each tap is summed across the group by DPP, and in every block
// of GROUP taps lane `member` adds tap j + member, so one atomic instruction
// with every lane active does the work of GROUP; the W mod GROUP last taps
// are added by lanes 0.. of the group.
template <int GROUP, int W, typename R, typename ACCT, typename F>
__device__ __forceinline__ void add_row(ACCT& tile, int row, int member, F tap) {
  if constexpr (GROUP == 1) {
#pragma unroll
    for (int j = 0; j < W; ++j) tile.add(row + j, tap(j));
  } else {
    constexpr int WB = W - W % GROUP;
#pragma unroll
    for (int j = 0; j < WB; j += GROUP) {
      R mine = R(0);
#pragma unroll
      for (int k = 0; k < GROUP; ++k) {
        const R v = group_sum<GROUP>(tap(j + k));
        mine = member == k ? v : mine;
      }
      tile.add(row + j + member, mine);
    }
#pragma unroll
    for (int j = WB; j < W; ++j) {
      const R v = group_sum<GROUP>(tap(j));
      if (member == j - WB) tile.add(row + j, v);
    }
  }
}

// Spreads GC consecutive sorted points that lie in one cell (so their windows
// start at the same offsets): per tap the GC contributions are summed in
// registers, and the tap costs one fixed-point conversion and one LDS atomic
// for the whole run.
// cnt (1..GC): the run's points; the others get weight zero and repeat the
// last point, so no read leaves the run.  GROUP: see add_row (member = lane % GROUP).
template <typename R, int D, int M, int ACC, int GC, int GROUP = 1>
__device__ __forceinline__ void spread_run(Acc<R, ACC>& tile, const SpreadArgs<R>& a, const WinEval<R>& ev, int E,
                                           int q0, double wm, int cnt = GC, int member = 0) {
  constexpr int W = 2 * M + 1;
  constexpr int FROM = D == 1 ? 0 : 1;
  Taps<R, D, M, FROM> tp[GC];
  R w[GC];
#pragma unroll
  for (int p = 0; p < GC; ++p) {
    const int q = q0 + min(p, cnt - 1);
    w[p] = p < cnt ? R(a.w[q] * wm) : R(0);
    R u[D];
#pragma unroll
    for (int c = 0; c < D; ++c) u[c] = a.coords[size_t(q) * D + c];
    tp[p].compute(u, ev);
  }
  if constexpr (D == 1) {
    add_row<GROUP, W, R>(tile, tp[0].off[0], member, [&](int j) {
      R v = R(0);
#pragma unroll
      for (int p = 0; p < GC; ++p) v += w[p] * tp[p].psi[0][j];
      return v;
    });
  } else if constexpr (D == 2) {
#pragma unroll 1
    for (int j0 = 0; j0 < W; ++j0) {
      R a0[GC];
#pragma unroll
      for (int p = 0; p < GC; ++p) a0[p] = w[p] * ev.template tap<poly_coef(M)>(j0, tp[p].x[0]);
      const int row = (tp[0].off[0] + j0) * E + tp[0].off[1];
      add_row<GROUP, W, R>(tile, row, member, [&](int j1) {
        R v = R(0);
#pragma unroll
        for (int p = 0; p < GC; ++p) v += a0[p] * tp[p].psi[1][j1];
        return v;
      });
    }
  } else {
#pragma unroll 1
    for (int j0 = 0; j0 < W; ++j0) {
      R b0[GC];
#pragma unroll
      for (int p = 0; p < GC; ++p) b0[p] = w[p] * ev.template tap<poly_coef(M)>(j0, tp[p].x[0]);
      if constexpr (sizeof(R) == 4) {
        // FP32: j1 unrolled, every window index static
#pragma unroll
        for (int j1 = 0; j1 < W; ++j1) {
          R a1[GC];
#pragma unroll
          for (int p = 0; p < GC; ++p) a1[p] = b0[p] * tp[p].psi[1][j1];
          const int row = ((tp[0].off[0] + j0) * E + tp[0].off[1] + j1) * E + tp[0].off[2];
          add_row<GROUP, W, R>(tile, row, member, [&](int j2) {
            R v = R(0);
#pragma unroll
            for (int p = 0; p < GC; ++p) v += a1[p] * tp[p].psi[2][j2];
            return v;
          });
        }
      } else {
        // FP64: the rolled j1 loop reads element 0 of the second-axis windows,
        // which are rotated by one per iteration (a full cycle restores them)
#pragma unroll 1
        for (int j1 = 0; j1 < W; ++j1) {
          R a1[GC];
#pragma unroll
          for (int p = 0; p < GC; ++p) a1[p] = b0[p] * tp[p].psi[1][0];
          const int row = ((tp[0].off[0] + j0) * E + tp[0].off[1] + j1) * E + tp[0].off[2];
          add_row<GROUP, W, R>(tile, row, member, [&](int j2) {
            R v = R(0);
#pragma unroll
            for (int p = 0; p < GC; ++p) v += a1[p] * tp[p].psi[2][j2];
            return v;
          });
#pragma unroll
          for (int p = 0; p < GC; ++p) rotate_left(tp[p].psi[1]);
        }
      }
    }
  }
}

// Threads per spreading workgroup: in 3-D the fixed-point LDS tile is large
// (25^3 words at tile 8, m = 8), one workgroup fills a CU's LDS, and 512
// threads give two waves per SIMD instead of one.
__host__ __device__ constexpr int spread_block(int d) { return d == 3 ? 512 : kBlock; }

template <typename R, int D, int M, int ACC>
__global__ __launch_bounds__(spread_block(D)) void spread_kernel(SpreadArgs<R> a) {
  constexpr int BS = spread_block(D);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Geom geo = a.geo;
  const int E = geo.E;
  const int ncell = D == 1 ? E : (D == 2 ? E * E : E * E * E);
  Acc<R, ACC> tile(smem_raw, ncell);
  const int cb = blockIdx.x;
  const Chunk ch = a.chunks[cb];
  if (a.pstate && a.pstate[kPState * ch.prob] == 2) return;  // the problem has stopped

  // the part store (per-tile reduction) needs the whole tile
  int lo, hi;
  chunk_rows<R, D, M>(a.coords, ch, geo, a.cell_order && !a.part, lo, hi);
  for (int i = lo + threadIdx.x; i < hi; i += BS) tile.zero(i);
  __syncthreads();

  // The chunk's run table lists full runs of G same-cell points, then the
  // remaining points one by one; each phase is free of lane divergence.
  constexpr int G = run_length<R>(D);
  const WinEval<R> ev(a.win, a.wpoly, M);
  const double wm = a.wconst * (a.wmul ? a.wmul[ch.prob] : 1.0);
  if (a.srun) {
    // every point in a run of at most G (the last run of a cell partial);
    // same-cell pairs of runs on adjacent lanes, 32 pairs per wave row,
    // spread over the chunk like the runs below
    const int* sr = a.srun + ch.start;
    const int nqe = a.nsrun[3 * cb], npe = a.nsrun[3 * cb + 1], nsolo = a.nsrun[3 * cb + 2];
    // groups of GROUP same-cell runs on aligned lanes, kWave / GROUP groups per wave row,
    // spread over the chunk like single runs
    auto grouped = [&](auto group_tag, const int* tab, int ngroups) {
      constexpr int GR = decltype(group_tag)::value;
      const int rows = (ngroups + kWave / GR - 1) / (kWave / GR);
      for (int slot = threadIdx.x; slot < rows * kWave; slot += BS) {
        const int lane = slot % kWave;
        const int grp = (lane / GR) * rows + slot / kWave;
        if (grp < ngroups) {
          const int e = tab[GR * grp + lane % GR];
          spread_run<R, D, M, ACC, G, GR>(tile, a, ev, E, ch.start + (e & 0xffff), wm, (e >> 16) + 1, lane % GR);
        }
      }
    };
    grouped(std::integral_constant<int, 4>{}, sr, nqe / 4);
    grouped(std::integral_constant<int, 2>{}, sr + nqe, npe / 2);
    const int rows = (nsolo + kWave - 1) / kWave;
    for (int slot = threadIdx.x; slot < rows * kWave; slot += BS) {
      const int rr = run_of_slot(slot, rows);
      if (rr < nsolo) {
        const int e = sr[nqe + npe + rr];
        spread_run<R, D, M, ACC, G>(tile, a, ev, E, ch.start + (e & 0xffff), wm, (e >> 16) + 1);
      }
    }
  } else {
    const int* runs = a.runs + ch.start;
    const int nfull = a.nruns[2 * cb], nsingle = a.nruns[2 * cb + 1];
    int rows = (nfull + kWave - 1) / kWave;
    for (int slot = threadIdx.x; slot < rows * kWave; slot += BS) {
      const int rr = run_of_slot(slot, rows);
      if (rr < nfull) spread_run<R, D, M, ACC, G>(tile, a, ev, E, ch.start + runs[rr], wm);
    }
    rows = (nsingle + kWave - 1) / kWave;
    for (int slot = threadIdx.x; slot < rows * kWave; slot += BS) {
      const int rr = run_of_slot(slot, rows);
      if (rr < nsingle) spread_run<R, D, M, ACC, 1>(tile, a, ev, E, ch.start + runs[nfull + rr], wm);
    }
  }
  __syncthreads();

  if (a.part) {
    R* dst = a.part + size_t(cb) * ncell;
    for (int i = threadIdx.x; i < ncell; i += BS) dst[i] = tile.get(i);
    return;
  }

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
  auto cell_of = [&](int i) {
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
    return size_t(ch.prob) * a.grid_stride + lin;
  };
  for (int i = lo + threadIdx.x; i < hi; i += BS) {
    if constexpr (ACC == ACC_FLOAT) {
      const R v = tile.get(i);
      if (v != R(0)) atomicAdd(&a.grid[cell_of(i)], v);
    } else if constexpr (ACC == ACC_FIX64) {
      // exact integer sums: the grid does not depend on the order of the flushes
      const long long q = tile.word(i);
      if (q != 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(a.grid) + cell_of(i), static_cast<unsigned long long>(q));
    } else {
      const long long qh = tile.word_hi(i), ql = tile.word_lo(i);
      if (qh != 0 || ql != 0) {
        unsigned long long* gw = reinterpret_cast<unsigned long long*>(a.grid) + cell_of(i);
        if (qh != 0) atomicAdd(gw, static_cast<unsigned long long>(qh));
        if (ql != 0) atomicAdd(gw + a.grid_plane, static_cast<unsigned long long>(ql));
      }
    }
  }
}

// --------------------------------------------------------------------------- spread reduction
// Tile b owns cells [b T, b T + T) per axis.  A chunk of neighbour tile
// nb = b + delta stores cells [nb T - M, nb T + T + M] (E = T + 2M + 1 values);
// per axis the overlap with tile b is
//   delta =  0: cells [0, T)      <-> e = M + l
//   delta = -1: cells [0, M+1)    <-> e = T + M + l
//   delta = +1: cells [T-M, T)    <-> e = l - (T - M)
// One workgroup per (tile, delta) sums that overlap over the chunks of nb in
// registers (index math hoisted out of the chunk loop) and adds it to the
// grid, so each grid cell receives at most 3^d atomic adds.  Requires
// T >= M + 1, T dividing g and at least 3 tiles per axis; the grid must be
// zero on entry.
constexpr int kRedPerThread = 8;

template <typename R, int D>
__global__ __launch_bounds__(kBlock) void spread_reduce_kernel(ReduceArgs<R> a) {
  if (a.pstate && a.pstate[0] == 2) return;  // the (single) problem has stopped
  const Geom geo = a.geo;
  const int T = geo.T, M = geo.M, E = geo.E, g = geo.g;
  constexpr int NNB = D == 1 ? 3 : (D == 2 ? 9 : 27);
  const int tile = blockIdx.x / NNB;
  const int k = blockIdx.x - tile * NNB;
  int bc[3] = {0, 0, 0}, dl[3] = {0, 0, 0};
  {
    int t = tile, r = k;
    for (int c = D - 1; c >= 0; --c) {
      bc[c] = t % geo.nt[c];
      t /= geo.nt[c];
      dl[c] = r % 3 - 1;
      r /= 3;
    }
  }
  int nb = 0, lb[3] = {0, 0, 0}, len[3] = {1, 1, 1}, e0[3] = {0, 0, 0}, cnt = 1;
  for (int c = 0; c < D; ++c) {
    int t = bc[c] + dl[c];
    t = t < 0 ? t + geo.nt[c] : (t >= geo.nt[c] ? t - geo.nt[c] : t);
    nb = nb * geo.nt[c] + t;
    if (dl[c] == 0) {
      lb[c] = 0;
      len[c] = T;
      e0[c] = M;
    } else if (dl[c] < 0) {
      lb[c] = 0;
      len[c] = M + 1;
      e0[c] = T + M;
    } else {
      lb[c] = T - M;
      len[c] = M;
      e0[c] = 0;
    }
    cnt *= len[c];
  }
  const int c0 = a.tile_chunks[nb], c1 = a.tile_chunks[nb + 1];
  if (c0 == c1) return;
  int ecell = 1;
  for (int c = 0; c < D; ++c) ecell *= E;
  int eidx[kRedPerThread];
  size_t gidx[kRedPerThread];
  R acc[kRedPerThread];
  int nmine = 0;
#pragma unroll
  for (int s = 0; s < kRedPerThread; ++s) {
    const int i = threadIdx.x + s * kBlock;
    eidx[s] = -1;
    gidx[s] = 0;
    acc[s] = R(0);
    if (i < cnt) {
      int rem = i, ei = 0;
      size_t gi = 0;
      int l[3], e[3];
      for (int c = D - 1; c >= 0; --c) {
        const int v = rem % len[c];
        rem /= len[c];
        l[c] = lb[c] + v;
        e[c] = e0[c] + v;
      }
      for (int c = 0; c < D; ++c) {
        ei = ei * E + e[c];
        gi = gi * g + size_t(bc[c] * T + l[c]);
      }
      eidx[s] = ei;
      gidx[s] = gi;
      nmine = s + 1;
    }
  }
  for (int ch = c0; ch < c1; ++ch) {
    const R* src = a.part + size_t(ch) * ecell;
#pragma unroll
    for (int s = 0; s < kRedPerThread; ++s)
      if (s < nmine && eidx[s] >= 0) acc[s] += src[eidx[s]];
  }
#pragma unroll
  for (int s = 0; s < kRedPerThread; ++s)
    if (s < nmine && eidx[s] >= 0 && acc[s] != R(0)) atomicAdd(&a.grid[gidx[s]], acc[s]);
}

template <typename R>
hipError_t launch_spread_reduce(const ReduceArgs<R>& a, int nbins, hipStream_t st) {
  size_t tc = 1;
  for (int c = 0; c < a.geo.d; ++c) tc *= a.geo.T;
  if (tc > size_t(kRedPerThread) * kBlock) return hipErrorInvalidValue;
  const int nnb = a.geo.d == 1 ? 3 : (a.geo.d == 2 ? 9 : 27);
  const dim3 grid(nbins * nnb);
  if (a.geo.d == 1) hipLaunchKernelGGL((spread_reduce_kernel<R, 1>), grid, dim3(kBlock), 0, st, a);
  else if (a.geo.d == 2) hipLaunchKernelGGL((spread_reduce_kernel<R, 2>), grid, dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((spread_reduce_kernel<R, 3>), grid, dim3(kBlock), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_spread_reduce<float>(const ReduceArgs<float>&, int, hipStream_t);
template hipError_t launch_spread_reduce<double>(const ReduceArgs<double>&, int, hipStream_t);

// --------------------------------------------------------------------------- block reduction
// Per-target quantities of a half-step, reduced over the problem's targets.
struct Red {
  double res2;  // sum of squared residuals
  double mass;  // sum alpha t
  double l1;    // sum |alpha_new|
  double mx;    // max alpha (log domain: max potential)
  double tmin;  // min t
  double tmax;  // max t
  double cnt;   // sums t <= 0 or non-finite
};
constexpr int kRedVals = 8;  // doubles per workgroup partial

__device__ __forceinline__ Red red_init(bool logd) {
  return {0.0, 0.0, 0.0, logd ? -INFINITY : 0.0, INFINITY, 0.0, 0.0};
}

__device__ __forceinline__ Red red_combine(Red a, Red b) {
  return {a.res2 + b.res2, a.mass + b.mass, a.l1 + b.l1, fmax(a.mx, b.mx),
          fmin(a.tmin, b.tmin), fmax(a.tmax, b.tmax), a.cnt + b.cnt};
}

template <int NT = kBlock>
__device__ Red block_reduce(Red v, Red* sh) {
  // wave64 butterfly, then across the NT / 64 waves in fixed order
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    Red w;
    w.res2 = __shfl_xor(v.res2, o, 64);
    w.mass = __shfl_xor(v.mass, o, 64);
    w.l1 = __shfl_xor(v.l1, o, 64);
    w.mx = __shfl_xor(v.mx, o, 64);
    w.tmin = __shfl_xor(v.tmin, o, 64);
    w.tmax = __shfl_xor(v.tmax, o, 64);
    w.cnt = __shfl_xor(v.cnt, o, 64);
    v = red_combine(v, w);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  Red r = sh[0];
  for (int k = 1; k < NT / 64; ++k) r = red_combine(r, sh[k]);
  return r;
}

// Per-problem reduction of the interpolation's per-chunk partials, in chunk
// order, by a kernel launched right after the interpolation (the kernel
// boundary makes the partials visible).  The chunks of problem pb are
// [prob_chunks[pb], prob_chunks[pb + 1]).  Writes the problem's statistics
// (layout kStat), sets wmul_next to 1/max (the normalization of the next
// spread's weights; log domain: the max itself, the shift of the next
// spread's potentials) and advances its stop state (kPState).  A problem that
// had stopped was skipped by the interpolation and is skipped here.
//
// A fence and a ticket per workgroup, the last one reducing, would save the
// launch but not time: on a part with one L2 per XCD the device-scope fence
// writes the L2 back, once per workgroup (22K per interpolation of the
// 512-problem batch, 2.9 ms per iteration).
template <typename R>
__global__ __launch_bounds__(kBlock) void reduce_stats_kernel(InterpArgs<R> a) {
  __shared__ Red red_sh[kBlock / 64];
  const int pb = blockIdx.x;
  int* pstate = a.pstate ? a.pstate + kPState * pb : nullptr;
  const int ps0 = pstate ? pstate[0] : 0;
  if (ps0 == 2) return;
  const bool logd = a.epi == EPI_LOGSINK || a.epi == EPI_LOGEVAL;
  const int c0 = a.prob_chunks[pb], c1 = a.prob_chunks[pb + 1];
  double* stats = a.stats + kStat * pb;
  // The scalars the writing thread needs are loaded before the partials, so
  // that their round trips overlap instead of following the reduction
  // (5.8 -> 5.0 us per launch on average over the 2-D and 3-D mixtures).
  double st4 = 0.0, st8 = 0.0, src_l1 = 0.0, tol2 = 0.0;
  int ps1 = 0;
  if (threadIdx.x == 0) {
    st4 = stats[4];
    st8 = stats[8];
    if (a.src_l1) src_l1 = a.src_l1[kStat * pb];
    if (pstate) {
      ps1 = pstate[1];
      tol2 = *a.tol2;
    }
  }
  Red v = red_init(logd);
#pragma unroll 4
  for (int b = c0 + threadIdx.x; b < c1; b += kBlock) {
    const double* pw = a.partials + kRedVals * size_t(b);
    const Red w{pw[0], pw[1], pw[2], pw[3], pw[4], pw[5], pw[6]};
    v = red_combine(v, w);
  }
  const Red r = block_reduce(v, red_sh);
  if (threadIdx.x != 0) return;
  stats[0] = r.res2;
  stats[1] = r.mass;
  stats[2] = r.mx;
  stats[3] = r.cnt;
  stats[4] = st4 + r.cnt;  // running count over all launches into this slot
  stats[5] = r.tmin;
  stats[6] = r.tmax;
  stats[7] = r.l1;
  if (a.src_l1) {
    // ||w||_1 / min t; a sum t <= 0 (or none positive) counts as an unbounded range
    const double range = r.tmin > 0.0 ? src_l1 / r.tmin : INFINITY;
    stats[8] = fmax(st8, range);
  }
  if (a.wmul_next) {
    if (logd)
      a.wmul_next[pb] = isfinite(r.mx) ? r.mx : 0.0;
    else
      a.wmul_next[pb] = (r.mx > 0.0 && r.mx < 1e300) ? 1.0 / r.mx : 1.0;
  }
  if (pstate) {
    if (a.half == 0) {
      // ||E|| of the state the previous iteration left (its column term is
      // zero up to rounding after an alpha_t update)
      if (ps0 == 0 && tol2 > 0.0 && r.res2 <= tol2) pstate[0] = 1;
    } else {
      pstate[1] = ps1 + 1;
      if (ps0 == 1) pstate[0] = 2;
    }
  }
}

// --------------------------------------------------------------------------- interp
constexpr int kInterpRun = 2;
// Threads per interpolation workgroup: 512 for FP32 in 3-D (1e6-point 3-D
// mixture, m = 8: 415 -> 380 us per launch, the iteration 3.09 -> 3.01 ms),
// 256 otherwise (2-D mixture: 48 us at 256 threads, 52 at 512; FP64 in 3-D
// needs more registers than 512 threads leave).
template <typename R, int D>
constexpr int interp_block() { return sizeof(R) == 4 && D == 3 ? 512 : kBlock; }

// Interpolates GC consecutive sorted points that lie in one cell: each row of
// taps is read from the LDS tile once and dotted with the GC windows.
template <typename R, int D, int M, int GC>
__device__ __forceinline__ void interp_run(const R* tile, const WinEval<R>& ev, int E, const R (&u)[GC][D],
                                           R (&acc)[GC]) {
  constexpr int W = 2 * M + 1;
  constexpr int FROM = D == 1 ? 0 : 1;
  Taps<R, D, M, FROM> tp[GC];
#pragma unroll
  for (int p = 0; p < GC; ++p) {
    tp[p].compute(u[p], ev);
    acc[p] = R(0);
  }
  if constexpr (D == 1) {
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const R gv = tile[tp[0].off[0] + j];
#pragma unroll
      for (int p = 0; p < GC; ++p) acc[p] += gv * tp[p].psi[0][j];
    }
  } else if constexpr (D == 2) {
#pragma unroll 1
    for (int j0 = 0; j0 < W; ++j0) {
      const R* row = tile + (tp[0].off[0] + j0) * E + tp[0].off[1];
      R gv[W];
#pragma unroll
      for (int j1 = 0; j1 < W; ++j1) gv[j1] = row[j1];
#pragma unroll
      for (int p = 0; p < GC; ++p) {
        R racc = R(0);
#pragma unroll
        for (int j1 = 0; j1 < W; ++j1) racc += gv[j1] * tp[p].psi[1][j1];
        acc[p] += racc * ev.template tap<poly_coef(M)>(j0, tp[p].x[0]);
      }
    }
  } else {
#pragma unroll 1
    for (int j0 = 0; j0 < W; ++j0) {
      R pacc[GC];
#pragma unroll
      for (int p = 0; p < GC; ++p) pacc[p] = R(0);
      if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int j1 = 0; j1 < W; ++j1) {
          const R* row = tile + ((tp[0].off[0] + j0) * E + tp[0].off[1] + j1) * E + tp[0].off[2];
          R gv[W];
#pragma unroll
          for (int j2 = 0; j2 < W; ++j2) gv[j2] = row[j2];
#pragma unroll
          for (int p = 0; p < GC; ++p) {
            R racc = R(0);
#pragma unroll
            for (int j2 = 0; j2 < W; ++j2) racc += gv[j2] * tp[p].psi[2][j2];
            pacc[p] += racc * tp[p].psi[1][j1];
          }
        }
      } else {
        // FP64: a fully unrolled j1 loop does not fit the register file; roll
        // it and rotate the second-axis windows (a full cycle restores them)
#pragma unroll 1
        for (int j1 = 0; j1 < W; ++j1) {
          const R* row = tile + ((tp[0].off[0] + j0) * E + tp[0].off[1] + j1) * E + tp[0].off[2];
          R gv[W];
#pragma unroll
          for (int j2 = 0; j2 < W; ++j2) gv[j2] = row[j2];
#pragma unroll
          for (int p = 0; p < GC; ++p) {
            R racc = R(0);
#pragma unroll
            for (int j2 = 0; j2 < W; ++j2) racc += gv[j2] * tp[p].psi[2][j2];
            pacc[p] += racc * tp[p].psi[1][0];
            rotate_left(tp[p].psi[1]);
          }
        }
      }
#pragma unroll
      for (int p = 0; p < GC; ++p) acc[p] += pacc[p] * ev.template tap<poly_coef(M)>(j0, tp[p].x[0]);
    }
  }
}

// Inputs of one interpolation step (GC consecutive sorted points from q0):
// their coordinates and, for the scaling epilogues, p and the old scaling
// (or potential).
template <typename R, int D, int GC>
struct PointIn {
  R u[GC][D];
  double p[GC], al[GC];
  __device__ __forceinline__ void load(const InterpArgs<R>& a, int q0, bool pa) {
#pragma unroll
    for (int k = 0; k < GC; ++k) {
#pragma unroll
      for (int c = 0; c < D; ++c) u[k][c] = a.coords[size_t(q0 + k) * D + c];
      p[k] = pa ? a.p[q0 + k] : 0.0;
      al[k] = pa ? a.alpha[q0 + k] : 0.0;
    }
  }
};

// LOG: the log-domain epilogues (EPI_LOGSINK / EPI_LOGEVAL), instantiated
// apart so that their log and exp do not raise the register count of the
// others.
// Minimum waves per SIMD the interpolation keeps: the FP32 3-D scaling
// instances sit at the 128-register edge of 4 waves and are held there.
template <typename R, int D, bool LOG>
constexpr int interp_min_waves() { return sizeof(R) == 4 && D == 3 && !LOG ? 4 : 1; }

template <typename R, int D, int M, bool LOG>
__global__ __launch_bounds__((interp_block<R, D>()), (interp_min_waves<R, D, LOG>())) void interp_kernel(InterpArgs<R> a) {
  constexpr int IB = interp_block<R, D>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* tile = reinterpret_cast<R*>(smem_raw);
  __shared__ Red red_sh[IB / 64];
  const Geom geo = a.geo;
  const int E = geo.E;
  const int g = geo.g;
  const int ncell = D == 1 ? E : (D == 2 ? E * E : E * E * E);
  const int cb = blockIdx.x;
  const Chunk ch = a.chunks[cb];
  if (a.pstate && a.pstate[kPState * ch.prob] == 2) return;  // the problem has stopped

  int org[3] = {0, 0, 0};
  {
    int t = ch.tile;
    for (int c = D - 1; c >= 0; --c) {
      org[c] = (t % geo.nt[c]) * geo.T - M;
      t /= geo.nt[c];
    }
  }
  // FP32 in 1-D and 2-D: each step's inputs are loaded one step ahead (the
  // first ones before the tile), so a thread waits on the run table and the
  // point data while it computes the step before, not after it.  FP64 and
  // 3-D load the coordinates at the step and p and the old scaling in the
  // epilogue: a second set of live registers would cost them occupancy.
  constexpr bool ahead = sizeof(R) == 4 && D <= 2;
  constexpr int G = run_length<R>(D);
  constexpr int GI = kInterpRun < G ? kInterpRun : G;  // points per interpolation run, divides G
  constexpr int SUB = G / GI;
  const bool pa = ahead && a.epi != EPI_OUT;
  const int* runs = a.runs + ch.start;
  const int nfull = a.nruns[2 * cb], nsingle = a.nruns[2 * cb + 1];
  const int nit = nfull * SUB;
  auto step_q0 = [&](int rr) { return ch.start + runs[rr / SUB] + (rr % SUB) * GI; };
  PointIn<R, D, GI> cur;
  int qc = 0;
  if constexpr (ahead) {
    if (int(threadIdx.x) < nit) {
      qc = step_q0(threadIdx.x);
      cur.load(a, qc, pa);
    }
  }

  int lo, hi;
  chunk_rows<R, D, M>(a.coords, ch, geo, a.cell_order, lo, hi);
  // The tile's grid values, kTileBatch loads per thread in flight before the
  // first LDS store: a store waits for its load, so the plain loop paid one
  // memory round trip per element, which sets the time of a chunk of few
  // points (small or sparse problems of a batch).
  const R* gp = a.grid + size_t(ch.prob) * a.grid_stride;
  auto grid_at = [&](int i) {
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
    return gp[lin];
  };
  constexpr int kTileBatch = 8;
  for (int base = lo + int(threadIdx.x); base < hi; base += kTileBatch * IB) {
    R v[kTileBatch];
#pragma unroll
    for (int u = 0; u < kTileBatch; ++u) {
      const int i = base + u * IB;
      if (i < hi) v[u] = grid_at(i);
    }
#pragma unroll
    for (int u = 0; u < kTileBatch; ++u) {
      const int i = base + u * IB;
      if (i < hi) tile[i] = v[u];
    }
  }
  __syncthreads();

  constexpr bool logd = LOG;
  const double outmul = logd ? a.norm : a.norm / (a.wmul_src ? a.wmul_src[ch.prob] : 1.0);
  // log domain: t = exp(shift/eps - 1/2) S, alpha = exp(beta/eps - 1/2)
  const double shift = logd ? a.wmul_src[ch.prob] : 0.0;
  const double linv = logd ? a.leps[kLepsStride * ch.prob] : 0.0;
  const double leps = logd ? a.leps[kLepsStride * ch.prob + 1] : 0.0;
  Red acc_red = red_init(logd);
  // nfq: the point's near-field sum, loaded by the caller before the
  // interpolation (a load inside here lets the compiler hoist it above the
  // tap loop together with the LDS reads, at a large cost in registers)
  auto epilogue = [&](int q, R acc, double nfq, double p, double aold) {
    const double t = (double(acc) + nfq) * outmul;
    if (!pa && a.epi != EPI_OUT) {
      p = a.p[q];
      aold = a.alpha[q];
    }
    if constexpr (LOG) {
      // alpha_old t = exp((beta_old + shift)/eps - 1) S: the marginal entry of
      // the state before the update
      const double bold = aold;
      const double m = p > 0.0 ? exp((bold + shift) * linv - 1.0) * t : 0.0;
      const double res = m - p;
      acc_red.res2 += res * res;
      if (a.epi == EPI_LOGSINK) {
        // beta = eps (log p - log t) + eps/2 with log t = shift/eps - 1/2 + log S;
        // a zero weight, or a sum t <= 0 (counted), gives the potential -inf
        double b = -INFINITY;
        if (p > 0.0) {
          if (t > 0.0 && isfinite(t)) {
            b = leps * (log(p) - log(t) + 1.0) - shift;
            acc_red.mx = fmax(acc_red.mx, b);
            acc_red.tmin = fmin(acc_red.tmin, t);
            acc_red.tmax = fmax(acc_red.tmax, t);
          } else {
            acc_red.cnt += 1.0;
          }
          acc_red.mass += p;
        }
        a.alpha[q] = b;
      } else {
        if (p > 0.0) {
          if (!(t > 0.0) || !isfinite(t)) acc_red.cnt += 1.0;
          acc_red.mass += m;
          acc_red.mx = fmax(acc_red.mx, bold);
        }
      }
    } else if (a.epi == EPI_OUT) {
      const double sc = a.scale_vec ? a.scale_vec[q] : 1.0;
      a.out[size_t(a.perm[q]) * a.out_stride + a.out_comp] = t * sc;
    } else {
      // EPI_SINK and EPI_EVAL: the residual of eq. (Error) of the state before
      // the update, alpha_old t - p (fused: no extra kernel product)
      const double res = aold * t - p;
      acc_red.res2 += res * res;
      if (p > 0.0) {
        if (!(t > 0.0) || !isfinite(t)) acc_red.cnt += 1.0;
        acc_red.tmin = fmin(acc_red.tmin, t);
        acc_red.tmax = fmax(acc_red.tmax, t);
      }
      if (a.epi == EPI_SINK) {
        // a point of weight zero gets scaling zero
        const double anew = p > 0.0 ? p / t : 0.0;
        a.alpha[q] = anew;
        if (p > 0.0) {
          acc_red.mass += anew * t;
          acc_red.l1 += fabs(anew);
          acc_red.mx = fmax(acc_red.mx, anew);
        }
      } else if (p > 0.0) {
        acc_red.mass += aold * t;
        acc_red.mx = fmax(acc_red.mx, aold);
      }
    }
  };
  // Full runs of G same-cell points first, then the remaining points one by
  // one (each phase free of lane divergence).  Consecutive lanes take
  // consecutive runs: global accesses stay coalesced, and lanes in the same
  // cell read the same LDS words (a broadcast).
  const WinEval<R> ev(a.win, a.wpoly, M);
  auto step = [&](int q0, const auto& in) {
    constexpr int GC = sizeof(in.u) / sizeof(in.u[0]);
    double nfq[GC];
#pragma unroll
    for (int p = 0; p < GC; ++p) nfq[p] = a.nf ? a.nf[q0 + p] : 0.0;
    R acc[GC];
    interp_run<R, D, M, GC>(tile, ev, E, in.u, acc);
#pragma unroll
    for (int p = 0; p < GC; ++p) epilogue(q0 + p, acc[p], nfq[p], in.p[p], in.al[p]);
  };
  if constexpr (ahead) {
    for (int rr = threadIdx.x; rr < nit; rr += IB) {
      const int rn = rr + IB;
      PointIn<R, D, GI> nxt;
      int qn = 0;
      if (rn < nit) {
        qn = step_q0(rn);
        nxt.load(a, qn, pa);
      }
      step(qc, cur);
      cur = nxt;
      qc = qn;
    }
    PointIn<R, D, 1> one;
    int q1 = 0;
    if (int(threadIdx.x) < nsingle) {
      q1 = ch.start + runs[nfull + threadIdx.x];
      one.load(a, q1, pa);
    }
    for (int rr = threadIdx.x; rr < nsingle; rr += IB) {
      const int rn = rr + IB;
      PointIn<R, D, 1> nxt;
      int qn = 0;
      if (rn < nsingle) {
        qn = ch.start + runs[nfull + rn];
        nxt.load(a, qn, pa);
      }
      step(q1, one);
      one = nxt;
      q1 = qn;
    }
  } else {
    for (int rr = threadIdx.x; rr < nit; rr += IB) {
      const int q0 = step_q0(rr);
      PointIn<R, D, GI> in;
      in.load(a, q0, false);
      step(q0, in);
    }
    for (int rr = threadIdx.x; rr < nsingle; rr += IB) {
      const int q0 = ch.start + runs[nfull + rr];
      PointIn<R, D, 1> in;
      in.load(a, q0, false);
      step(q0, in);
    }
  }
  if (a.epi != EPI_OUT) {
    // this chunk's partial; reduce_stats_kernel combines them per problem
    const Red r = block_reduce<IB>(acc_red, red_sh);
    if (threadIdx.x == 0) {
      double* pw = a.partials + kRedVals * size_t(cb);
      pw[0] = r.res2;
      pw[1] = r.mass;
      pw[2] = r.l1;
      pw[3] = r.mx;
      pw[4] = r.tmin;
      pw[5] = r.tmax;
      pw[6] = r.cnt;
    }
  }
}

// --------------------------------------------------------------------------- launchers
template <typename R>
size_t tile_bytes(const Geom& geo) {
  size_t n = geo.E;
  for (int c = 1; c < geo.d; ++c) n *= geo.E;
  return n * sizeof(R);
}

#define NFS_DISPATCH_M_X(D_, R_, KERNEL, X_, ARGS, NBLK, SHM, STREAM)                                        \
  switch (geo.M) {                                                                                          \
    case 2: hipLaunchKernelGGL((KERNEL<R_, D_, 2, X_>), dim3(NBLK), dim3(interp_block<R_, D_>()), SHM, STREAM, ARGS); break; \
    case 3: hipLaunchKernelGGL((KERNEL<R_, D_, 3, X_>), dim3(NBLK), dim3(interp_block<R_, D_>()), SHM, STREAM, ARGS); break; \
    case 4: hipLaunchKernelGGL((KERNEL<R_, D_, 4, X_>), dim3(NBLK), dim3(interp_block<R_, D_>()), SHM, STREAM, ARGS); break; \
    case 5: hipLaunchKernelGGL((KERNEL<R_, D_, 5, X_>), dim3(NBLK), dim3(interp_block<R_, D_>()), SHM, STREAM, ARGS); break; \
    case 6: hipLaunchKernelGGL((KERNEL<R_, D_, 6, X_>), dim3(NBLK), dim3(interp_block<R_, D_>()), SHM, STREAM, ARGS); break; \
    case 7: hipLaunchKernelGGL((KERNEL<R_, D_, 7, X_>), dim3(NBLK), dim3(interp_block<R_, D_>()), SHM, STREAM, ARGS); break; \
    case 8: hipLaunchKernelGGL((KERNEL<R_, D_, 8, X_>), dim3(NBLK), dim3(interp_block<R_, D_>()), SHM, STREAM, ARGS); break; \
    default: return hipErrorInvalidValue;                                                                   \
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

// Bytes of LDS per cell of the spread tile for each accumulation mode.
template <typename R>
int acc_mode_for(const Geom& geo, size_t* shm) {
  size_t n = geo.E;
  for (int c = 1; c < geo.d; ++c) n *= geo.E;
  const size_t lds_max = 160 * 1024;
  if (sizeof(R) == 4 && n * 8 <= lds_max) {
    *shm = n * 8;
    return ACC_FIX64;
  }
  if (sizeof(R) == 8 && n * 16 <= lds_max) {
    *shm = n * 16;
    return ACC_FIX128;
  }
  *shm = n * sizeof(R);
  return ACC_FLOAT;
}

#define NFS_SPREAD_M(D_, R_, ACC_, NBLK, SHM, STREAM)                                                          \
  switch (geo.M) {                                                                                             \
    case 2: hipLaunchKernelGGL((spread_kernel<R_, D_, 2, ACC_>), dim3(NBLK), dim3(spread_block(D_)), SHM, STREAM, a); break; \
    case 3: hipLaunchKernelGGL((spread_kernel<R_, D_, 3, ACC_>), dim3(NBLK), dim3(spread_block(D_)), SHM, STREAM, a); break; \
    case 4: hipLaunchKernelGGL((spread_kernel<R_, D_, 4, ACC_>), dim3(NBLK), dim3(spread_block(D_)), SHM, STREAM, a); break; \
    case 5: hipLaunchKernelGGL((spread_kernel<R_, D_, 5, ACC_>), dim3(NBLK), dim3(spread_block(D_)), SHM, STREAM, a); break; \
    case 6: hipLaunchKernelGGL((spread_kernel<R_, D_, 6, ACC_>), dim3(NBLK), dim3(spread_block(D_)), SHM, STREAM, a); break; \
    case 7: hipLaunchKernelGGL((spread_kernel<R_, D_, 7, ACC_>), dim3(NBLK), dim3(spread_block(D_)), SHM, STREAM, a); break; \
    case 8: hipLaunchKernelGGL((spread_kernel<R_, D_, 8, ACC_>), dim3(NBLK), dim3(spread_block(D_)), SHM, STREAM, a); break; \
    default: return hipErrorInvalidValue;                                                                      \
  }

template <typename R, int ACC>
hipError_t launch_spread_acc(const SpreadArgs<R>& a, int nchunks, size_t shm, hipStream_t st) {
  const Geom& geo = a.geo;
  if (geo.d == 1) {
    NFS_SPREAD_M(1, R, ACC, nchunks, shm, st)
  } else if (geo.d == 2) {
    NFS_SPREAD_M(2, R, ACC, nchunks, shm, st)
  } else {
    NFS_SPREAD_M(3, R, ACC, nchunks, shm, st)
  }
  return hipGetLastError();
}

int spread_grid_mode(const Geom& geo, int rbytes, bool two_level) {
  if (two_level) return GRID_REAL;
  size_t shm = 0;
  const int mode = rbytes == 4 ? acc_mode_for<float>(geo, &shm) : acc_mode_for<double>(geo, &shm);
  return mode == ACC_FIX64 ? GRID_FIX64 : (mode == ACC_FIX128 ? GRID_FIX128 : GRID_REAL);
}

template <typename R>
hipError_t launch_spread(const SpreadArgs<R>& a, int nchunks, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  size_t shm = 0;
  const int mode = acc_mode_for<R>(a.geo, &shm);
  // the flush writes the grid format of the accumulation mode (the chunk-tile
  // store of the per-tile reduction writes R values)
  const int want = a.part ? GRID_REAL
                          : (mode == ACC_FIX64 ? GRID_FIX64 : (mode == ACC_FIX128 ? GRID_FIX128 : GRID_REAL));
  if (!a.part && a.gmode != want) return hipErrorInvalidValue;
  if constexpr (sizeof(R) == 4) {
    if (mode == ACC_FIX64) return launch_spread_acc<R, ACC_FIX64>(a, nchunks, shm, st);
  } else {
    if (mode == ACC_FIX128) return launch_spread_acc<R, ACC_FIX128>(a, nchunks, shm, st);
  }
  return launch_spread_acc<R, ACC_FLOAT>(a, nchunks, shm, st);
}

template <typename R>
hipError_t launch_interp(const InterpArgs<R>& a, int nchunks, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  const Geom& geo = a.geo;
  const size_t shm = tile_bytes<R>(geo);
  const bool log_epi = a.epi == EPI_LOGSINK || a.epi == EPI_LOGEVAL;
  if (log_epi && (!a.wmul_src || !a.leps)) return hipErrorInvalidValue;
  if (geo.d == 1) {
    if (log_epi) {
      NFS_DISPATCH_M_X(1, R, interp_kernel, true, a, nchunks, shm, st)
    } else {
      NFS_DISPATCH_M_X(1, R, interp_kernel, false, a, nchunks, shm, st)
    }
  } else if (geo.d == 2) {
    if (log_epi) {
      NFS_DISPATCH_M_X(2, R, interp_kernel, true, a, nchunks, shm, st)
    } else {
      NFS_DISPATCH_M_X(2, R, interp_kernel, false, a, nchunks, shm, st)
    }
  } else {
    if (log_epi) {
      NFS_DISPATCH_M_X(3, R, interp_kernel, true, a, nchunks, shm, st)
    } else {
      NFS_DISPATCH_M_X(3, R, interp_kernel, false, a, nchunks, shm, st)
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.epi == EPI_OUT) return e;
  if (a.nprob <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reduce_stats_kernel<R>, dim3(a.nprob), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template hipError_t launch_spread<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread<double>(const SpreadArgs<double>&, int, hipStream_t);
template hipError_t launch_interp<float>(const InterpArgs<float>&, int, hipStream_t);
template hipError_t launch_interp<double>(const InterpArgs<double>&, int, hipStream_t);

}  // namespace nfs
