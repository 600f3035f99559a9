// Stockham FFTs on the oversampled grid, staged in LDS (gfx950).
//
// The d-dimensional real FFT of fast summation is split into one pass per axis:
//   rows_kernel  - contiguous last axis, two real rows of one problem packed
//                  into one complex FFT; R2C keeps the half spectrum
//                  k = 0..N/2, C2R rebuilds the rows from it.  For d = 1 the
//                  whole chain forward -> multiplier -> inverse runs here
//                  (FUSED1D), one problem's row per pencil.
//   axis_kernel  - a strided axis, several adjacent pencils per workgroup so
//                  global accesses are contiguous across pencils.  Modes: forward
//                  with pruned centered output k = -N/2..N/2, inverse from that
//                  pruned input, or fused forward -> multiplier -> inverse
//                  (the diagonal of eq. (fastsum) applied in LDS, so the
//                  spectrum never goes back to HBM).
// Each pencil of length L = 2^p is transformed by radix-4 Stockham passes plus
// one radix-2 pass when p is odd, ping-ponging between two LDS buffers.  Both
// kernels are compiled once per p (2..12): with L, the pencils per workgroup
// and every pass's stride and twiddle offset known at compile time, a pass is
// a few dozen instructions with no integer multiply or divide, which is what
// bounds these latency-bound passes (one wave per SIMD, one pass after the
// other).  Twiddles come from per-pass tables (fft_pass_bits) whose entries
// the lanes of a wave read contiguously.
#pragma once

#include "common.h"
#include "kernels.h"

namespace nfs {

__host__ __device__ inline int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

// A workgroup-strided loop over i < n whose global loads are issued kBatch at
// a time: load(i) only reads, use(i, v) consumes its result.  Every load of a
// batch is in flight before the first use, so the loop waits on memory once
// per batch instead of once per element (a store between two loads of the
// plain loop keeps the second from issuing until the first has returned).
constexpr int kBatch = 8;
template <typename T, typename Load, typename Use>
__device__ __forceinline__ void batched(int n, Load load, Use use) {
  for (int base = threadIdx.x; base < n; base += kBatch * kBlock) {
    T v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = base + u * kBlock;
      if (i < n) v[u] = load(i);
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = base + u * kBlock;
      if (i < n) use(i, v[u]);
    }
  }
}

// Staging of the twiddle table in LDS, split so that its loads travel with
// the data loads of the pass: start() fetches the first kRegs kBlock entries
// into registers, the data loads follow, and finish() writes them to LDS
// (copying any rest of a longer table) before the barrier that precedes the
// first Stockham pass.  One memory round trip instead of two.
template <typename R>
struct TwiddleStage {
  static constexpr int kRegs = 4;
  cplx<R> v[kRegs];
  __device__ __forceinline__ void start(const cplx<R>* tw, int L) {
#pragma unroll
    for (int u = 0; u < kRegs; ++u) {
      const int i = threadIdx.x + u * kBlock;
      if (i < L) v[u] = tw[i];
    }
  }
  __device__ __forceinline__ void finish(cplx<R>* t, const cplx<R>* tw, int L) {
#pragma unroll
    for (int u = 0; u < kRegs; ++u) {
      const int i = threadIdx.x + u * kBlock;
      if (i < L) t[i] = v[u];
    }
    constexpr int kHead = kRegs * kBlock;
    if (L > kHead)
      batched<cplx<R>>(
          L - kHead, [&](int i) { return tw[kHead + i]; }, [&](int i, cplx<R> x) { t[kHead + i] = x; });
  }
};

// One complete FFT of P pencils (each L = 2^LG contiguous complex values) held
// in buffer `A`; `B` is scratch of the same size.  Returns the buffer holding
// the result.  Forward uses exp(-2 pi i jk/L), inverse exp(+2 pi i jk/L), both
// unnormalized.  Pass s (Ns = 4^s) takes butterfly j (k = j mod Ns) from
// entries j + m L/4, multiplies entry m by e^(-+2 pi i m k/(4 Ns)) (the pass
// table's entry (m - 1) Ns + k), and writes output m to (j - k) 4 + k + m Ns;
// an odd LG ends with the radix-2 pass at Ns = L/2.  Must be called by all
// threads of the block.
template <typename R, int LG, int P>
__device__ __forceinline__ cplx<R>* stockham(cplx<R>* A, cplx<R>* B, const cplx<R>* tw, bool inverse) {
  constexpr int L = 1 << LG;
  constexpr int Q = L >> 2;
  cplx<R>* src = A;
  cplx<R>* dst = B;
  int off = 0;
#pragma unroll
  for (int s = 0; s < LG / 2; ++s) {
    const int Ns = 1 << (2 * s);
#pragma unroll
    for (int b0 = 0; b0 < P * Q; b0 += kBlock) {
      const int b = b0 + int(threadIdx.x);
      if ((P * Q) % kBlock == 0 || b < P * Q) {
        const int p = b >> (LG - 2);
        const int j = b & (Q - 1);
        const int k = j & (Ns - 1);
        const cplx<R>* sp = src + p * L + j;
        cplx<R> a0 = sp[0], a1 = sp[Q], a2 = sp[2 * Q], a3 = sp[3 * Q];
        if (Ns > 1) {
          const cplx<R>* t = tw + off + k;
          cplx<R> w1 = t[0], w2 = t[Ns], w3 = t[2 * Ns];
          if (inverse) {
            w1.y = -w1.y;
            w2.y = -w2.y;
            w3.y = -w3.y;
          }
          a1 = cmul(a1, w1);
          a2 = cmul(a2, w2);
          a3 = cmul(a3, w3);
        }
        const cplx<R> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
        // forward: b1 = t1 - i t3, b3 = t1 + i t3; inverse swaps the signs
        const cplx<R> it3 = inverse ? cplx<R>{-t3.y, t3.x} : cplx<R>{t3.y, -t3.x};
        cplx<R>* d = dst + p * L + (j - k) * 4 + k;
        d[0] = cadd(t0, t2);
        d[Ns] = cadd(t1, it3);
        d[2 * Ns] = csub(t0, t2);
        d[3 * Ns] = csub(t1, it3);
      }
    }
    if (Ns > 1) off += 3 * Ns;
    __syncthreads();
    cplx<R>* t = src;
    src = dst;
    dst = t;
  }
  if (LG & 1) {
    constexpr int H = L >> 1;  // = Ns of this pass, so k = j
#pragma unroll
    for (int b0 = 0; b0 < P * H; b0 += kBlock) {
      const int b = b0 + int(threadIdx.x);
      if ((P * H) % kBlock == 0 || b < P * H) {
        const int p = b >> (LG - 1);
        const int j = b & (H - 1);
        const cplx<R>* sp = src + p * L + j;
        cplx<R> w = H > 1 ? tw[off + j] : cplx<R>{R(1), R(0)};
        if (inverse) w.y = -w.y;
        const cplx<R> a0 = sp[0];
        const cplx<R> a1 = cmul(sp[H], w);
        cplx<R>* d = dst + p * L + j;
        d[0] = cadd(a0, a1);
        d[H] = csub(a0, a1);
      }
    }
    __syncthreads();
    src = dst;
  }
  return src;
}

// stockham with the twiddles in LDS (tl) when staged there, else in global
// memory (tg).  Two inlined copies, so that each reads its table through a
// pointer of known address space: a pointer that may be either makes every
// twiddle read a flat load, which waits on global and LDS counters alike.
template <typename R, int LG, int P>
__device__ __forceinline__ cplx<R>* fft(cplx<R>* A, cplx<R>* B, bool tw_lds, const cplx<R>* tl, const cplx<R>* tg,
                                        bool inverse) {
  return tw_lds ? stockham<R, LG, P>(A, B, tl, inverse) : stockham<R, LG, P>(A, B, tg, inverse);
}

// Table entry of problem prob at |k|.  32-bit offsets: the host keeps the
// tables of all problems below 2^32 entries.
template <typename R>
__device__ __forceinline__ R table_value(const Multiplier& mu, long prob, int d, int N, int k0, int k1, int k2) {
  const unsigned H = unsigned(N / 2 + 1);
  unsigned idx = unsigned(abs(k0));
  if (d >= 2) idx = idx * H + unsigned(abs(k1));
  if (d >= 3) idx = idx * H + unsigned(abs(k2));
  return reinterpret_cast<const R*>(mu.tab)[unsigned(prob) * unsigned(mu.tab_stride) + idx];
}

// v times the multiplier value m at frequency (k0, k1, k2), times i 2 pi k_c
// for a derivative along axis c.
template <typename R>
__device__ __forceinline__ cplx<R> scale_multiplier(cplx<R> v, R m, const Multiplier& mu, int k0, int k1, int k2) {
  v.x *= m;
  v.y *= m;
  if (mu.deriv >= 0) {
    const int kc = mu.deriv == 0 ? k0 : (mu.deriv == 1 ? k1 : k2);
    const R f = R(6.283185307179586476925286766559) * R(kc);
    v = cplx<R>{-v.y * f, v.x * f};
  }
  return v;
}

template <typename R>
__device__ __forceinline__ cplx<R> apply_multiplier(cplx<R> v, const Multiplier& mu, long prob, int d, int N, int k0,
                                                   int k1, int k2) {
  return scale_multiplier(v, table_value<R>(mu, prob, d, N, k0, k1, k2), mu, k0, k1, k2);
}

// Cell idx of the spread grid as an R value, in the grid's format (GridMode),
// and its clearing for the next spreading.
template <typename R>
__device__ __forceinline__ R grid_value(const R* g, int mode, long plane, long idx) {
  if (mode == GRID_REAL) return g[idx];
  const long long* w = reinterpret_cast<const long long*>(g);
  if (mode == GRID_FIX64) return R(double(w[idx]) * 2.3283064365386963e-10);
  return R(double(w[idx]) * 9.313225746154785e-10 + double(w[plane + idx]) * 8.673617379884035e-19);
}
template <typename R>
__device__ __forceinline__ void grid_clear(R* g, int mode, long plane, long idx) {
  if (mode == GRID_REAL) {
    g[idx] = R(0);
    return;
  }
  long long* w = reinterpret_cast<long long*>(g);
  w[idx] = 0;
  if (mode == GRID_FIX128) w[plane + idx] = 0;
}

__host__ __device__ constexpr int rows_pencils(int L) { return L >= 1024 ? 1 : 1024 / L; }

template <typename R, int LG>
__global__ __launch_bounds__(kBlock) void rows_kernel(RowArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int L = 1 << LG;
  constexpr int P = rows_pencils(L);
  cplx<R>* A = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* B = A + P * L;
  // twiddles staged in LDS (read by every pass) when they fit
  cplx<R>* tlds = B + P * L;
  TwiddleStage<R> tws;
  if (a.tw_lds) tws.start(a.tw, L);
  const int K0 = a.N / 2 + 1;
  constexpr int lshift = LG;

  if (a.mode == ROW_FUSED1D) {
    // Each row is one problem, transformed alone in a pencil of its own (zero
    // imaginary part): packed two to a complex FFT, a problem's rounding would
    // scale with the other's grid, whatever that holds (a diverging FP32
    // problem of a batch holds huge or negative scalings).  The multiplier
    // is real and even, so D Z stays Hermitian and the inverse is real.
    const long row0 = long(blockIdx.x) * P;
    batched<R>(
        P * L,
        [&](int i) {
          const long row = row0 + (i >> lshift);
          return row < a.nrows ? grid_value(a.real_in, a.gmode, a.grid_plane, row * L + (i & (L - 1))) : R(0);
        },
        [&](int i, R v) { A[i] = cplx<R>{v, R(0)}; });
    if (a.tw_lds) tws.finish(tlds, a.tw, L);
    __syncthreads();
    cplx<R>* res = fft<R, LG, P>(A, B, a.tw_lds, tlds, a.tw, false);
    cplx<R>* other = res == A ? B : A;
    // table value at k (zero outside the symmetric set I_N), times i 2 pi k
    // for a derivative
    batched<R>(
        P * L,
        [&](int i) {
          const int j = i & (L - 1);
          const int kk = j <= L / 2 ? j : j - L;
          const long row = row0 + (i >> lshift);
          return abs(kk) <= a.N / 2 && row < a.nrows ? table_value<R>(a.mul, row, 1, a.N, kk, 0, 0) : R(0);
        },
        [&](int i, R m) {
          const int j = i & (L - 1);
          other[i] = scale_multiplier(res[i], m, a.mul, j <= L / 2 ? j : j - L, 0, 0);
        });
    __syncthreads();
    cplx<R>* out = fft<R, LG, P>(other, res, a.tw_lds, tlds, a.tw, true);
    for (int i = threadIdx.x; i < P * L; i += kBlock) {
      const long row = row0 + (i >> lshift);
      if (row < a.nrows) a.real_io[row * L + (i & (L - 1))] = out[i].x;
    }
    // the source grid is cleared for the next spreading last, after every
    // use of a loaded value (see zero_source below)
    if (a.zero_src) {
      R* z = const_cast<R*>(a.real_in);
      for (int i = threadIdx.x; i < P * L; i += kBlock) {
        const long row = row0 + (i >> lshift);
        if (row < a.nrows) grid_clear(z, a.gmode, a.grid_plane, row * L + (i & (L - 1)));
      }
    }
    return;
  }

  // R2C and C2R: pencil p packs rows a = row0 + 2p and b = a + 1 of one
  // problem (the rows of a 2-D or 3-D grid come in pairs) as Z = A + i B.
  const long row0 = long(blockIdx.x) * 2 * P;
  if (a.mode == ROW_R2C) {
    const R* src = a.real_io;
    // The source grid is cleared for the next spreading after the last use
    // of anything loaded: a store issued between the loads and their use
    // would make each use wait for it as well.
    auto zero_source = [&]() {
      if (!a.zero_src) return;
      R* z = const_cast<R*>(src);
      for (int i = threadIdx.x; i < 2 * P * L; i += kBlock) {
        const long row = row0 + (i >> lshift);
        if (row < a.nrows) grid_clear(z, a.gmode, a.grid_plane, row * L + (i & (L - 1)));
      }
    };
    batched<R>(
        2 * P * L,
        [&](int i) {
          const long row = row0 + (i >> lshift);
          return row < a.nrows ? grid_value(src, a.gmode, a.grid_plane, row * L + (i & (L - 1))) : R(0);
        },
        [&](int i, R v) {
          const int r = i >> lshift;
          const int c = i & (L - 1);
          cplx<R>* e = A + (r >> 1) * L + c;
          if (r & 1) e->y = v;
          else e->x = v;
        });
    if (a.tw_lds) tws.finish(tlds, a.tw, L);
    __syncthreads();
    cplx<R>* res = fft<R, LG, P>(A, B, a.tw_lds, tlds, a.tw, false);
    for (int i = threadIdx.x; i < P * K0; i += kBlock) {
      const int p = i / K0;
      const int k = i - p * K0;
      const cplx<R> Z = res[p * L + k];
      const cplx<R> Zm = cconj(res[p * L + ((L - k) & (L - 1))]);
      const cplx<R> s = cadd(Z, Zm), df = csub(Z, Zm);
      const cplx<R> Av{s.x * R(0.5), s.y * R(0.5)};
      const cplx<R> Bv{df.y * R(0.5), -df.x * R(0.5)};
      const long ra = row0 + 2 * p;
      if (ra < a.nrows) a.spec[ra * K0 + k] = Av;
      if (ra + 1 < a.nrows) a.spec[(ra + 1) * K0 + k] = Bv;
    }
    zero_source();
    return;
  }

  // ROW_C2R: Z = A + i B on k = 0..N/2 and its Hermitian mirror on L - k
  struct Pair {
    cplx<R> a, b;
  };
  batched<Pair>(
      P * L,
      [&](int i) {
        const int j = i & (L - 1);
        const long ra = row0 + 2 * (i >> lshift);
        const int k = j < K0 ? j : (L - j < K0 ? L - j : -1);
        Pair s{{R(0), R(0)}, {R(0), R(0)}};
        if (k >= 0) {
          if (ra < a.nrows) s.a = a.spec[ra * K0 + k];
          if (ra + 1 < a.nrows) s.b = a.spec[(ra + 1) * K0 + k];
        }
        return s;
      },
      [&](int i, Pair s) {
        const int j = i & (L - 1);
        cplx<R> Z{R(0), R(0)};
        if (j < K0 || L - j < K0) {
          if (j >= K0) {  // mirrored bin L - k
            s.a.y = -s.a.y;
            s.b.y = -s.b.y;
          }
          Z = cplx<R>{s.a.x - s.b.y, s.a.y + s.b.x};
        }
        A[i] = Z;
      });
  if (a.tw_lds) tws.finish(tlds, a.tw, L);
  __syncthreads();
  cplx<R>* out = fft<R, LG, P>(A, B, a.tw_lds, tlds, a.tw, true);
  for (int i = threadIdx.x; i < 2 * P * L; i += kBlock) {
    const int r = i >> lshift;
    const int c = i & (L - 1);
    const long row = row0 + r;
    if (row < a.nrows) {
      const cplx<R> v = out[(r >> 1) * L + c];
      a.real_io[row * L + c] = (r & 1) ? v.y : v.x;
    }
  }
}

// Pencil q of an axis pass -> its outer group o and offset ii in the group.
// Pencil numbers and element offsets are 32-bit: the launcher rejects passes
// with 2^31 pencils or arrays of 2^32 elements or more.
template <typename R>
__device__ __forceinline__ void pencil_origin(const AxisArgs<R>& a, long q, unsigned& o, unsigned& ii) {
  o = unsigned(q) / unsigned(a.inner);
  ii = unsigned(q) - o * unsigned(a.inner);
}

// Frequencies (k1, k2) of the other axes for offset ii of a 2-D or 3-D pass.
__device__ __forceinline__ void other_freqs(int d, int half, unsigned ii, int& k1, int& k2) {
  k1 = 0;
  k2 = 0;
  if (d == 2) k1 = int(ii);
  else if (d == 3) {
    const unsigned K0 = unsigned(half + 1);
    k1 = int(ii / K0) - half;
    k2 = int(ii % K0);
  }
}

__host__ __device__ constexpr int axis_pencils(int L) { return L >= 1024 ? 1 : 1024 / L; }

template <typename R, int LG>
__global__ __launch_bounds__(kBlock) void axis_kernel(AxisArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int L = 1 << LG;
  constexpr int P = axis_pencils(L);
  cplx<R>* A = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* B = A + P * L;
  // twiddles staged in LDS (read by every pass) when they fit
  cplx<R>* tlds = B + P * L;
  TwiddleStage<R> tws;
  if (a.tw_lds) tws.start(a.tw, L);
  // pencils numbered per XCD: a strided line holds 16 adjacent pencils' values,
  // which then come from one XCD's L2
  const long q0 = xcd_block(blockIdx.x, gridDim.x) * P;
  const int half = a.N / 2;
  constexpr int pshift = LG >= 10 ? 0 : 10 - LG;
  constexpr int lshift = LG;

  // Fused pass: the multiplier values of the elements i = threadIdx.x +
  // u kBlock this thread rescales after the forward FFT do not depend on the
  // transform, so they are fetched here with the data (0 outside the
  // symmetric set and past the last pencil).  Longer passes load them after.
  constexpr int kMulRegs = 4;
  R mreg[kMulRegs];
  const bool mul_pre = a.mode == AX_FUSED && P * L <= kMulRegs * kBlock;
  if (mul_pre) {
#pragma unroll
    for (int u = 0; u < kMulRegs; ++u) {
      const int i = threadIdx.x + u * kBlock;
      const int bin = i & (L - 1);
      const int k0 = bin <= L / 2 ? bin : bin - L;
      const long q = q0 + (i >> lshift);
      mreg[u] = R(0);
      if (i < P * L && abs(k0) <= half && q < a.npen) {
        unsigned o, ii;
        pencil_origin(a, q, o, ii);
        int k1, k2;
        other_freqs(a.d, half, ii, k1, k2);
        mreg[u] = table_value<R>(a.mul, o, a.d, a.N, k0, k1, k2);
      }
    }
  }

  if (a.mode == AX_INV || a.nin < L) {
    for (int i = threadIdx.x; i < P * L; i += kBlock) A[i] = cplx<R>{R(0), R(0)};
    __syncthreads();
  }
  // entry e of pencil p: i = e P + p, so adjacent lanes read adjacent pencils.
  // The inverse pass from a centered spectrum may apply the multiplier on
  // load; its table value travels with the entry and is applied on use.
  const bool inv_mul = a.in_centered && a.mode == AX_INV && a.apply_mul;
  struct Entry {
    cplx<R> v;
    R m;
  };
  batched<Entry>(
      P * a.nin,
      [&](int i) {
        const int e = i >> pshift;
        const long q = q0 + (i & (P - 1));
        Entry t{{R(0), R(0)}, R(0)};
        if (q < a.npen) {
          unsigned o, ii;
          pencil_origin(a, q, o, ii);
          t.v = a.in[o * unsigned(a.in_ostride) + ii + unsigned(e) * unsigned(a.in_stride)];
          if (inv_mul) {
            int k1, k2;
            other_freqs(a.d, half, ii, k1, k2);
            t.m = table_value<R>(a.mul, o, a.d, a.N, e - half, k1, k2);
          }
        }
        return t;
      },
      [&](int i, Entry t) {
        const int p = i & (P - 1);
        const int e = i >> pshift;
        const long q = q0 + p;
        if (q >= a.npen) return;
        int bin = e;
        if (a.in_centered) {
          const int k = e - half;
          bin = k < 0 ? k + L : k;
          if (inv_mul) {
            unsigned o, ii;
            pencil_origin(a, q, o, ii);
            int k1, k2;
            other_freqs(a.d, half, ii, k1, k2);
            t.v = scale_multiplier(t.v, t.m, a.mul, k, k1, k2);
          }
        }
        A[p * L + bin] = t.v;
      });
  if (a.tw_lds) tws.finish(tlds, a.tw, L);
  __syncthreads();

  cplx<R>* res;
  if (a.mode == AX_INV) {
    res = fft<R, LG, P>(A, B, a.tw_lds, tlds, a.tw, true);
  } else {
    res = fft<R, LG, P>(A, B, a.tw_lds, tlds, a.tw, false);
    if (mul_pre) {
#pragma unroll
      for (int u = 0; u < kMulRegs; ++u) {
        const int i = threadIdx.x + u * kBlock;
        if (i < P * L) {
          const int bin = i & (L - 1);
          const int k0 = bin <= L / 2 ? bin : bin - L;
          int k1 = 0, k2 = 0;
          if (a.mul.deriv > 0 && q0 + (i >> lshift) < a.npen) {
            unsigned o, ii;
            pencil_origin(a, q0 + (i >> lshift), o, ii);
            other_freqs(a.d, half, ii, k1, k2);
          }
          res[i] = scale_multiplier(res[i], mreg[u], a.mul, k0, k1, k2);
        }
      }
      __syncthreads();
      cplx<R>* other = res == A ? B : A;
      res = fft<R, LG, P>(res, other, a.tw_lds, tlds, a.tw, true);
    } else if (a.mode == AX_FUSED) {
      // in place: each element is read and rewritten by the same thread
      batched<cplx<R>>(
          P * L,
          [&](int i) {
            const int bin = i & (L - 1);
            const int k0 = bin <= L / 2 ? bin : bin - L;
            const long q = q0 + (i >> lshift);
            cplx<R> v{R(0), R(0)};
            if (abs(k0) <= half && q < a.npen) {
              unsigned o, ii;
              pencil_origin(a, q, o, ii);
              int k1, k2;
              other_freqs(a.d, half, ii, k1, k2);
              v = apply_multiplier(res[i], a.mul, o, a.d, a.N, k0, k1, k2);
            }
            return v;
          },
          [&](int i, cplx<R> v) { res[i] = v; });
      __syncthreads();
      cplx<R>* other = res == A ? B : A;
      res = fft<R, LG, P>(res, other, a.tw_lds, tlds, a.tw, true);
    }
  }

  for (int i = threadIdx.x; i < P * a.nout; i += kBlock) {
    const int p = i & (P - 1);
    const int e = i >> pshift;
    const long q = q0 + p;
    if (q >= a.npen) continue;
    unsigned o, ii;
    pencil_origin(a, q, o, ii);
    int bin = e;
    if (a.out_centered) {
      const int k = e - half;
      bin = k < 0 ? k + L : k;
    }
    a.out[o * unsigned(a.out_ostride) + ii + unsigned(e) * unsigned(a.out_stride)] = res[p * L + bin];
  }
}

// LDS bytes of a pass with P pencils of length L: two ping-pong buffers, plus
// the twiddle table when that still fits in 160 KiB.
template <typename R>
static size_t fft_lds(int P, int L, int* tw_lds) {
  const size_t buf = size_t(2) * P * L * sizeof(cplx<R>);
  const size_t twb = size_t(L) * sizeof(cplx<R>);
  *tw_lds = buf + twb <= size_t(160) * 1024;
  return buf + (*tw_lds ? twb : 0);
}

// Kernel instance for L = 2^lg, lg in [kMinLg, kMaxLg] (grids of 4 to 4096).
constexpr int kMinLg = 2, kMaxLg = 12;
template <typename R, int LG>
static void* rows_instance(int lg) {
  if constexpr (LG > kMaxLg) {
    return nullptr;
  } else {
    return lg == LG ? reinterpret_cast<void*>(&rows_kernel<R, LG>) : rows_instance<R, LG + 1>(lg);
  }
}
template <typename R, int LG>
static void* axis_instance(int lg) {
  if constexpr (LG > kMaxLg) {
    return nullptr;
  } else {
    return lg == LG ? reinterpret_cast<void*>(&axis_kernel<R, LG>) : axis_instance<R, LG + 1>(lg);
  }
}

template <typename R>
hipError_t launch_rows(const RowArgs<R>& a_in, hipStream_t st) {
  RowArgs<R> a = a_in;
  const int lg = ilog2(a.L);
  if ((1 << lg) != a.L || lg < kMinLg || lg > kMaxLg) return hipErrorInvalidValue;
  const int P = rows_pencils(a.L);
  const int rows_per_block = a.mode == ROW_FUSED1D ? P : 2 * P;  // FUSED1D: one row per pencil
  const long nblk = (a.nrows + rows_per_block - 1) / rows_per_block;
  const size_t shm = fft_lds<R>(P, a.L, &a.tw_lds);
  void* args[] = {&a};
  return hipLaunchKernel(rows_instance<R, kMinLg>(lg), dim3(nblk), dim3(kBlock), args, shm, st);
}

template <typename R>
hipError_t launch_axis(const AxisArgs<R>& a_in, hipStream_t st) {
  AxisArgs<R> a = a_in;
  const int lg = ilog2(a.L);
  if ((1 << lg) != a.L || lg < kMinLg || lg > kMaxLg) return hipErrorInvalidValue;
  if (a.npen >= (long(1) << 31) || a.inner <= 0) return hipErrorInvalidValue;
  const long groups = (a.npen + a.inner - 1) / a.inner;
  const long ext_in = groups * a.in_ostride, ext_out = groups * a.out_ostride;
  if (ext_in >= (long(1) << 32) || ext_out >= (long(1) << 32)) return hipErrorInvalidValue;
  const int P = axis_pencils(a.L);
  const long nblk = (a.npen + P - 1) / P;
  const size_t shm = fft_lds<R>(P, a.L, &a.tw_lds);
  void* args[] = {&a};
  return hipLaunchKernel(axis_instance<R, kMinLg>(lg), dim3(nblk), dim3(kBlock), args, shm, st);
}

}  // namespace nfs
