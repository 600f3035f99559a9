// Stockham FFTs on the oversampled grid, staged in LDS (gfx950).
//
// The d-dimensional real FFT of fast summation is split into one pass per axis:
//   rows_kernel  - contiguous last axis, two real rows packed into one complex
//                  FFT; R2C keeps the half spectrum k = 0..N/2, C2R rebuilds
//                  the rows from it.  For d = 1 the whole chain
//                  forward -> multiplier -> inverse runs here (FUSED1D).
//   axis_kernel  - a strided axis, several adjacent pencils per workgroup so
//                  global accesses are contiguous across pencils.  Modes: forward
//                  with pruned centered output k = -N/2..N/2, inverse from that
//                  pruned input, or fused forward -> multiplier -> inverse
//                  (the diagonal of eq. (fastsum) applied in LDS, so the
//                  spectrum never goes back to HBM).
// Each pencil of length L = 2^p is transformed by radix-4 Stockham passes plus
// one radix-2 pass when p is odd, ping-ponging between two LDS buffers.
#include "common.h"
#include "kernels.h"

namespace nfs {

__host__ __device__ inline int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

// One complete FFT of P pencils (each L contiguous complex values) held in
// buffer `A`; `B` is scratch of the same size.  Returns the buffer holding the
// result.  Forward uses exp(-2 pi i jk/L), inverse exp(+2 pi i jk/L), both
// unnormalized.  Must be called by all threads of the block.
template <typename R>
__device__ cplx<R>* stockham(cplx<R>* A, cplx<R>* B, int L, int P, const cplx<R>* tw,
                             bool inverse) {
  const int log2L = ilog2(L);
  cplx<R>* src = A;
  cplx<R>* dst = B;
  int Ns = 1;
  int rem = log2L;
  const int Q = L >> 2;
  const int qshift = log2L - 2;
  while (rem >= 2) {
    const int step = L / (4 * Ns);
    for (int b = threadIdx.x; b < P * Q; b += kBlock) {
      const int p = b >> qshift;
      const int j = b & (Q - 1);
      const int k = j & (Ns - 1);
      const cplx<R>* s = src + p * L;
      cplx<R> a0 = s[j], a1 = s[j + Q], a2 = s[j + 2 * Q], a3 = s[j + 3 * Q];
      if (Ns > 1) {
        const int i1 = k * step;
        cplx<R> w1 = tw[i1], w2 = tw[2 * i1], w3 = tw[3 * i1];
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
    __syncthreads();
    cplx<R>* t = src;
    src = dst;
    dst = t;
    Ns *= 4;
    rem -= 2;
  }
  if (rem == 1) {
    const int H = L >> 1;
    const int hshift = log2L - 1;
    const int step = L / (2 * Ns);
    for (int b = threadIdx.x; b < P * H; b += kBlock) {
      const int p = b >> hshift;
      const int j = b & (H - 1);
      const int k = j & (Ns - 1);
      const cplx<R>* s = src + p * L;
      cplx<R> w = tw[k * step];
      if (inverse) w.y = -w.y;
      const cplx<R> a0 = s[j];
      const cplx<R> a1 = cmul(s[j + H], w);
      cplx<R>* d = dst + p * L + (j - k) * 2 + k;
      d[0] = cadd(a0, a1);
      d[Ns] = csub(a0, a1);
    }
    __syncthreads();
    src = dst;
  }
  return src;
}

template <typename R>
__device__ __forceinline__ R table_value(const Multiplier& mu, long prob, int d, int N, int k0, int k1, int k2) {
  const int H = N / 2 + 1;
  const int a0 = abs(k0), a1 = abs(k1), a2 = abs(k2);
  long idx = a0;
  if (d >= 2) idx = idx * H + a1;
  if (d >= 3) idx = idx * H + a2;
  return reinterpret_cast<const R*>(mu.tab)[prob * mu.tab_stride + idx];
}

template <typename R>
__device__ __forceinline__ cplx<R> apply_multiplier(cplx<R> v, const Multiplier& mu, long prob, int d, int N, int k0,
                                                   int k1, int k2) {
  const R m = table_value<R>(mu, prob, d, N, k0, k1, k2);
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
__host__ __device__ inline int rows_pencils(int L) {
  return L >= 1024 ? 1 : 1024 / L;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void rows_kernel(RowArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  const int P = rows_pencils<R>(L);
  cplx<R>* A = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* B = A + P * L;
  // twiddles staged in LDS (read by every pass) when they fit
  const cplx<R>* tw = a.tw;
  if (a.tw_lds) {
    cplx<R>* t = B + P * L;
    for (int i = threadIdx.x; i < L; i += kBlock) t[i] = a.tw[i];
    tw = t;
  }
  const int K0 = a.N / 2 + 1;
  const long row0 = long(blockIdx.x) * 2 * P;
  const int lshift = ilog2(L);

  if (a.mode == ROW_R2C || a.mode == ROW_FUSED1D) {
    const R* src = a.mode == ROW_R2C ? a.real_io : a.real_in;
    for (int i = threadIdx.x; i < 2 * P * L; i += kBlock) {
      const int r = i >> lshift;
      const int c = i & (L - 1);
      const long row = row0 + r;
      R v = R(0);
      if (row < a.nrows) {
        v = src[row * L + c];
        if (a.zero_src) const_cast<R*>(src)[row * L + c] = R(0);
      }
      cplx<R>* e = A + (r >> 1) * L + c;
      if (r & 1) e->y = v;
      else e->x = v;
    }
    __syncthreads();
    cplx<R>* res = stockham(A, B, L, P, tw, false);
    if (a.mode == ROW_R2C) {
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
      return;
    }
    // FUSED1D: each row is one problem; pencil p packs rows a = row0+2p and
    // b = a+1 as Z = A + iB.  With real even tables Da, Db the product
    // Da A + i Db B is ((Da+Db)/2) Z_k + ((Da-Db)/2) conj(Z_{-k}) (zero outside
    // the symmetric set I_N, boundary weights in the tables), times i 2 pi k for
    // a derivative.
    cplx<R>* other = res == A ? B : A;
    for (int i = threadIdx.x; i < P * L; i += kBlock) {
      const int p = i >> lshift;
      const int j = i & (L - 1);
      const int kk = j <= L / 2 ? j : j - L;
      cplx<R> v{R(0), R(0)};
      if (abs(kk) <= a.N / 2) {
        const long ra = row0 + 2 * p;
        const R da = ra < a.nrows ? table_value<R>(a.mul, ra, 1, a.N, kk, 0, 0) : R(0);
        const R db = ra + 1 < a.nrows ? table_value<R>(a.mul, ra + 1, 1, a.N, kk, 0, 0) : R(0);
        const cplx<R> z = res[i];
        const cplx<R> zm = cconj(res[p * L + ((L - j) & (L - 1))]);
        const R sp = R(0.5) * (da + db), sm = R(0.5) * (da - db);
        v = cplx<R>{sp * z.x + sm * zm.x, sp * z.y + sm * zm.y};
        if (a.mul.deriv >= 0) {
          const R f = R(6.283185307179586476925286766559) * R(kk);
          v = cplx<R>{-v.y * f, v.x * f};
        }
      }
      other[i] = v;
    }
    __syncthreads();
    cplx<R>* out = stockham(other, res, L, P, tw, true);
    for (int i = threadIdx.x; i < 2 * P * L; i += kBlock) {
      const int r = i >> lshift;
      const int c = i & (L - 1);
      const long row = row0 + r;
      if (row < a.nrows) {
        const cplx<R> v = out[(r >> 1) * L + c];
        a.real_io[row * L + c] = (r & 1) ? v.y : v.x;
      }
    }
    return;
  }

  // ROW_C2R: Z = A + i B on k = 0..N/2 and its Hermitian mirror on L - k
  for (int i = threadIdx.x; i < P * L; i += kBlock) {
    const int p = i >> lshift;
    const int j = i & (L - 1);
    const long ra = row0 + 2 * p;
    cplx<R> Z{R(0), R(0)};
    int k = -1;
    bool mirror = false;
    if (j < K0) k = j;
    else if (L - j < K0) {
      k = L - j;
      mirror = true;
    }
    if (k >= 0) {
      cplx<R> Av{R(0), R(0)}, Bv{R(0), R(0)};
      if (ra < a.nrows) Av = a.spec[ra * K0 + k];
      if (ra + 1 < a.nrows) Bv = a.spec[(ra + 1) * K0 + k];
      if (mirror) {
        Av.y = -Av.y;
        Bv.y = -Bv.y;
      }
      Z = cplx<R>{Av.x - Bv.y, Av.y + Bv.x};
    }
    A[i] = Z;
  }
  __syncthreads();
  cplx<R>* out = stockham(A, B, L, P, tw, true);
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

template <typename R>
__host__ __device__ inline int axis_pencils(int L) {
  return L >= 1024 ? 1 : 1024 / L;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void axis_kernel(AxisArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  const int P = axis_pencils<R>(L);
  cplx<R>* A = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* B = A + P * L;
  // twiddles staged in LDS (read by every pass) when they fit
  const cplx<R>* tw = a.tw;
  if (a.tw_lds) {
    cplx<R>* t = B + P * L;
    for (int i = threadIdx.x; i < L; i += kBlock) t[i] = a.tw[i];
    tw = t;
  }
  const long q0 = long(blockIdx.x) * P;
  const int half = a.N / 2;

  if (a.mode == AX_INV || a.nin < L) {
    for (int i = threadIdx.x; i < P * L; i += kBlock) A[i] = cplx<R>{R(0), R(0)};
    __syncthreads();
  }
  for (int i = threadIdx.x; i < P * a.nin; i += kBlock) {
    const int p = i % P;
    const int e = i / P;
    const long q = q0 + p;
    if (q >= a.npen) continue;
    const long o = q / a.inner;
    const long ii = q - o * a.inner;
    cplx<R> v = a.in[o * a.in_ostride + ii + e * a.in_stride];
    int bin = e;
    if (a.in_centered) {
      const int k = e - half;
      bin = k < 0 ? k + L : k;
      if (a.mode == AX_INV && a.apply_mul) {
        int k1 = 0, k2 = 0;
        if (a.d == 2) k1 = int(ii);
        else if (a.d == 3) {
          const int K0 = half + 1;
          k1 = int(ii / K0) - half;
          k2 = int(ii % K0);
        }
        v = apply_multiplier(v, a.mul, o, a.d, a.N, k, k1, k2);
      }
    }
    A[p * L + bin] = v;
  }
  __syncthreads();

  cplx<R>* res;
  if (a.mode == AX_INV) {
    res = stockham(A, B, L, P, tw, true);
  } else {
    res = stockham(A, B, L, P, tw, false);
    if (a.mode == AX_FUSED) {
      for (int i = threadIdx.x; i < P * L; i += kBlock) {
        const int p = i / L;
        const int bin = i - p * L;
        const int k0 = bin <= L / 2 ? bin : bin - L;
        const long q = q0 + p;
        cplx<R> v{R(0), R(0)};
        if (abs(k0) <= half && q < a.npen) {
          const long o = q / a.inner;
          const long ii = q - o * a.inner;
          int k1 = 0, k2 = 0;
          if (a.d == 2) k1 = int(ii);
          else if (a.d == 3) {
            const int K0 = half + 1;
            k1 = int(ii / K0) - half;
            k2 = int(ii % K0);
          }
          v = apply_multiplier(res[i], a.mul, o, a.d, a.N, k0, k1, k2);
        }
        res[i] = v;
      }
      __syncthreads();
      cplx<R>* other = res == A ? B : A;
      res = stockham(res, other, L, P, tw, true);
    }
  }

  for (int i = threadIdx.x; i < P * a.nout; i += kBlock) {
    const int p = i % P;
    const int e = i / P;
    const long q = q0 + p;
    if (q >= a.npen) continue;
    const long o = q / a.inner;
    const long ii = q - o * a.inner;
    int bin = e;
    if (a.out_centered) {
      const int k = e - half;
      bin = k < 0 ? k + L : k;
    }
    a.out[o * a.out_ostride + ii + e * a.out_stride] = res[p * L + bin];
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

template <typename R>
hipError_t launch_rows(const RowArgs<R>& a_in, hipStream_t st) {
  RowArgs<R> a = a_in;
  const int P = rows_pencils<R>(a.L);
  const long nblk = (a.nrows + 2 * P - 1) / (2 * P);
  const size_t shm = fft_lds<R>(P, a.L, &a.tw_lds);
  hipLaunchKernelGGL(rows_kernel<R>, dim3(nblk), dim3(kBlock), shm, st, a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_axis(const AxisArgs<R>& a_in, hipStream_t st) {
  AxisArgs<R> a = a_in;
  const int P = axis_pencils<R>(a.L);
  const long nblk = (a.npen + P - 1) / P;
  const size_t shm = fft_lds<R>(P, a.L, &a.tw_lds);
  hipLaunchKernelGGL(axis_kernel<R>, dim3(nblk), dim3(kBlock), shm, st, a);
  return hipGetLastError();
}

template hipError_t launch_rows<float>(const RowArgs<float>&, hipStream_t);
template hipError_t launch_rows<double>(const RowArgs<double>&, hipStream_t);
template hipError_t launch_axis<float>(const AxisArgs<float>&, hipStream_t);
template hipError_t launch_axis<double>(const AxisArgs<double>&, hipStream_t);

}  // namespace nfs
