// Near-field correction of fast summation for the non-smooth kernels
// exp(-r^rho/eps), rho = 1 or a real rho (Section 3.1: the regularized kernel
// K_R replaces the kernel inside the near-field radius eps_I, and the sum over
// close pairs adds K - K_R back), with its gradient for rho = 1.
//
// The kernels are templates over the form of the kernel (rho = 1, a real rho,
// or the primal cost's kernel |z|^rho exp(-|z|^rho/eps)); each form is compiled
// in its own translation unit (nearfield_r1.hip, nearfield_real.hip,
// nearfield_cost.hip), so the rho = 1 instances carry none of the others' code.
#pragma once

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace nfs {

// --------------------------------------------------------------------------- near field
// One workgroup per target chunk (at most kNearTargets targets, kept in
// registers, kNearTPT per thread); sources of each neighbour tile are staged
// through LDS in batches of kBlock.  Distances are taken in grid cells
// relative to the target tile's origin, so they stay small and exact enough
// in FP32.
constexpr int kNearTPT = 4;
constexpr int kNearTargets = kNearTPT * kBlock;

// The kernel K(r) of a pair from its squared cell distance r2 is written out
// at each use, rho = 1 in the exact form the compiler has register-allocated
// well (a helper function for it cost six more VGPRs in the cell-culled
// kernel, one wave per SIMD less for some shapes):
//   rho = 1, FP32: exp(-r/eps) = exp2(r (-log2(e)/eps)) on the hardware exp2
//     and square root (about 1 ulp each); FP64: exp(-sqrt(r2)/eps).
//   real rho: exp(-r^rho/eps) with r^rho = r2^(rho/2) = exp2((rho/2) log2 r2)
//     (hardware log2 and exp2 in FP32, pow in FP64; r2 = 0 gives K = 1).
template <typename R, int D, int PS, int FORM>
__global__ __launch_bounds__(kBlock) void nearfield_kernel(NearArgs<R> a) {
  __shared__ R su[D][kBlock];
  __shared__ R sw[kBlock];
  const Geom geo = a.geo;
  const Chunk ch = a.tchunks[blockIdx.x];
  if (a.pstate && a.pstate[kPState * ch.prob] == 2) return;  // the problem has stopped
  const int pb = ch.prob;
  const int nbins = geo.nt[0] * geo.nt[1] * geo.nt[2];
  const double* cf = a.coef + size_t(pb) * kNearStride;
  const R inv_e = R(cf[0]), ei2 = R(cf[1]), inv_ei2 = R(cf[2]);
  // FP32: exp(-r/eps) = exp2(r * (-log2(e)/eps)) on the hardware exp2 and
  // square root (about 1 ulp each; the correctly rounded sqrtf costs a dozen
  // more instructions per pair)
  const float nle = float(-cf[0] * 1.4426950408889634);
  // real exponent rho: exp(-r^rho/eps) = exp2(r2^(rho/2) * (-log2(e)/(eps g^rho)))
  const R hr = R(cf[kNearRhoHalf]), inv_er = R(cf[kNearRhoInv]);
  const float nler = float(-cf[kNearRhoInv] * 1.4426950408889634);
  const R cmul = R(cf[kNearCostMul]);
  R c[PS];
#pragma unroll
  for (int j = 0; j < PS; ++j) c[j] = R(cf[4 + j]);
  const double wm = a.wconst * (a.wmul ? a.wmul[pb] : 1.0);

  int tc[3] = {0, 0, 0};
  {
    int t = ch.tile;
    for (int k = D - 1; k >= 0; --k) {
      tc[k] = t % geo.nt[k];
      t /= geo.nt[k];
    }
  }
  R ut[kNearTPT][D];
  R acc[kNearTPT];
#pragma unroll
  for (int k = 0; k < kNearTPT; ++k) {
    acc[k] = R(0);
    const int q = ch.start + threadIdx.x + k * kBlock;
#pragma unroll
    for (int cc = 0; cc < D; ++cc)
      ut[k][cc] = (q < ch.start + ch.count) ? a.tcoords[size_t(q) * D + cc] : R(1e30);
  }
  const int span = 2 * a.kt + 1;
  int nnb = 1;
  for (int k = 0; k < D; ++k) nnb *= span;
  for (int nbi = 0; nbi < nnb; ++nbi) {
    int rem = nbi, tile = 0;
    R shift[3] = {R(0), R(0), R(0)};
    for (int k = 0; k < D; ++k) {
      const int dl = rem % span - a.kt;
      rem /= span;
      int t = tc[k] + dl;
      t = ((t % geo.nt[k]) + geo.nt[k]) % geo.nt[k];
      tile = tile * geo.nt[k] + t;
      shift[k] = R(dl * geo.T);
    }
    const int so = a.soffsets[size_t(pb) * nbins + tile];
    const int sc = a.scounts[size_t(pb) * nbins + tile];
    for (int s0 = 0; s0 < sc; s0 += kBlock) {
      const int nb = min(kBlock, sc - s0);
      __syncthreads();
      if (threadIdx.x < nb) {
        const int j = so + s0 + threadIdx.x;
#pragma unroll
        for (int cc = 0; cc < D; ++cc) su[cc][threadIdx.x] = a.scoords[size_t(j) * D + cc] + shift[cc];
        sw[threadIdx.x] = R(a.sw[j] * wm);
      }
      __syncthreads();
      for (int j = 0; j < nb; ++j) {
        R ys[D];
#pragma unroll
        for (int cc = 0; cc < D; ++cc) ys[cc] = su[cc][j];
        const R wj = sw[j];
#pragma unroll
        for (int k = 0; k < kNearTPT; ++k) {
          R r2 = R(0);
#pragma unroll
          for (int cc = 0; cc < D; ++cc) {
            const R dz = ut[k][cc] - ys[cc];
            r2 += dz * dz;
          }
          if (r2 < ei2) {
            const R rho2 = r2 * inv_ei2;
            R P = c[PS - 1];
#pragma unroll
            for (int jj = PS - 2; jj >= 0; --jj) P = P * rho2 + c[jj];
            if constexpr (FORM == kNearCost) {
              if constexpr (sizeof(R) == 4) {
                const R rr = __builtin_amdgcn_exp2f(hr * __builtin_amdgcn_logf(r2));
                acc[k] += wj * (rr * cmul * __builtin_amdgcn_exp2f(rr * nler) - P);
              } else {
                const R rr = pow(r2, hr);
                acc[k] += wj * (rr * cmul * exp(-rr * inv_er) - P);
              }
            } else if constexpr (FORM == kNearReal) {
              if constexpr (sizeof(R) == 4)
                acc[k] += wj * (__builtin_amdgcn_exp2f(__builtin_amdgcn_exp2f(hr * __builtin_amdgcn_logf(r2)) * nler) - P);
              else
                acc[k] += wj * (exp(-pow(r2, hr) * inv_er) - P);
            } else if constexpr (sizeof(R) == 4)
              acc[k] += wj * (__builtin_amdgcn_exp2f(__builtin_amdgcn_sqrtf(r2) * nle) - P);
            else
              acc[k] += wj * (exp(-sqrt(r2) * inv_e) - P);
          }
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kNearTPT; ++k) {
    const int q = ch.start + threadIdx.x + k * kBlock;
    if (q < ch.start + ch.count) a.out[q] = double(acc[k]);
  }
}

// Gradient of the near-field sum at the targets: for every target,
//   out[c * plane + q] = sum_{sources j within eps_I} w_j wm d/dx'_c (K - K_R)(x'_q - y'_j),
// the derivative in torus units (x' = g x_cells).  With z the target-source
// offset in cells, r = |z| and u = r^2 / eps_I^2 (cells),
//   grad (K - K_R) = -g [k'(r) + 2 inv_ei2 sum_{j>=1} j c_j u^{j-1}] z,
//   rho = 1:  k'(r) = inv_e e^{-r inv_e} / r,
//   real rho: k'(r) = rho inv_er r^(rho-2) e^{-r^rho inv_er}  (inv_er = coef[kNearRhoInv]),
// the first term taken as 0 at r = 0 (the cost's gradient is zero where the
// points coincide; r^(rho-1) -> 0 there for rho > 1).  Same tiling as nearfield_kernel.
template <typename R, int D, int PS, int FORM>
__global__ __launch_bounds__(kBlock) void nearfield_grad_kernel(NearArgs<R> a) {
  __shared__ R su[D][kBlock];
  __shared__ R sw[kBlock];
  const Geom geo = a.geo;
  const Chunk ch = a.tchunks[blockIdx.x];
  const int pb = ch.prob;
  const int nbins = geo.nt[0] * geo.nt[1] * geo.nt[2];
  const double* cf = a.coef + size_t(pb) * kNearStride;
  const R inv_e = R(cf[0]), ei2 = R(cf[1]), inv_ei2 = R(cf[2]);
  const R hr = R(cf[kNearRhoHalf]), inv_er = R(cf[kNearRhoInv]);
  // derivative coefficients j c_j of the inner polynomial, in rho
  R dc[PS > 1 ? PS - 1 : 1];
#pragma unroll
  for (int j = 1; j < PS; ++j) dc[j - 1] = R(double(j) * cf[4 + j]);
  const double wm = a.wconst * (a.wmul ? a.wmul[pb] : 1.0);

  int tc[3] = {0, 0, 0};
  {
    int t = ch.tile;
    for (int k = D - 1; k >= 0; --k) {
      tc[k] = t % geo.nt[k];
      t /= geo.nt[k];
    }
  }
  R ut[kNearTPT][D];
  R acc[kNearTPT][D];
#pragma unroll
  for (int k = 0; k < kNearTPT; ++k) {
    const int q = ch.start + threadIdx.x + k * kBlock;
#pragma unroll
    for (int cc = 0; cc < D; ++cc) {
      acc[k][cc] = R(0);
      ut[k][cc] = (q < ch.start + ch.count) ? a.tcoords[size_t(q) * D + cc] : R(1e30);
    }
  }
  const int span = 2 * a.kt + 1;
  int nnb = 1;
  for (int k = 0; k < D; ++k) nnb *= span;
  for (int nbi = 0; nbi < nnb; ++nbi) {
    int rem = nbi, tile = 0;
    R shift[3] = {R(0), R(0), R(0)};
    for (int k = 0; k < D; ++k) {
      const int dl = rem % span - a.kt;
      rem /= span;
      int t = tc[k] + dl;
      t = ((t % geo.nt[k]) + geo.nt[k]) % geo.nt[k];
      tile = tile * geo.nt[k] + t;
      shift[k] = R(dl * geo.T);
    }
    const int so = a.soffsets[size_t(pb) * nbins + tile];
    const int sc = a.scounts[size_t(pb) * nbins + tile];
    for (int s0 = 0; s0 < sc; s0 += kBlock) {
      const int nb = min(kBlock, sc - s0);
      __syncthreads();
      if (threadIdx.x < nb) {
        const int j = so + s0 + threadIdx.x;
#pragma unroll
        for (int cc = 0; cc < D; ++cc) su[cc][threadIdx.x] = a.scoords[size_t(j) * D + cc] + shift[cc];
        sw[threadIdx.x] = R(a.sw[j] * wm);
      }
      __syncthreads();
      for (int j = 0; j < nb; ++j) {
        const R wj = sw[j];
#pragma unroll
        for (int k = 0; k < kNearTPT; ++k) {
          R z[D];
          R r2 = R(0);
#pragma unroll
          for (int cc = 0; cc < D; ++cc) {
            z[cc] = ut[k][cc] - su[cc][j];
            r2 += z[cc] * z[cc];
          }
          if (r2 < ei2) {
            const R rho = r2 * inv_ei2;
            R dP = PS > 1 ? dc[PS - 2] : R(0);
#pragma unroll
            for (int jj = PS - 3; jj >= 0; --jj) dP = dP * rho + dc[jj];
            R ek;
            if constexpr (FORM == kNearReal) {
              // r^rho = r2^(rho/2); k'(r) = rho inv_er (r^rho / r2) e^{-r^rho inv_er}
              const R rr = r2 > R(0) ? pow(r2, hr) : R(0);
              ek = r2 > R(0) ? R(2) * hr * inv_er * (rr / r2) * exp(-rr * inv_er) : R(0);
            } else {
              const R r = sqrt(r2);
              ek = r > R(0) ? inv_e * exp(-r * inv_e) / r : R(0);
            }
            const R h = wj * (ek + R(2) * inv_ei2 * dP);
#pragma unroll
            for (int cc = 0; cc < D; ++cc) acc[k][cc] += h * z[cc];
          }
        }
      }
    }
  }
  const R ng = -R(geo.g);
#pragma unroll
  for (int k = 0; k < kNearTPT; ++k) {
    const int q = ch.start + threadIdx.x + k * kBlock;
    if (q < ch.start + ch.count)
#pragma unroll
      for (int cc = 0; cc < D; ++cc) a.out[size_t(cc) * a.out_plane + q] = double(ng * acc[k][cc]);
  }
}

// The same near-field sum with the sources chosen per cell.  Each wave takes
// its kNearTPT groups of 64 consecutive targets (cell order, so each group is
// compact) one at a time and reduces the group's bounding box.  The source
// cells that can hold a source within eps_I of that box form rows along the
// last axis; a row is one contiguous source range per tile (sources are sorted
// by cell inside their tile, `scell` holds each cell's first position).
//   - The rows (and their tile pieces) are enumerated 64 at a time, one per
//     lane, so the bound look-ups of 64 pieces share one memory latency.
//   - A wave scan packs the sources of those pieces into batches of 64; each
//     lane finds its source's piece by binary search over the 64 prefix sums,
//     loads it (one coalesced load per batch) into the wave's LDS slice, and
//     the wave reads the batch back as broadcasts.
// The pair test and correction are those of nearfield_kernel.
template <typename R>
struct NearSrc {
  R c[3];
  R w;
};

__device__ __forceinline__ int floor_div(int c, int T) { return c >= 0 ? c / T : -((-c + T - 1) / T); }

template <typename R>
__device__ __forceinline__ R wave_min(R v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
template <typename R>
__device__ __forceinline__ R wave_max(R v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

template <typename R, int D, int PS, int FORM>
__global__ __launch_bounds__(kBlock) void nearfield_cells_kernel(NearArgs<R> a) {
  __shared__ NearSrc<R> sbuf[kBlock];
  __shared__ int spre[kBlock];  // per wave: inclusive prefix of the round's piece lengths
  const int lane = threadIdx.x & 63;
  const int wbase = threadIdx.x & ~63;
  NearSrc<R>* wb = sbuf + wbase;
  int* wp = spre + wbase;
  const Geom geo = a.geo;
  const Chunk ch = a.tchunks[blockIdx.x];
  if (a.pstate && a.pstate[kPState * ch.prob] == 2) return;  // the problem has stopped
  const int pb = ch.prob;
  const int T = geo.T;
  const int nbins = geo.nt[0] * geo.nt[1] * geo.nt[2];
  int nc = 1;
  for (int k = 0; k < D; ++k) nc *= T;
  const double* cf = a.coef + size_t(pb) * kNearStride;
  const R inv_e = R(cf[0]), ei2 = R(cf[1]), inv_ei2 = R(cf[2]);
  const float nle = float(-cf[0] * 1.4426950408889634);
  const R hr = R(cf[kNearRhoHalf]), inv_er = R(cf[kNearRhoInv]);
  const float nler = float(-cf[kNearRhoInv] * 1.4426950408889634);
  const R cmul = R(cf[kNearCostMul]);
  R c[PS];
#pragma unroll
  for (int j = 0; j < PS; ++j) c[j] = R(cf[4 + j]);
  const double wm = a.wconst * (a.wmul ? a.wmul[pb] : 1.0);
  // cell ranges relative to the target tile stay inside the (2 kt + 1)^D neighbour tiles
  const int kt = a.kt, span = 2 * kt + 1;
  const int cmin = -kt * T, cmax = T - 1 + kt * T;
  const R ei = sqrt(ei2);
  const R margin = R(1e-3);  // cells; guards the range bounds against rounding

  int tc[3] = {0, 0, 0};
  {
    int t = ch.tile;
    for (int k = D - 1; k >= 0; --k) {
      tc[k] = t % geo.nt[k];
      t /= geo.nt[k];
    }
  }

#pragma unroll
  for (int k = 0; k < kNearTPT; ++k) {
    const int q = ch.start + threadIdx.x + k * kBlock;
    const bool valid = q < ch.start + ch.count;
    R u[D], lo[D], hi[D];
#pragma unroll
    for (int cc = 0; cc < D; ++cc) {
      u[cc] = valid ? a.tcoords[size_t(q) * D + cc] : R(1e30);
      lo[cc] = wave_min(valid ? u[cc] : R(1e30));
      hi[cc] = wave_max(valid ? u[cc] : R(-1e30));
    }
    R acc = R(0);
    if (lo[0] <= hi[0]) {
      // rows: cells of the axes before the last inside the box grown by eps_I,
      // times the span tile pieces of the last axis
      int rlo[3] = {0, 0, 0}, rn[3] = {1, 1, 1};
      int nrows = span;
#pragma unroll
      for (int cc = 0; cc < D - 1; ++cc) {
        rlo[cc] = max(cmin, int(floor(lo[cc] - ei - margin)));
        rn[cc] = min(cmax, int(floor(hi[cc] + ei + margin))) - rlo[cc] + 1;
        nrows *= rn[cc];
      }
      for (int r0 = 0; r0 < nrows; r0 += 64) {
        // this lane's piece: [beg, end) of one source tile, and its shift
        int beg = 0, len = 0, packed = 0;
        const int row = r0 + lane;
        if (row < nrows) {
          int rest = row;
          const int piece = rest % span;
          rest /= span;
          int cidx[3] = {0, 0, 0};
          R rem = ei2;
#pragma unroll
          for (int cc = D - 2; cc >= 0; --cc) {
            cidx[cc] = rlo[cc] + rest % rn[cc];
            rest /= rn[cc];
          }
#pragma unroll
          for (int cc = 0; cc < D - 1; ++cc) {
            const R g = fmax(R(0), fmax(R(cidx[cc]) - hi[cc], lo[cc] - R(cidx[cc] + 1)));
            rem -= g * g;
          }
          const int dlast = piece - kt;
          if (rem > R(0)) {
            const R rad = sqrt(rem);
            const int A = max(max(cmin, dlast * T), int(floor(lo[D - 1] - rad - margin)));
            const int B = min(min(cmax, dlast * T + T - 1), int(floor(hi[D - 1] + rad + margin)));
            if (A <= B) {
              int tile = 0, cell = 0;
              int dl[3];
#pragma unroll
              for (int cc = 0; cc < D; ++cc) {
                dl[cc] = cc < D - 1 ? floor_div(cidx[cc], T) : dlast;
                int t = tc[cc] + dl[cc];
                t = ((t % geo.nt[cc]) + geo.nt[cc]) % geo.nt[cc];
                tile = tile * geo.nt[cc] + t;
                if (cc < D - 1) cell = cell * T + (cidx[cc] - dl[cc] * T);
              }
              const size_t tix = size_t(pb) * nbins + tile;
              const int* cst = a.scell + tix * (nc + 1);
              const int base = a.soffsets[tix];
              beg = base + cst[cell * T + (A - dlast * T)];
              len = base + cst[cell * T + (B - dlast * T) + 1] - beg;
              // tile offsets in [-kt, kt], packed 8 bits per axis
              for (int cc = 0; cc < D; ++cc) packed |= (dl[cc] + 128) << (8 * cc);
            }
          }
        }
        const int incl = wave_incl_scan(len, lane);
        const int total = __shfl(incl, 63);
        if (total == 0) continue;
        __builtin_amdgcn_wave_barrier();
        wp[lane] = incl;
        __builtin_amdgcn_wave_barrier();
        for (int f0 = 0; f0 < total; f0 += 64) {
          const int cnt = min(64, total - f0);
          __builtin_amdgcn_wave_barrier();
          // the piece holding flat index f: the first lane whose inclusive
          // prefix exceeds f (all lanes search and shuffle, so every source
          // lane of the shuffles is active; lanes past cnt repeat the last f)
          const int f = f0 + min(lane, cnt - 1);
          int lo_l = 0, hi_l = 63;
          while (lo_l < hi_l) {
            const int mid = (lo_l + hi_l) >> 1;
            if (wp[mid] > f) hi_l = mid;
            else lo_l = mid + 1;
          }
          const int pbeg = __shfl(beg, lo_l), ppk = __shfl(packed, lo_l);
          const int prev = lo_l > 0 ? wp[lo_l - 1] : 0;
          if (lane < cnt) {
            const int j = pbeg + (f - prev);
            NearSrc<R> rec;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
              const int dlc = ((ppk >> (8 * cc)) & 255) - 128;
              rec.c[cc] = cc < D ? a.scoords[size_t(j) * D + cc] + R(dlc * T) : R(0);
            }
            rec.w = R(a.sw[j] * wm);
            wb[lane] = rec;
          }
          __builtin_amdgcn_wave_barrier();
          // Branch free: about half of the candidates are within eps_I, so
          // nearly every wave would take the branch anyway; the select drops
          // the others (their sqrt, exp2 and polynomial stay finite or are
          // discarded).  Four records are read before they are used.
          auto pair = [&](const NearSrc<R>& sr) {
            R r2 = R(0);
#pragma unroll
            for (int cc = 0; cc < D; ++cc) {
              const R dz = u[cc] - sr.c[cc];
              r2 += dz * dz;
            }
            const R rho2 = r2 * inv_ei2;
            R P = c[PS - 1];
#pragma unroll
            for (int jj2 = PS - 2; jj2 >= 0; --jj2) P = P * rho2 + c[jj2];
            R e;
            if constexpr (FORM == kNearCost) {
              if constexpr (sizeof(R) == 4) {
                const R rr = __builtin_amdgcn_exp2f(hr * __builtin_amdgcn_logf(r2));
                e = rr * cmul * __builtin_amdgcn_exp2f(rr * nler);
              } else {
                const R rr = pow(r2, hr);
                e = rr * cmul * exp(-rr * inv_er);
              }
            } else if constexpr (FORM == kNearReal) {
              if constexpr (sizeof(R) == 4)
                e = __builtin_amdgcn_exp2f(__builtin_amdgcn_exp2f(hr * __builtin_amdgcn_logf(r2)) * nler);
              else
                e = exp(-pow(r2, hr) * inv_er);
            } else if constexpr (sizeof(R) == 4)
              e = __builtin_amdgcn_exp2f(__builtin_amdgcn_sqrtf(r2) * nle);
            else
              e = exp(-sqrt(r2) * inv_e);
            acc += r2 < ei2 ? sr.w * (e - P) : R(0);
          };
          int jj = 0;
          for (; jj + 4 <= cnt; jj += 4) {
            const NearSrc<R> s0 = wb[jj], s1 = wb[jj + 1], s2 = wb[jj + 2], s3 = wb[jj + 3];
            pair(s0);
            pair(s1);
            pair(s2);
            pair(s3);
          }
          for (; jj < cnt; ++jj) pair(wb[jj]);
        }
      }
    }
    if (valid) a.out[q] = double(acc);
  }
}

#define NFS_NEAR_P(KERNEL, D_)                                                                                       \
  switch (a.ps) {                                                                                          \
    case 2: hipLaunchKernelGGL((KERNEL<R, D_, 2, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break;   \
    case 3: hipLaunchKernelGGL((KERNEL<R, D_, 3, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break;   \
    case 4: hipLaunchKernelGGL((KERNEL<R, D_, 4, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break;   \
    case 5: hipLaunchKernelGGL((KERNEL<R, D_, 5, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break;   \
    case 6: hipLaunchKernelGGL((KERNEL<R, D_, 6, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break;   \
    case 7: hipLaunchKernelGGL((KERNEL<R, D_, 7, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break;   \
    case 8: hipLaunchKernelGGL((KERNEL<R, D_, 8, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break;   \
    case 9: hipLaunchKernelGGL((KERNEL<R, D_, 9, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break;   \
    case 10: hipLaunchKernelGGL((KERNEL<R, D_, 10, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break; \
    case 11: hipLaunchKernelGGL((KERNEL<R, D_, 11, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break; \
    case 12: hipLaunchKernelGGL((KERNEL<R, D_, 12, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break; \
    case 13: hipLaunchKernelGGL((KERNEL<R, D_, 13, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break; \
    case 14: hipLaunchKernelGGL((KERNEL<R, D_, 14, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break; \
    case 15: hipLaunchKernelGGL((KERNEL<R, D_, 15, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break; \
    case 16: hipLaunchKernelGGL((KERNEL<R, D_, 16, FORM>), dim3(nchunks), dim3(kBlock), 0, st, a); break; \
    default: return hipErrorInvalidValue;                                                                  \
  }

// The near-field sum in one form (FORM: kNearR1, kNearReal or kNearCost),
// instantiated by nearfield_r1.hip and nearfield_real.hip.
template <typename R, int FORM>
hipError_t launch_nearfield_form(const NearArgs<R>& a, int nchunks, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  // cell-culled sources when the plan left per-cell starts (sources in cell order)
  if (a.scell) {
    if (a.geo.d == 1) {
      NFS_NEAR_P(nearfield_cells_kernel, 1)
    } else if (a.geo.d == 2) {
      NFS_NEAR_P(nearfield_cells_kernel, 2)
    } else {
      NFS_NEAR_P(nearfield_cells_kernel, 3)
    }
  } else if (a.geo.d == 1) {
    NFS_NEAR_P(nearfield_kernel, 1)
  } else if (a.geo.d == 2) {
    NFS_NEAR_P(nearfield_kernel, 2)
  } else {
    NFS_NEAR_P(nearfield_kernel, 3)
  }
  return hipGetLastError();
}
extern template hipError_t launch_nearfield_form<float, kNearR1>(const NearArgs<float>&, int, hipStream_t);
extern template hipError_t launch_nearfield_form<double, kNearR1>(const NearArgs<double>&, int, hipStream_t);
extern template hipError_t launch_nearfield_form<float, kNearReal>(const NearArgs<float>&, int, hipStream_t);
extern template hipError_t launch_nearfield_form<double, kNearReal>(const NearArgs<double>&, int, hipStream_t);
extern template hipError_t launch_nearfield_form<float, kNearCost>(const NearArgs<float>&, int, hipStream_t);
extern template hipError_t launch_nearfield_form<double, kNearCost>(const NearArgs<double>&, int, hipStream_t);

// Its gradient in one exponent form, instantiated like the sum.
template <typename R, int FORM>
hipError_t launch_nearfield_grad_form(const NearArgs<R>& a, int nchunks, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  if (a.geo.d == 1) {
    NFS_NEAR_P(nearfield_grad_kernel, 1)
  } else if (a.geo.d == 2) {
    NFS_NEAR_P(nearfield_grad_kernel, 2)
  } else {
    NFS_NEAR_P(nearfield_grad_kernel, 3)
  }
  return hipGetLastError();
}
extern template hipError_t launch_nearfield_grad_form<float, kNearR1>(const NearArgs<float>&, int, hipStream_t);
extern template hipError_t launch_nearfield_grad_form<double, kNearR1>(const NearArgs<double>&, int, hipStream_t);
extern template hipError_t launch_nearfield_grad_form<float, kNearReal>(const NearArgs<float>&, int, hipStream_t);
extern template hipError_t launch_nearfield_grad_form<double, kNearReal>(const NearArgs<double>&, int, hipStream_t);

}  // namespace nfs
