// Plan-stage kernels (bounding box, tile keys, counting-sort scatter) and the
// small elementwise / reduction kernels around the fast summation.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace nfs {

// ------------------------------------------------------------------ block helpers
template <int NV>
__device__ void block_reduce_arr(double (&v)[NV], const bool (&is_min)[NV], const bool (&is_max)[NV],
                                 double (*sh)[kBlock]) {
  for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      for (int k = 0; k < NV; ++k) {
        const double a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + s];
        sh[k][threadIdx.x] = is_min[k] ? fmin(a, b) : (is_max[k] ? fmax(a, b) : a + b);
      }
    }
    __syncthreads();
  }
  for (int k = 0; k < NV; ++k) v[k] = sh[k][0];
  __syncthreads();
}

// Writes this block's values to partials[blockIdx.x NV + k]; the
// finish_partials kernel launched after the kernel combines them.
template <int NV>
__device__ void grid_reduce_arr(double (&v)[NV], const bool (&is_min)[NV], const bool (&is_max)[NV],
                                double* partials) {
  __shared__ double sh[NV][kBlock];
  block_reduce_arr<NV>(v, is_min, is_max, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) partials[size_t(blockIdx.x) * NV + k] = v[k];
}

// Combines the nb partials of a grid reduction, in block order, into out[NV]:
// entry k is a min where bit k of min_mask is set, a max where it is set in
// max_mask, else a sum.  Launched right after the kernel that wrote them, so
// that the kernel boundary makes them visible.  (A fence and a ticket per
// workgroup, the last one combining, write the L2 back once per workgroup on
// a part with one L2 per XCD.)
template <int NV>
__global__ __launch_bounds__(kBlock) void finish_partials_kernel(const double* partials, int nb, unsigned min_mask,
                                                                 unsigned max_mask, double* out) {
  __shared__ double sh[NV][kBlock];
  bool is_min[NV], is_max[NV];
  double acc[NV];
  for (int k = 0; k < NV; ++k) {
    is_min[k] = (min_mask >> k) & 1u;
    is_max[k] = (max_mask >> k) & 1u;
    acc[k] = is_min[k] ? 1e308 : (is_max[k] ? -1e308 : 0.0);
  }
  for (int b = threadIdx.x; b < nb; b += kBlock)
    for (int k = 0; k < NV; ++k) {
      const double x = partials[size_t(b) * NV + k];
      acc[k] = is_min[k] ? fmin(acc[k], x) : (is_max[k] ? fmax(acc[k], x) : acc[k] + x);
    }
  block_reduce_arr<NV>(acc, is_min, is_max, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) out[k] = acc[k];
}

template <int NV>
static hipError_t finish_partials(const double* partials, int nb, unsigned min_mask, unsigned max_mask, double* out,
                                  hipStream_t st) {
  hipLaunchKernelGGL(finish_partials_kernel<NV>, dim3(1), dim3(kBlock), 0, st, partials, nb, min_mask, max_mask, out);
  return hipGetLastError();
}

// Per-entry kinds of the grid reductions below (bit k: entry k is a min / a max).
constexpr unsigned kBoxMin = 0x87u, kBoxMax = 0x78u;  // box: min_c (0-2), max_c (3-5), max|w|, min w (7)
constexpr unsigned kMaxSumMax = 0x1u;                 // maxsum: max, sum

constexpr int kGridBlocks = 1024;

// ------------------------------------------------------------------ bounding box
// out = {min_0..min_{d-1}, max_0..max_{d-1}} padded to 3 dims, then max|w|, min w, sum w,
// and with a.wsum the weighted coordinate sums of pts[0].
__global__ __launch_bounds__(kBlock) void bbox_kernel(BoxArgs a, const BoxJob* jobs, int njobs) {
  constexpr int NV = kBoxVals;
  long blk = blockIdx.x, nblk = gridDim.x;
  if (jobs) {
    // this workgroup's box: the last job whose first workgroup is at or before it
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].blk0 <= blk) lo = mid;
      else hi = mid - 1;
    }
    const int d = a.d;
    double* partials = a.partials;
    a = jobs[lo].box;
    a.d = d;
    a.partials = partials;
    blk -= jobs[lo].blk0;
    nblk = jobs[lo].nblk;
  }
  double v[NV];
  bool is_min[NV], is_max[NV];
  for (int k = 0; k < NV; ++k) {
    is_min[k] = (kBoxMin >> k) & 1u;
    is_max[k] = (kBoxMax >> k) & 1u;
    v[k] = is_min[k] ? 1e308 : (is_max[k] ? -1e308 : 0.0);
  }
  const long stride = nblk * kBlock;
  for (int s = 0; s < 2; ++s) {
    const double* p = a.pts[s];
    if (!p) continue;
    for (long i = blk * kBlock + threadIdx.x; i < a.n[s]; i += stride)
      for (int c = 0; c < a.d; ++c) {
        const double x = p[i * a.d + c];
        v[c] = fmin(v[c], x);
        v[3 + c] = fmax(v[3 + c], x);
      }
  }
  if (a.w)
    for (long i = blk * kBlock + threadIdx.x; i < a.nw; i += stride) {
      const double w = a.w[i];
      v[6] = fmax(v[6], fabs(w));
      v[7] = fmin(v[7], w);
      v[8] += w;
      if (a.wsum)
        for (int c = 0; c < a.d; ++c) v[9 + c] += w * a.pts[0][i * a.d + c];
    }
  grid_reduce_arr<NV>(v, is_min, is_max, a.partials);
}

// ------------------------------------------------------------------ centred form read-out
template <typename R>
__global__ __launch_bounds__(kBlock) void uncenter_kernel(UncenterArgs<R> a) {
  const Chunk ch = a.chunks[blockIdx.x];
  const Geom geo = a.geo;
  const double* pb = a.pb + size_t(kUncStride) * ch.prob;
  const double scale = pb[0], cst = pb[7], eps = pb[8];
  int org[3] = {0, 0, 0};
  {
    int t = ch.tile;
    for (int c = geo.d - 1; c >= 0; --c) {
      org[c] = (t % geo.nt[c]) * geo.T;
      t /= geo.nt[c];
    }
  }
  for (int i = threadIdx.x; i < ch.count; i += kBlock) {
    const int q = ch.start + i;
    double lf = cst;
    for (int c = 0; c < geo.d; ++c) {
      // torus coordinate in [-1/2, 1/2): the grid coordinate is tau g wrapped into [0, g)
      double tau = (double(org[c]) + double(a.coords[size_t(q) * geo.d + c])) / double(geo.g);
      if (tau >= 0.5) tau -= 1.0;
      lf += pb[4 + c] * (pb[1 + c] + tau / scale);
    }
    const double v = a.src[q];
    if (a.perm)
      a.out[a.perm[q]] = a.logd ? v + eps * lf : v * exp(lf);
    else
      a.out[q] = a.logd ? v - eps * lf : v * exp(-lf);
  }
}

template <typename R>
hipError_t launch_uncenter(const UncenterArgs<R>& a, int nchunks, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(uncenter_kernel<R>, dim3(nchunks), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_uncenter<float>(const UncenterArgs<float>&, int, hipStream_t);
template hipError_t launch_uncenter<double>(const UncenterArgs<double>&, int, hipStream_t);

int bbox_blocks(long n) { return int(std::min<long>(kGridBlocks, std::max<long>(1, (n + 8 * kBlock - 1) / (8 * kBlock)))); }

hipError_t launch_bbox(const BoxArgs& a, hipStream_t st) {
  const int nb = bbox_blocks(std::max(std::max(a.n[0], a.n[1]), a.nw));
  hipLaunchKernelGGL(bbox_kernel, dim3(nb), dim3(kBlock), 0, st, a, (const BoxJob*)nullptr, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish_partials<kBoxVals>(a.partials, nb, kBoxMin, kBoxMax, a.out, st);
}

// One workgroup per box: its workgroups' partials, in order, into its out.
__global__ __launch_bounds__(kBlock) void bbox_finish_kernel(const double* partials, const BoxJob* jobs) {
  constexpr int NV = kBoxVals;
  __shared__ double sh[NV][kBlock];
  const BoxJob& jb = jobs[blockIdx.x];
  bool is_min[NV], is_max[NV];
  double acc[NV];
  for (int k = 0; k < NV; ++k) {
    is_min[k] = (kBoxMin >> k) & 1u;
    is_max[k] = (kBoxMax >> k) & 1u;
    acc[k] = is_min[k] ? 1e308 : (is_max[k] ? -1e308 : 0.0);
  }
  for (int b = threadIdx.x; b < jb.nblk; b += kBlock)
    for (int k = 0; k < NV; ++k) {
      const double x = partials[size_t(jb.blk0 + b) * NV + k];
      acc[k] = is_min[k] ? fmin(acc[k], x) : (is_max[k] ? fmax(acc[k], x) : acc[k] + x);
    }
  block_reduce_arr<NV>(acc, is_min, is_max, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) jb.box.out[k] = acc[k];
}

hipError_t launch_bbox_jobs(const BoxJob* jobs, int njobs, long nblocks, int d, double* partials, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  if (nblocks >= (long(1) << 31)) return hipErrorInvalidValue;
  BoxArgs a{};
  a.d = d;
  a.partials = partials;
  hipLaunchKernelGGL(bbox_kernel, dim3(unsigned(nblocks)), dim3(kBlock), 0, st, a, jobs, njobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bbox_finish_kernel, dim3(njobs), dim3(kBlock), 0, st, (const double*)partials, jobs);
  return hipGetLastError();
}

// ------------------------------------------------------------------ keys + histogram
__device__ __forceinline__ double grid_coord(double x, double center, double scale, int g) {
  const double tau = scale > 0.0 ? scale * (x - center) : x;
  double v = double(g) * tau;
  v -= double(g) * floor(v / double(g));
  if (v >= double(g)) v -= double(g);
  if (v < 0.0) v = 0.0;
  return v;
}

__global__ __launch_bounds__(kBlock) void keys_kernel(KeyArgs a) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= a.n) return;
  int key = 0;
  for (int c = 0; c < a.d; ++c) {
    const double v = grid_coord(a.pts[i * a.d + c], a.center[c], a.scale, a.g);
    const int cell = min(int(v), a.g - 1);
    key = key * a.nt[c] + cell / a.T;
  }
  a.keys[i] = key;
  atomicAdd(&a.counts[key], 1);
}

// Clustered clouds put most points into a few tiles, so per-point global
// atomics on the tile counters serialize.  With at most kPlanBins tiles, each
// workgroup histograms kPlanPerThread * kBlock points in LDS first and adds
// one count per (workgroup, tile) to the global counters.
constexpr int kPlanBins = 8192;
constexpr int kPlanPerThread = 16;
constexpr int kPlanPerBlock = kPlanPerThread * kBlock;

long plan_block_points() { return kPlanPerBlock; }
bool plan_batchable(int nbins) { return nbins <= kPlanBins; }

// Batched form: the problem whose workgroups include blk (the last with blk0
// <= blk), and blk made relative to its first workgroup.
__device__ __forceinline__ int plan_problem(const PlanProb* probs, int nprob, long& blk) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].blk0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  blk -= probs[lo].blk0;
  return lo;
}

__device__ __forceinline__ int tile_key(const double* pts, long i, int d, const double* center, double scale, int g,
                                        int T, const int* nt) {
  int key = 0;
  for (int c = 0; c < d; ++c) {
    const double v = grid_coord(pts[i * d + c], center[c], scale, g);
    const int cell = min(int(v), g - 1);
    key = key * nt[c] + cell / T;
  }
  return key;
}

__global__ __launch_bounds__(kBlock) void keys_lds_kernel(KeyArgs a) {
  extern __shared__ int hist[];
  const int nbins = a.nt[0] * a.nt[1] * a.nt[2];
  long blk = blockIdx.x;
  if (a.probs) {
    const int pb = plan_problem(a.probs, a.nprob, blk);
    const PlanProb& pp = a.probs[pb];
    a.pts += pp.o * a.d;
    a.n = pp.n;
    for (int c = 0; c < 3; ++c) a.center[c] = pp.center[c];
    a.scale = pp.scale;
    a.keys += pp.o;
    a.counts += size_t(pb) * nbins;
  }
  for (int b = threadIdx.x; b < nbins; b += kBlock) hist[b] = 0;
  __syncthreads();
  const long base = blk * kPlanPerBlock;
  const long end = min(base + kPlanPerBlock, a.n);
  for (long i = base + threadIdx.x; i < end; i += kBlock) {
    const int key = tile_key(a.pts, i, a.d, a.center, a.scale, a.g, a.T, a.nt);
    a.keys[i] = key;
    atomicAdd(&hist[key], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += kBlock)
    if (hist[b]) atomicAdd(&a.counts[b], hist[b]);
}

hipError_t launch_keys(const KeyArgs& a, hipStream_t st) {
  const int nbins = a.nt[0] * a.nt[1] * a.nt[2];
  if (a.probs) {
    // a.n: the launch's workgroups (the last problem's blk0 + its workgroups)
    if (!plan_batchable(nbins) || a.n <= 0 || a.n >= (long(1) << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(keys_lds_kernel, dim3(unsigned(a.n)), dim3(kBlock), sizeof(int) * nbins, st, a);
    return hipGetLastError();
  }
  if (a.n <= 0) return hipSuccess;
  if (nbins <= kPlanBins) {
    const long nblk = (a.n + kPlanPerBlock - 1) / kPlanPerBlock;
    hipLaunchKernelGGL(keys_lds_kernel, dim3(nblk), dim3(kBlock), sizeof(int) * nbins, st, a);
  } else {
    hipLaunchKernelGGL(keys_kernel, dim3((a.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
  }
  return hipGetLastError();
}

template <typename R>
__global__ __launch_bounds__(kBlock) void scatter_kernel(ScatterArgs<R> a) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int key = a.keys[i];
  const int pos = a.offsets[key] + atomicAdd(&a.cursor[key], 1);
  for (int c = 0; c < a.d; ++c) {
    const double v = grid_coord(a.pts[i * a.d + c], a.center[c], a.scale, a.g);
    const int cell = min(int(v), a.g - 1);
    const double u = v - double((cell / a.T) * a.T);
    R ur = R(u);
    if (ur >= R(a.T)) ur = nextafter(R(a.T), R(0));
    if (ur < R(0)) ur = R(0);
    a.coords[size_t(pos) * a.d + c] = ur;
  }
  a.perm[pos] = int(i) + a.idx_base;
  if (a.w0) a.w0s[pos] = a.w0[i];
  if (a.w1) a.w1s[pos] = a.w1[i];
}

template <typename R>
__device__ __forceinline__ void scatter_point(const ScatterArgs<R>& a, long i, int pos) {
  for (int c = 0; c < a.d; ++c) {
    const double v = grid_coord(a.pts[i * a.d + c], a.center[c], a.scale, a.g);
    const int cell = min(int(v), a.g - 1);
    const double u = v - double((cell / a.T) * a.T);
    R ur = R(u);
    if (ur >= R(a.T)) ur = nextafter(R(a.T), R(0));
    if (ur < R(0)) ur = R(0);
    a.coords[size_t(pos) * a.d + c] = ur;
  }
  a.perm[pos] = int(i) + a.idx_base;
  if (a.w0) a.w0s[pos] = a.w0[i];
  if (a.w1) a.w1s[pos] = a.w1[i];
}

// Workgroup-local counting: each point's rank among the workgroup's points of
// its tile (LDS atomics), one global atomic per (workgroup, tile) to reserve
// the workgroup's slots, then the writes.
template <typename R>
__global__ __launch_bounds__(kBlock) void scatter_lds_kernel(ScatterArgs<R> a, int nbins) {
  extern __shared__ int sh[];
  int* hist = sh;
  int* slot = sh + nbins;
  long blk = blockIdx.x;
  if (a.probs) {
    const int pb = plan_problem(a.probs, a.nprob, blk);
    const PlanProb& pp = a.probs[pb];
    a.pts += pp.o * a.d;
    a.n = pp.n;
    for (int c = 0; c < 3; ++c) a.center[c] = pp.center[c];
    a.scale = pp.scale;
    a.keys += pp.o;
    a.offsets += size_t(pb) * nbins;
    a.cursor += size_t(pb) * nbins;
    a.idx_base = int(pp.o);
    if (a.w0) a.w0 += pp.o;
    if (a.w1) a.w1 += pp.o;
  }
  for (int b = threadIdx.x; b < nbins; b += kBlock) hist[b] = 0;
  __syncthreads();
  const long base = blk * kPlanPerBlock;
  int key[kPlanPerThread], rank[kPlanPerThread];
#pragma unroll
  for (int k = 0; k < kPlanPerThread; ++k) {
    const long i = base + threadIdx.x + long(k) * kBlock;
    key[k] = -1;
    if (i < a.n) {
      key[k] = a.keys[i];
      rank[k] = atomicAdd(&hist[key[k]], 1);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += kBlock)
    if (hist[b]) slot[b] = a.offsets[b] + atomicAdd(&a.cursor[b], hist[b]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPlanPerThread; ++k)
    if (key[k] >= 0) scatter_point(a, base + threadIdx.x + long(k) * kBlock, slot[key[k]] + rank[k]);
}

template <typename R>
hipError_t launch_scatter(const ScatterArgs<R>& a, hipStream_t st) {
  const int nbins = a.nt[0] * a.nt[1] * a.nt[2];
  if (a.probs) {
    // a.n: the launch's workgroups, as for launch_keys
    if (!plan_batchable(nbins) || a.n <= 0 || a.n >= (long(1) << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scatter_lds_kernel<R>, dim3(unsigned(a.n)), dim3(kBlock), sizeof(int) * 2 * nbins, st, a,
                       nbins);
    return hipGetLastError();
  }
  if (a.n <= 0) return hipSuccess;
  if (nbins <= kPlanBins) {
    const long nblk = (a.n + kPlanPerBlock - 1) / kPlanPerBlock;
    hipLaunchKernelGGL(scatter_lds_kernel<R>, dim3(nblk), dim3(kBlock), sizeof(int) * 2 * nbins, st, a, nbins);
  } else {
    hipLaunchKernelGGL(scatter_kernel<R>, dim3((a.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
  }
  return hipGetLastError();
}
template hipError_t launch_scatter<float>(const ScatterArgs<float>&, hipStream_t);
template hipError_t launch_scatter<double>(const ScatterArgs<double>&, hipStream_t);

// ------------------------------------------------------------------ cell order and run tables
// Exclusive prefix sum over the workgroup of NT threads; returns this
// thread's prefix and the total in *total.  `part` holds NT ints of LDS.
template <int NT = kBlock>
__device__ int block_exclusive_scan(int v, int* part, int* total) {
  part[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < NT; off <<= 1) {
    const int u = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += u;
    __syncthreads();
  }
  const int incl = part[threadIdx.x];
  *total = part[NT - 1];
  __syncthreads();
  return incl - v;
}

template <typename R>
__device__ __forceinline__ int cell_key_at(const R* coords, size_t q, int d, int T) {
  int k = 0;
  for (int c = 0; c < d; ++c) k = k * T + min(max(int(coords[q * d + c]), 0), T - 1);
  return k;
}

// Exclusive scan of hist[0..nc) in place (nc <= kSortBins) by a workgroup of
// NT threads; each thread owns a contiguous run of bins.  Returns the total.
template <int NT>
__device__ int scan_bins(int* hist, int nc, int* part) {
  const int per = (nc + NT - 1) / NT;
  const int b0 = min(int(threadIdx.x) * per, nc), b1 = min(b0 + per, nc);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += hist[i];
  int total;
  int run = block_exclusive_scan<NT>(s, part, &total);
  for (int i = b0; i < b1; ++i) {
    const int c = hist[i];
    hist[i] = run;
    run += c;
  }
  __syncthreads();
  return total;
}

// One workgroup per (problem, tile): LDS histogram of the tile's points over
// its T^d cells, exclusive scan, then each point goes to its cell's next slot,
// and the points of each cell are put in the order of their input index.
// Each pass over the tile's points is a chain of dependent global accesses
// per thread, and the densest tile (85K points on the 2-D mixture) sets the
// plan time: 1024 threads per workgroup cut that chain by four.
constexpr int kSortThreads = 1024;
constexpr int kCanonCell = 1024;
// Ranks are counted from a copy of the input indices in LDS (dynamic, 112 KiB
// next to the 33 KiB of bins), one window of whole cells of at most
// kCanonStage points at a time: one LDS read per point of the cell instead of
// one global load.
constexpr int kCanonStage = 28 * 1024;

template <typename R>
__global__ __launch_bounds__(kSortThreads) void tile_sort_kernel(TileSortArgs<R> a) {
  // distinct buffers: unrolled iterations may issue their loads before the
  // stores of the ones before
  R* __restrict__ in_coords = a.in_coords;
  int* __restrict__ in_perm = a.in_perm;
  double* __restrict__ in_w0 = a.in_w0;
  double* __restrict__ in_w1 = a.in_w1;
  R* __restrict__ coords = a.coords;
  int* __restrict__ perm = a.perm;
  double* __restrict__ w0s = a.w0s;
  double* __restrict__ w1s = a.w1s;
  __shared__ int slot[kSortBins];
  __shared__ int first[kSortBins];
  __shared__ int part[kSortThreads];
  extern __shared__ int stage[];  // kCanonStage entries
  const int cnt = a.counts[blockIdx.x];
  const int d = a.d, T = a.T;
  int nc = 1;
  for (int c = 0; c < d; ++c) nc *= T;
  int* cs = a.cellstart ? a.cellstart + size_t(blockIdx.x) * (nc + 1) : nullptr;
  if (cnt == 0) {
    if (cs)
      for (int i = threadIdx.x; i <= nc; i += kSortThreads) cs[i] = 0;
    return;
  }
  const size_t off = size_t(a.offsets[blockIdx.x]);
  for (int i = threadIdx.x; i < nc; i += kSortThreads) slot[i] = 0;
  __syncthreads();
#pragma unroll 4
  for (int i = threadIdx.x; i < cnt; i += kSortThreads) atomicAdd(&slot[cell_key_at(in_coords, off + i, d, T)], 1);
  __syncthreads();
  scan_bins<kSortThreads>(slot, nc, part);
  if (cs) {
    for (int i = threadIdx.x; i < nc; i += kSortThreads) cs[i] = slot[i];
    if (threadIdx.x == 0) cs[nc] = cnt;
  }
  for (int i = threadIdx.x; i < nc; i += kSortThreads) first[i] = slot[i];
  __syncthreads();
#pragma unroll 4
  for (int i = threadIdx.x; i < cnt; i += kSortThreads) {
    const size_t q = off + i;
    const size_t pos = off + atomicAdd(&slot[cell_key_at(in_coords, q, d, T)], 1);
    for (int c = 0; c < d; ++c) coords[pos * d + c] = in_coords[q * d + c];
    perm[pos] = in_perm[q];
    if (w0s) w0s[pos] = in_w0[q];
    if (w1s) w1s[pos] = in_w1[q];
  }
  // Canonical order inside each cell: by the points' input index.  The
  // scatter and the placement above leave a cell's points in the order their
  // atomics happened to run; ranking them by input index makes the sorted
  // clouds, hence every sum over them, the same from run to run.  The ranks
  // go through the staging arrays (free now), then back.  Cells of more than
  // kCanonCell points keep their placement order.
  __threadfence_block();
  __syncthreads();
  // The cells occupy consecutive positions now, so a window of whole cells
  // is a contiguous range [s, e); it takes the most cells whose points fit
  // the stage.  A cell larger than the stage (beyond kCanonCell, so it keeps
  // its placement order) is a window of its own, not staged.
  auto pos = [&](int c) { return c < nc ? first[c] : cnt; };
  for (int c_lo = 0; c_lo < nc;) {
    const int s = first[c_lo];
    int lo = c_lo, hi = nc;  // largest c_hi in [c_lo, nc] with pos(c_hi) - s <= kCanonStage
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pos(mid) - s <= kCanonStage) lo = mid;
      else hi = mid - 1;
    }
    const bool staged = lo > c_lo;
    const int c_hi = staged ? lo : c_lo + 1;
    const int e = pos(c_hi);
    if (staged) {
      for (int i = s + int(threadIdx.x); i < e; i += kSortThreads) stage[i - s] = perm[off + i];
      __syncthreads();
    }
#pragma unroll 4
    for (int i = s + int(threadIdx.x); i < e; i += kSortThreads) {
      const size_t q = off + i;
      const int cell = cell_key_at(coords, q, d, T);
      const int c0 = first[cell], c1 = slot[cell];
      const int pq = perm[q];
      int rank = i - c0;
      if (staged && c1 - c0 <= kCanonCell) {
        rank = 0;
        for (int j = c0; j < c1; ++j) rank += stage[j - s] < pq ? 1 : 0;
      }
      const size_t dst = off + c0 + rank;
      for (int c = 0; c < d; ++c) in_coords[dst * d + c] = coords[q * d + c];
      in_perm[dst] = pq;
      if (w0s) in_w0[dst] = w0s[q];
      if (w1s) in_w1[dst] = w1s[q];
    }
    __syncthreads();  // the next window overwrites the stage
    c_lo = c_hi;
  }
  __threadfence_block();
  __syncthreads();
#pragma unroll 4
  for (int i = threadIdx.x; i < cnt; i += kSortThreads) {
    const size_t q = off + i;
    for (int c = 0; c < d; ++c) coords[q * d + c] = in_coords[q * d + c];
    perm[q] = in_perm[q];
    if (w0s) w0s[q] = in_w0[q];
    if (w1s) w1s[q] = in_w1[q];
  }
}

template <typename R>
hipError_t launch_tile_sort(const TileSortArgs<R>& a, hipStream_t st) {
  if (a.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(tile_sort_kernel<R>, dim3(a.ntiles), dim3(kSortThreads), kCanonStage * sizeof(int), st, a);
  return hipGetLastError();
}
template hipError_t launch_tile_sort<float>(const TileSortArgs<float>&, hipStream_t);
template hipError_t launch_tile_sort<double>(const TileSortArgs<double>&, hipStream_t);

// One workgroup per chunk.  With the chunk in cell order, an LDS histogram of
// its points over the tile's cells and a scan give each cell's first
// position in the chunk; every cell's c points become c / G full runs and
// c mod G single points.  The table lists all full runs, then all singles.
template <typename R>
__global__ __launch_bounds__(kBlock) void chunk_runs_kernel(ChunkRunArgs<R> a) {
  __shared__ int start[kSortBins];
  __shared__ int part[kBlock];
  const Chunk ch = a.chunks[blockIdx.x];
  int* runs = a.runs + ch.start;
  if (!a.sorted) {
    for (int i = threadIdx.x; i < ch.count; i += kBlock) runs[i] = i;
    if (threadIdx.x == 0) {
      a.nruns[2 * blockIdx.x] = 0;
      a.nruns[2 * blockIdx.x + 1] = ch.count;
    }
    return;
  }
  const int d = a.d, T = a.T, G = a.G;
  int nc = 1;
  for (int c = 0; c < d; ++c) nc *= T;
  for (int i = threadIdx.x; i < nc; i += kBlock) start[i] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < ch.count; i += kBlock)
    atomicAdd(&start[cell_key_at(a.coords, size_t(ch.start) + i, d, T)], 1);
  __syncthreads();
  // per-thread cells [b0, b1): points, full runs and singles, then scans
  const int per = (nc + kBlock - 1) / kBlock;
  const int b0 = min(int(threadIdx.x) * per, nc), b1 = min(b0 + per, nc);
  int npts = 0, nfull = 0, nsing = 0;
  for (int i = b0; i < b1; ++i) {
    const int c = start[i];
    npts += c;
    nfull += c / G;
    nsing += c % G;
  }
  int total_pts, total_full, total_sing;
  int pos = block_exclusive_scan(npts, part, &total_pts);
  int fpos = block_exclusive_scan(nfull, part, &total_full);
  int spos = total_full + block_exclusive_scan(nsing, part, &total_sing);
  for (int i = b0; i < b1; ++i) {
    const int c = start[i];
    const int f = c / G;
    for (int o = 0; o < f; ++o) runs[fpos++] = pos + o * G;
    for (int o = f * G; o < c; ++o) runs[spos++] = pos + o;
    pos += c;
  }
  if (threadIdx.x == 0) {
    a.nruns[2 * blockIdx.x] = total_full;
    a.nruns[2 * blockIdx.x + 1] = total_sing;
  }
  if (!a.srun) return;
  // spreading's table: ceil(c / G) runs per cell (the last partial).  Cells
  // with at least kQuadRuns runs put them in groups of four same-cell runs;
  // other runs go in same-cell pairs, then the odd run of a cell alone.
  // Groups of four cost a second DPP step and a wider select per tap: on the
  // 2-D mixture (14 points per occupied cell, cells of 29+ points in groups)
  // spreading went from 66 to 79 us.  In very dense cells many pairs of one
  // cell share a wave and contend on the same words, and groups pay: 1e7
  // uniform points (610 per cell) 7.5 -> 4.9 ms per FP64 iteration.
  constexpr int kQuadRuns = 64;
  int* srun = a.srun + ch.start;
  auto split = [&](int q, int& nq, int& np) {
    nq = q >= kQuadRuns ? 4 * (q / 4) : 0;
    np = 2 * ((q - nq) / 2);
  };
  int nqe = 0, npe = 0, nsolo = 0;
  for (int i = b0; i < b1; ++i) {
    const int q = (start[i] + G - 1) / G;
    int nq, np;
    split(q, nq, np);
    nqe += nq;
    npe += np;
    nsolo += q - nq - np;
  }
  int total_qe, total_pe, total_solo;
  int qpos = block_exclusive_scan(nqe, part, &total_qe);
  int ppos = total_qe + block_exclusive_scan(npe, part, &total_pe);
  int opos = total_qe + total_pe + block_exclusive_scan(nsolo, part, &total_solo);
  int p0 = pos;  // pos was advanced over this thread's cells above: rewind it
  for (int i = b0; i < b1; ++i) p0 -= start[i];
  for (int i = b0; i < b1; ++i) {
    const int c = start[i];
    const int q = (c + G - 1) / G;
    int nq, np;
    split(q, nq, np);
    for (int r = 0; r < q; ++r) {
      const int e = (p0 + r * G) | ((min(G, c - r * G) - 1) << 16);
      if (r < nq) srun[qpos++] = e;
      else if (r < nq + np) srun[ppos++] = e;
      else srun[opos++] = e;
    }
    p0 += c;
  }
  if (threadIdx.x == 0) {
    a.nsrun[3 * blockIdx.x] = total_qe;
    a.nsrun[3 * blockIdx.x + 1] = total_pe;
    a.nsrun[3 * blockIdx.x + 2] = total_solo;
  }
}

template <typename R>
hipError_t launch_chunk_runs(const ChunkRunArgs<R>& a, hipStream_t st) {
  if (a.nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(chunk_runs_kernel<R>, dim3(a.nchunks), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_chunk_runs<float>(const ChunkRunArgs<float>&, hipStream_t);
template hipError_t launch_chunk_runs<double>(const ChunkRunArgs<double>&, hipStream_t);

// ------------------------------------------------------------------ fills / permutations
__global__ __launch_bounds__(kBlock) void fill_kernel(uint32_t* p, size_t nwords) {
  const size_t stride = size_t(gridDim.x) * kBlock;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < nwords; i += stride) p[i] = 0u;
}

hipError_t launch_fill(void* p, size_t bytes, hipStream_t st) {
  const size_t nw = bytes / 4;
  if (nw == 0) return hipSuccess;
  const size_t nb = std::min<size_t>((nw + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(fill_kernel, dim3(nb), dim3(kBlock), 0, st, reinterpret_cast<uint32_t*>(p), nw);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void fill_double_kernel(double* p, long n, double v) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_double(double* p, long n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_double_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void unpermute_kernel(const double* src, const int* perm, long n, double* dst) {
  const long q = long(blockIdx.x) * kBlock + threadIdx.x;
  if (q < n) dst[perm[q]] = src[q];
}

hipError_t launch_unpermute(const double* src, const int* perm, long n, double* dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(unpermute_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, src, perm, n, dst);
  return hipGetLastError();
}

// ------------------------------------------------------------------ diagonal tables (r = 2)
template <typename R>
__global__ __launch_bounds__(kBlock) void gauss_tables_kernel(int d, int N, long H, const double* pb,
                                                              const double* inv_phi, R* kernel, R* cost) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= H) return;
  const double e = pb[2 * b], s = pb[2 * b + 1];
  const size_t o = size_t(b) * H + i;
  if (!(e > 0.0)) {
    kernel[o] = R(0);
    cost[o] = R(0);
    return;
  }
  const int h = N / 2 + 1;
  const double pi = 3.14159265358979323846;
  long rem = i;
  double prod = 1.0, k2 = 0.0;
  for (int c = d - 1; c >= 0; --c) {
    const int kc = int(rem % h);
    rem /= h;
    double f = sqrt(pi * e) * exp(-pi * pi * e * double(kc) * kc) * inv_phi[kc] * inv_phi[kc];
    if (kc == N / 2) f *= 0.5;
    prod *= f;
    k2 += double(kc) * kc;
  }
  kernel[o] = R(prod);
  cost[o] = R(prod * (0.5 * d * e - pi * pi * e * e * k2) / (s * s));
}

template <typename R>
hipError_t launch_gauss_tables(int d, int N, int B, const double* pb, const double* inv_phi, R* kernel, R* cost,
                               hipStream_t st) {
  long H = 1;
  for (int c = 0; c < d; ++c) H *= N / 2 + 1;
  if (B <= 0 || B > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gauss_tables_kernel<R>, dim3(unsigned((H + kBlock - 1) / kBlock), unsigned(B)), dim3(kBlock), 0,
                     st, d, N, H, pb, inv_phi, kernel, cost);
  return hipGetLastError();
}
template hipError_t launch_gauss_tables<float>(int, int, int, const double*, const double*, float*, float*,
                                               hipStream_t);
template hipError_t launch_gauss_tables<double>(int, int, int, const double*, const double*, double*, double*,
                                                hipStream_t);

// ------------------------------------------------------------------ diagonal tables (real rho)
template <typename R>
__global__ __launch_bounds__(kBlock) void kernel_samples_kernel(int d, int g, long ncell, const double* cf, int cost,
                                                                R* out) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= ncell) return;
  long rem = i;
  double r2 = 0.0;  // squared distance in cells to the nearest image of the origin
  for (int c = 0; c < d; ++c) {
    const long l = rem % g;
    rem /= g;
    const double x = double(l < g / 2 ? l : l - g);
    r2 += x * x;
  }
  double v;
  if (r2 < cf[1]) {
    const int ps = int(cf[3]);
    const double u2 = r2 * cf[2];
    v = cf[4 + ps - 1];
    for (int j = ps - 2; j >= 0; --j) v = v * u2 + cf[4 + j];
  } else {
    const double rr = pow(r2, cf[kNearRhoHalf]);
    v = exp(-rr * cf[kNearRhoInv]);
    if (cost) v *= rr * cf[kNearCostMul];
  }
  out[i] = R(v);
}

template <typename R>
hipError_t launch_kernel_samples(int d, int g, const double* cf, int cost, R* out, hipStream_t st) {
  long ncell = 1;
  for (int c = 0; c < d; ++c) ncell *= g;
  hipLaunchKernelGGL(kernel_samples_kernel<R>, dim3(unsigned((ncell + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, d, g,
                     ncell, cf, cost, out);
  return hipGetLastError();
}
template hipError_t launch_kernel_samples<float>(int, int, const double*, int, float*, hipStream_t);
template hipError_t launch_kernel_samples<double>(int, int, const double*, int, double*, hipStream_t);

template <typename R>
__global__ __launch_bounds__(kBlock) void spec_table_kernel(int d, int N, int g, long H, const cplx<R>* spec,
                                                            const double* inv_phi, R* tab) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= H) return;
  const int h = N / 2 + 1;
  long rem = i, o = 0, stride = 1;
  double f = 1.0;
  for (int c = d - 1; c >= 0; --c) {
    const int kc = int(rem % h);
    rem /= h;
    // the last axis holds k = 0..N/2, the others the centered k = -N/2..N/2
    o += stride * (c == d - 1 ? kc : kc + N / 2);
    stride *= c == d - 1 ? h : N + 1;
    f *= inv_phi[kc] * inv_phi[kc];
    if (kc == N / 2) f *= 0.5;
  }
  tab[i] = R(double(spec[o].x) * f / pow(double(g), d));
}

template <typename R>
hipError_t launch_spec_table(int d, int N, int g, const cplx<R>* spec, const double* inv_phi, R* tab, hipStream_t st) {
  long H = 1;
  for (int c = 0; c < d; ++c) H *= N / 2 + 1;
  hipLaunchKernelGGL(spec_table_kernel<R>, dim3(unsigned((H + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, d, N, g, H,
                     spec, inv_phi, tab);
  return hipGetLastError();
}
template hipError_t launch_spec_table<float>(int, int, int, const cplx<float>*, const double*, float*, hipStream_t);
template hipError_t launch_spec_table<double>(int, int, int, const cplx<double>*, const double*, double*,
                                              hipStream_t);

// ------------------------------------------------------------------ read-out sums
__global__ __launch_bounds__(kBlock) void readout_kernel(ReadoutArgs a) {
  constexpr int NV = 3;
  double v[NV] = {0.0, 0.0, 0.0};
  const bool is_min[NV] = {false, false, false}, is_max[NV] = {false, false, false};
  const long stride = long(gridDim.x) * kBlock;
  for (long i = long(blockIdx.x) * kBlock + threadIdx.x; i < a.n; i += stride) {
    const double x = a.a[i];
    if (x > 0.0) {
      v[0] += x * (a.logv ? a.b[i] : log(a.b[i]));
      v[1] += x * log(x);
    }
    v[2] += x;
  }
  grid_reduce_arr<NV>(v, is_min, is_max, a.partials);
}

hipError_t launch_readout(const ReadoutArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(readout_kernel, dim3(256), dim3(kBlock), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish_partials<3>(a.partials, 256, 0u, 0u, a.out, st);
}

// Log domain: the spread weights exp((pot - shift)/eps) of one chunk per workgroup.
__global__ __launch_bounds__(kBlock) void logweights_kernel(const Chunk* chunks, const double* pot,
                                                            const double* shift, const double* leps, double* out,
                                                            const int* pstate) {
  const Chunk ch = chunks[blockIdx.x];
  if (pstate && pstate[kPState * ch.prob] == 2) return;  // the problem has stopped
  const double sh = shift[ch.prob], inv = leps[kLepsStride * ch.prob];
  for (int i = threadIdx.x; i < ch.count; i += kBlock) {
    const int q = ch.start + i;
    out[q] = exp((pot[q] - sh) * inv);
  }
}

hipError_t launch_logweights(const Chunk* chunks, int nchunks, const double* pot, const double* shift,
                             const double* leps, double* out, const int* pstate, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(logweights_kernel, dim3(nchunks), dim3(kBlock), 0, st, chunks, pot, shift, leps, out, pstate);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void mul_kernel(const double* a, const double* b, long n, double* out) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

hipError_t launch_mul(const double* a, const double* b, long n, double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mul_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a, b, n, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void maxsum_kernel(const double* vals, long n, double* partials) {
  constexpr int NV = 2;
  double v[NV] = {-INFINITY, 0.0};
  const bool is_min[NV] = {false, false}, is_max[NV] = {(kMaxSumMax & 1u) != 0, false};
  const long stride = long(gridDim.x) * kBlock;
  for (long i = long(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
    v[0] = fmax(v[0], vals[i]);
    v[1] += vals[i];
  }
  grid_reduce_arr<NV>(v, is_min, is_max, partials);
}

hipError_t launch_maxsum(const double* v, long n, double* partials, double* out, hipStream_t st) {
  hipLaunchKernelGGL(maxsum_kernel, dim3(256), dim3(kBlock), 0, st, v, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish_partials<2>(partials, 256, 0u, kMaxSumMax, out, st);
}

// eps log alpha_i enters the weight gradient only where alpha_i > 0: a point of
// weight zero has scaling zero and contributes 0 log 0 = 0 to the dual.
__device__ __forceinline__ double log_or_zero(double a) { return a > 0.0 ? log(a) : 0.0; }

__global__ __launch_bounds__(kBlock) void logmean_kernel(const double* alpha, long n, double* partials) {
  constexpr int NV = 1;
  double v[NV] = {0.0};
  const bool is_min[NV] = {false}, is_max[NV] = {false};
  const long stride = long(gridDim.x) * kBlock;
  for (long i = long(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) v[0] += log_or_zero(alpha[i]);
  grid_reduce_arr<NV>(v, is_min, is_max, partials);
}

__global__ __launch_bounds__(kBlock) void gradmu_kernel(const double* alpha, long n, double eps,
                                                        const double* sumlog, const int* perm, double* g) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) g[perm ? long(perm[i]) : i] = eps * (log_or_zero(alpha[i]) - *sumlog / double(n));
}

hipError_t launch_gradmu(const double* alpha, long n, double eps, double* partials, double* mean_out,
                         double* grad_mu, hipStream_t st, const int* perm) {
  hipLaunchKernelGGL(logmean_kernel, dim3(256), dim3(kBlock), 0, st, alpha, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = finish_partials<1>(partials, 256, 0u, 0u, mean_out, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(gradmu_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, alpha, n, eps,
                     (const double*)mean_out, perm, grad_mu);
  return hipGetLastError();
}

// ------------------------------------------------------------------ NFFT spectrum conversions
// Internal half spectrum: all axes but the last centered (N+1 entries, k + N/2),
// the last axis k = 0..N/2 (K0 entries).
__device__ __forceinline__ long spec_index(int d, int N, const int* k) {
  const int K0 = N / 2 + 1;
  long idx = 0;
  for (int c = 0; c < d - 1; ++c) idx = idx * (N + 1) + (k[c] + N / 2);
  return idx * K0 + k[d - 1];
}

template <typename R>
__global__ __launch_bounds__(kBlock) void spec_to_user_kernel(SpecArgs<R> a) {
  long total = 1;
  for (int c = 0; c < a.d; ++c) total *= a.N;
  const long u = long(blockIdx.x) * kBlock + threadIdx.x;
  if (u >= total) return;
  int k[3];
  long rem = u;
  for (int c = a.d - 1; c >= 0; --c) {
    k[c] = int(rem % a.N) - a.N / 2;
    rem /= a.N;
  }
  double f = a.scale;
  for (int c = 0; c < a.d; ++c) f *= a.inv_phi[abs(k[c])];
  cplx<R> h;
  if (k[a.d - 1] >= 0) {
    h = a.spec_in[spec_index(a.d, a.N, k)];
  } else {
    int km[3];
    for (int c = 0; c < a.d; ++c) km[c] = -k[c];
    h = a.spec_in[spec_index(a.d, a.N, km)];
    h.y = -h.y;
  }
  a.user_out[2 * u] = double(h.x) * f;
  a.user_out[2 * u + 1] = double(h.y) * f;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void user_to_spec_kernel(SpecArgs<R> a) {
  const int K0 = a.N / 2 + 1;
  long total = K0;
  for (int c = 0; c < a.d - 1; ++c) total *= (a.N + 1);
  const long s = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= total) return;
  int k[3];
  long rem = s;
  k[a.d - 1] = int(rem % K0);
  rem /= K0;
  for (int c = a.d - 2; c >= 0; --c) {
    k[c] = int(rem % (a.N + 1)) - a.N / 2;
    rem /= (a.N + 1);
  }
  // F(k) and F(-k) from the user array (zero outside I_N = [-N/2, N/2-1]^d)
  double fr = 0.0, fi = 0.0, gr = 0.0, gi = 0.0;
  bool in_p = true, in_m = true;
  long up = 0, um = 0;
  for (int c = 0; c < a.d; ++c) {
    in_p = in_p && (k[c] <= a.N / 2 - 1);
    in_m = in_m && (-k[c] <= a.N / 2 - 1);
    up = up * a.N + (k[c] + a.N / 2);
    um = um * a.N + (-k[c] + a.N / 2);
  }
  if (in_p) {
    fr = a.user_in[2 * up];
    fi = a.user_in[2 * up + 1];
  }
  if (in_m) {
    gr = a.user_in[2 * um];
    gi = a.user_in[2 * um + 1];
  }
  double f = 0.5;
  for (int c = 0; c < a.d; ++c) f *= a.inv_phi[abs(k[c])];
  a.spec_out[s] = cplx<R>{R((fr + gr) * f), R((fi - gi) * f)};
}

template <typename R>
hipError_t launch_spec_to_user(const SpecArgs<R>& a, hipStream_t st) {
  long total = 1;
  for (int c = 0; c < a.d; ++c) total *= a.N;
  hipLaunchKernelGGL(spec_to_user_kernel<R>, dim3((total + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_user_to_spec(const SpecArgs<R>& a, hipStream_t st) {
  long total = a.N / 2 + 1;
  for (int c = 0; c < a.d - 1; ++c) total *= (a.N + 1);
  hipLaunchKernelGGL(user_to_spec_kernel<R>, dim3((total + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template hipError_t launch_spec_to_user<float>(const SpecArgs<float>&, hipStream_t);
template hipError_t launch_spec_to_user<double>(const SpecArgs<double>&, hipStream_t);
template hipError_t launch_user_to_spec<float>(const SpecArgs<float>&, hipStream_t);
template hipError_t launch_user_to_spec<double>(const SpecArgs<double>&, hipStream_t);

}  // namespace nfs
