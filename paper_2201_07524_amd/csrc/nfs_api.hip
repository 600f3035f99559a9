// C ABI of the NFFT-boosted Sinkhorn library: argument checks, workspace
// layout, the plan stage (torus scaling, binning), the fast-summation chain
// and the Sinkhorn iteration (Algorithm 3) with hipGraph replay.
//
// Everything is written for a batch of B independent problems that share d,
// N, m and sigma (so one grid geometry): every stage is one kernel launch
// over all problems (chunks carry their problem index, grids and diagonal
// tables are stacked per problem).  A single problem is the batch B = 1.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nfs.h"
#include "common.h"
#include "host_math.h"
#include "kernels.h"

namespace nfs {

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define NFS_HIP(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail(NFS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));                \
  } while (0)

#define NFS_TRY(expr)              \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != NFS_OK) return rc_; \
  } while (0)

static int next_pow2(long v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

static int grid_size(const nfs_params* p) {
  const double want = std::ceil(p->sigma * p->N - 1e-9);
  return next_pow2(long(std::max(want, double(p->N) + 2.0)));
}

static int default_tile(int d, int precision) {
  (void)precision;
  return d == 1 ? 64 : (d == 2 ? 32 : 8);
}

// Tile sizes that NFS_FLAG_AUTOTUNE times on a solver (r = 2, tile left at
// 0): half, one and two times the default, those whose (T + 2m + 1)^d LDS
// tile fits and whose T^d cells the per-tile cell sort can order.  Empty
// when the tile is not tuned.
static std::vector<int> tile_candidates(const nfs_params* p) {
  std::vector<int> c;
  if (!(p->flags & NFS_FLAG_AUTOTUNE) || p->tile != 0 || p->r != 2) return c;
  const int T0 = default_tile(p->d, p->precision);
  for (int T : {T0 / 2, T0, 2 * T0}) {
    if (T < 4) continue;
    const double tb = std::pow(double(T + 2 * p->m + 1), p->d) * (p->precision == NFS_FP32 ? 4.0 : 8.0);
    if (tb <= 160.0 * 1024.0 && std::pow(double(T), p->d) <= double(kSortBins)) c.push_back(T);
  }
  return c;
}

// Points per chunk: 1536 for the FP32 2-D path (measured best on the 2-D
// mixture: longer same-cell runs, fewer tile loads and flushes per point,
// still about 700 workgroups per launch), 1024 otherwise (r = 1 needs <= 1024).
// Measured defaults: FP32 2-D 1536 (sweep 384..4096 on the 2-D mixture), FP32
// 3-D 4096 (picked by NFS_FLAG_AUTOTUNE on the 3-D mixture: iteration 3.25 ms
// against 3.41 at 2048 and 4.2 at 1024), 1024 otherwise.  r = 1 needs at most
// 1024 (near field).
static int default_chunk(const nfs_params* p) {
  if (p->r != 2) return 1024;
  if (p->precision == NFS_FP32 && p->d == 2) return 1536;
  if (p->precision == NFS_FP32 && p->d == 3) return 4096;
  return 1024;
}

// Near-field radius (times N) and smoothness of the r = 1 regularization by
// default: eps_I N = 4, p = 8.  A sweep of eps_I N in {2, ..., 4} x p in
// {4, ..., 12} (ball/shell, eps = 0.02, N = 128) shows the near field's cost
// falling as eps_I^3 (47 ms per half-step at 4e6 points down to 11 ms at
// eps_I N = 2), but the fast sums' error over all targets rising from 5e-6
// at (4, 8) to 1.5e-4 at (2, 4): smaller radii miss the FP32 bar.
static double default_eps_I(const nfs_params*) { return 4.0; }
static int default_p_smooth(const nfs_params*) { return 8; }

static int check_params(const nfs_params* p, int64_t n, int64_t nt) {
  if (!p) return fail(NFS_EINVAL, "params is NULL");
  if (p->d < 1 || p->d > 3) return fail(NFS_EINVAL, "d must be 1, 2 or 3");
  if (p->r != 0 && p->r != 1 && p->r != 2) return fail(NFS_EUNSUPPORTED, "cost exponent r must be 0, 1 or 2");
  if (p->r == 0 && (!(p->rexp > 1.0 && p->rexp <= 4.0) || p->rexp == 2.0))
    return fail(NFS_EINVAL, "r = 0 needs a real exponent rexp in (1, 4] other than 2 (use r = 1 or r = 2)");
  if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(NFS_EINVAL, "eps must be positive and finite");
  if (p->N < 4 || (p->N & 1)) return fail(NFS_EINVAL, "N must be even and >= 4");
  if (p->m < 2 || p->m > 8) return fail(NFS_EINVAL, "m must be in [2, 8]");
  if (!(p->sigma >= 1.0) || p->sigma > 16.0) return fail(NFS_EINVAL, "sigma must be in [1, 16]");
  if (p->precision != NFS_FP64 && p->precision != NFS_FP32)
    return fail(NFS_EINVAL, "precision must be NFS_FP64 or NFS_FP32 (NFS_AUTO: solve calls only)");
  const int g = grid_size(p);
  if (g > 4096) return fail(NFS_EUNSUPPORTED, "grid size sigma*N above 4096 per dimension");
  if (p->tile < 0 || p->tile > 256) return fail(NFS_EINVAL, "tile must be in [0, 256]");
  if (p->chunk < 0 || p->chunk > 32768) return fail(NFS_EINVAL, "chunk must be in [0, 32768]");
  if (n < 1 || nt < 1) return fail(NFS_EINVAL, "point counts must be >= 1");
  if (n > (int64_t(1) << 30) || nt > (int64_t(1) << 30)) return fail(NFS_EUNSUPPORTED, "point counts above 2^30");
  const double gd = std::pow(double(g), p->d);
  if (gd > double(1u << 30)) return fail(NFS_EUNSUPPORTED, "grid with more than 2^30 cells");
  const int T = p->tile ? p->tile : default_tile(p->d, p->precision);
  const int E = T + 2 * p->m + 1;
  const double tb = std::pow(double(E), p->d) * (p->precision == NFS_FP32 ? 4.0 : 8.0);
  if (tb > 160.0 * 1024.0) return fail(NFS_EINVAL, "LDS tile (tile + 2m + 1)^d exceeds 160 KiB; use a smaller tile");
  if (p->r != 2) {
    const double eIN = p->eps_I > 0.0 ? p->eps_I : default_eps_I(p);
    const int ps = p->p_smooth ? p->p_smooth : default_p_smooth(p);
    if (!(eIN > 0.0) || eIN > 0.25 * p->N) return fail(NFS_EINVAL, "eps_I (near-field radius times N) must be in (0, N/4]");
    if (ps < 2 || ps > 16) return fail(NFS_EINVAL, "p_smooth must be in [2, 16]");
    if (p->chunk > 1024) return fail(NFS_EINVAL, "r = 1 needs chunk <= 1024");
    const int kt = int(std::ceil(eIN * (double(g) / p->N) / T - 1e-12));
    if ((g + T - 1) / T < 2 * kt + 1)
      return fail(NFS_EUNSUPPORTED, "near-field radius too large for the grid (needs 2 kt + 1 tiles per axis)");
  }
  return NFS_OK;
}

// Per-problem slot of the bounding-box buffer: the x box, then the y box.
constexpr int kBoxSlot = 2 * kBoxVals;

// Near-field radius on the torus and smoothness (r = 1 and real exponents).
static double near_radius(const nfs_params* p) { return (p->eps_I > 0.0 ? p->eps_I : default_eps_I(p)) / p->N; }
static int near_smooth(const nfs_params* p) { return p->p_smooth ? p->p_smooth : default_p_smooth(p); }

// The cost exponent: r, or the real rexp when r = 0.
static double cost_exponent(const nfs_params* p) { return p->r ? double(p->r) : p->rexp; }

// Torus mapping of one problem with temperature eps and bounding box [lo, hi]:
// closed-form Gaussian (r = 2), else a periodization error below exp(-L)
// (L = 20 for FP32 grids, 36 for FP64).
static Scaling near_scaling(const nfs_params* p, double eps, const double* lo, const double* hi) {
  const double L = p->precision == NFS_FP32 ? 20.0 : 36.0;
  if (p->r == 2) return choose_scaling(p->d, 2, eps, p->N, lo, hi);
  if (p->r == 1) return choose_scaling_r1(p->d, eps, L, lo, hi);
  return choose_scaling_rho(p->d, eps, p->rexp, L, lo, hi);
}

// ----------------------------------------------------------------------------- workspace layout
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// One point set (x or y) of every problem, packed in problem order.
template <typename R>
struct CloudBuf {
  long n = 0;                 // total points
  std::vector<long> off;      // B + 1 host offsets into the packed arrays
  R* coords = nullptr;        // sorted tile-local coordinates
  int* perm = nullptr;        // sorted position -> packed input index
  int* keys = nullptr;
  int* counts = nullptr;      // B x nbins
  int* offsets = nullptr;     // B x nbins (global positions)
  int* cursor = nullptr;      // B x nbins
  Chunk* chunks = nullptr;
  long max_chunks = 0;
  int nchunks = 0;
  int* prob_chunks = nullptr;  // B + 1: chunks of problem b
  int* tile_chunks = nullptr;  // nbins + 1 (single problem, per-tile reduction only)
  double* w0s = nullptr;       // sorted weights
  double* w1s = nullptr;       // sorted scalings
  int* runs = nullptr;         // n: run table of each chunk (offsets from the chunk start)
  int* cellstart = nullptr;    // r = 1 with cell order: B x nbins x (T^d + 1) cell starts per tile
  std::vector<int> hcounts;    // host copy of counts (the chunk tables are rebuilt from it)
  int* nruns = nullptr;        // 2 x max_chunks: full runs and single points per chunk
  int* srun = nullptr;         // n: spreading's run table (cell order only)
  int* nsrun = nullptr;        // 3 x max_chunks: its quad entries, pair entries and solo runs per chunk
};

template <typename R>
struct Work {
  int B = 1;
  Geom geo{};
  WindowConst win{};
  void* wpoly = nullptr;     // WindowPoly (FP32) or WindowPoly64 (FP64) coefficients (device)
  int K0 = 0, nbins = 0, chunk = 0;
  long ncell = 0;     // g^d
  long H = 0;         // diagonal table entries per problem, (N/2+1)^d
  CloudBuf<R> X, Y;   // X: x / sources, Y: y / targets
  bool cell_order = false;  // points sorted by cell inside each tile (runs of same-cell points)
  R* stage_coords = nullptr;  // scatter output before the cell sort (max cloud size)
  int* stage_perm = nullptr;
  double* stage_w0 = nullptr;
  double* stage_w1 = nullptr;
  bool two_level = false;
  R* part = nullptr;
  long ecell = 0;
  R* S = nullptr;     // B spread grids, in the format gmode (exact int64 sums unless GRID_REAL)
  int gmode = GRID_REAL;
  long gplane = 0;    // cells of all B grids: the offset of the second plane of GRID_FIX128
  R* U = nullptr;     // B interpolation grids
  cplx<R>* W = nullptr;
  cplx<R>* V = nullptr;
  cplx<R>* spec = nullptr;
  cplx<R>* tw = nullptr;
  R* dtab = nullptr;   // B kernel tables
  R* dtab2 = nullptr;  // B cost tables
  double* inv_phi = nullptr;
  double* partials = nullptr;
  double* st_row = nullptr;   // B x kStat: statistics of the alpha updates
  double* st_col = nullptr;   // B x kStat: statistics of the alpha_t updates
  double* st_eval = nullptr;  // B x kStat: statistics of the evaluation half-steps
  int* pstate = nullptr;      // B x kPState: stop state and completed iterations of each problem
  double* tol2 = nullptr;     // squared tolerance of the stop test (0: run every iteration)
  double* st_rdx = nullptr;   // B x 4
  double* st_rdy = nullptr;   // B x 4
  double* st_cost = nullptr;  // B x 4
  double* wmul_x = nullptr;   // B
  double* wmul_y = nullptr;   // B
  double* leps = nullptr;     // B x kLepsStride: log-domain constants {1/eps, eps}
  double* st_box = nullptr;   // B x kBoxSlot + kBoxSlot: per problem, x box at 0, y box at kBoxVals
  double* unc = nullptr;      // 2 x B x kUncStride: centred form read-out constants (x side, then y)
  double* gfac = nullptr;     // 2 x B: per-problem factors of the gradient on a solver
  double* tabpar = nullptr;   // 2 x B: torus temperature and scale per problem (diagonal tables)
  PlanProb* planprobs = nullptr;  // B: batched key / scatter launches of the plan
  BoxJob* boxjobs = nullptr;      // 2 x B: batched boxes of the plan
  long npartials = 0;             // workgroup partials (kBoxVals doubles each) the partials buffer holds
  double* tmp = nullptr;
  int r = 2;                  // 2: Gaussian; 1: a kernel with a near field (r = 1 or a real exponent)
  double rho = 2.0;           // the cost exponent
  double* nf = nullptr;       // near-field sums (r != 2), per sorted target
  double* nfcoef = nullptr;   // B x kNearStride (r != 2)
  double* nfcoef_c = nullptr; // B x kNearStride: the primal cost's kernel (r != 2)
  int kt = 0;
  int ps = 0;
  std::vector<Scaling> sc;
  size_t bytes = 0;
};

template <typename R>
static void carve(Work<R>& w, const nfs_params* p, int B, long nA, long nB, char* base, int nvec) {
  Carver cv{base};
  const int d = p->d;
  const int g = grid_size(p);
  const int T = p->tile ? p->tile : default_tile(d, p->precision);
  int chunk = p->chunk ? p->chunk : default_chunk(p);
  if (!p->chunk && p->r == 2) {
    // dense clouds (more than 8 points per grid cell): every tile holds many
    // chunks, and their tile flushes contend on the same grid words.  Chunks
    // of 4096 points cut the spreading time of 1e6 uniform points on a 128^2
    // grid from 0.70 to 0.43 ms (FP64), when they still give about one chunk
    // per compute unit (here 247 for 256 units).  At this density a
    // workgroup runs long, so the count matters: 259 chunks of 3906 points
    // take a second round and the 0.70 ms again.
    double cells = double(B);
    for (int c = 0; c < d; ++c) cells *= g;
    const long n = std::max(nA, nB);
    if (double(n) > 8.0 * cells && n >= 200L * 4096) chunk = std::max(chunk, 4096);
  }
  w.B = B;
  w.chunk = chunk;
  w.geo.d = d;
  w.geo.g = g;
  w.geo.N = p->N;
  w.geo.M = p->m;
  w.geo.T = T;
  w.geo.E = T + 2 * p->m + 1;
  int nbins = 1;
  for (int c = 0; c < 3; ++c) {
    w.geo.nt[c] = c < d ? (g + T - 1) / T : 1;
    nbins *= w.geo.nt[c];
  }
  w.nbins = nbins;
  w.K0 = p->N / 2 + 1;
  long ncell = 1, H = 1;
  for (int c = 0; c < d; ++c) {
    ncell *= g;
    H *= w.K0;
  }
  w.ncell = ncell;
  w.H = H;
  auto cloud = [&](CloudBuf<R>& cb, long n) {
    cb.n = n;
    cb.coords = cv.take<R>(size_t(n) * d);
    cb.perm = cv.take<int>(n);
    cb.keys = cv.take<int>(n);
    cb.counts = cv.take<int>(size_t(B) * nbins);
    cb.offsets = cv.take<int>(size_t(B) * nbins);
    cb.cursor = cv.take<int>(size_t(B) * nbins);
    cb.max_chunks = n / chunk + std::min<long>(long(B) * nbins, n) + B + 1;
    cb.chunks = cv.take<Chunk>(cb.max_chunks);
    cb.prob_chunks = cv.take<int>(B + 1);
    cb.tile_chunks = cv.take<int>(nbins + 1);
    cb.runs = cv.take<int>(n);
    cb.nruns = cv.take<int>(2 * cb.max_chunks);
    cb.srun = cv.take<int>(n);
    cb.nsrun = cv.take<int>(3 * cb.max_chunks);
    cb.w0s = nvec >= 1 ? cv.take<double>(n) : nullptr;
    cb.w1s = nvec >= 2 ? cv.take<double>(n) : nullptr;
  };
  cloud(w.X, nA);
  cloud(w.Y, nB);
  long ecell = 1, tcells = 1;
  for (int c = 0; c < d; ++c) {
    ecell *= w.geo.E;
    tcells *= T;
  }
  w.ecell = ecell;
  w.cell_order = tcells <= kSortBins;
  if (w.cell_order && p->r != 2) {
    w.X.cellstart = cv.take<int>(size_t(B) * nbins * (tcells + 1));
    w.Y.cellstart = cv.take<int>(size_t(B) * nbins * (tcells + 1));
  }
  if (w.cell_order) {
    const long ns = std::max(nA, nB);
    w.stage_coords = cv.take<R>(size_t(ns) * d);
    w.stage_perm = cv.take<int>(ns);
    w.stage_w0 = nvec >= 1 ? cv.take<double>(ns) : nullptr;
    w.stage_w1 = nvec >= 2 ? cv.take<double>(ns) : nullptr;
  }
  bool two = (p->flags & NFS_FLAG_TILE_REDUCE) && B == 1 && T >= p->m + 1 && (g % T) == 0 && tcells <= 2048;
  for (int c = 0; c < d; ++c) two = two && w.geo.nt[c] >= 3;
  w.two_level = two;
  w.part = two ? cv.take<R>(size_t(std::max(w.X.max_chunks, w.Y.max_chunks)) * ecell) : nullptr;
  w.gmode = spread_grid_mode(w.geo, int(sizeof(R)), two);
  w.gplane = long(B) * ncell;
  w.S = reinterpret_cast<R*>(cv.take<unsigned char>(size_t(B) * ncell * grid_cell_bytes(w.gmode, sizeof(R))));
  w.U = cv.take<R>(size_t(B) * ncell);
  const long rows = ncell / g;
  w.W = cv.take<cplx<R>>(size_t(B) * rows * w.K0);
  w.V = d == 3 ? cv.take<cplx<R>>(size_t(B) * g * (p->N + 1) * w.K0) : nullptr;
  long spec_n = w.K0;
  for (int c = 0; c < d - 1; ++c) spec_n *= (p->N + 1);
  w.spec = cv.take<cplx<R>>(spec_n);
  w.tw = cv.take<cplx<R>>(g);
  w.dtab = cv.take<R>(size_t(B) * H);
  w.dtab2 = cv.take<R>(size_t(B) * H);
  w.inv_phi = cv.take<double>(w.K0);
  w.wpoly = cv.take<double>((sizeof(R) == 4 ? sizeof(WindowPoly) : sizeof(WindowPoly64)) / sizeof(double) + 1);
  const long maxch = std::max(w.X.max_chunks, w.Y.max_chunks);
  w.npartials = std::max<long>(maxch, 1024);
  w.partials = cv.take<double>(size_t(w.npartials) * kBoxVals);
  w.st_row = cv.take<double>(size_t(B) * kStat);
  w.st_col = cv.take<double>(size_t(B) * kStat);
  w.st_eval = cv.take<double>(size_t(B) * kStat);
  w.pstate = cv.take<int>(size_t(B) * kPState);
  w.tol2 = cv.take<double>(1);
  w.st_rdx = cv.take<double>(size_t(B) * 4);
  w.st_rdy = cv.take<double>(size_t(B) * 4);
  w.st_cost = cv.take<double>(size_t(B) * 4);
  w.wmul_x = cv.take<double>(B);
  w.wmul_y = cv.take<double>(B);
  w.leps = cv.take<double>(size_t(B) * kLepsStride);
  w.st_box = cv.take<double>(size_t(B) * kBoxSlot + kBoxSlot);
  w.unc = cv.take<double>(size_t(2) * B * kUncStride);
  w.gfac = cv.take<double>(size_t(2) * B);
  w.tabpar = cv.take<double>(size_t(2) * B);
  w.planprobs = cv.take<PlanProb>(B);
  w.boxjobs = cv.take<BoxJob>(size_t(2) * B);
  w.tmp = cv.take<double>(size_t(std::max(nA, nB)) * std::max(d, 1));
  // w.r: 2 for the Gaussian, 1 for every kernel with a near field (r = 1 and real exponents)
  w.r = p->r == 2 ? 2 : 1;
  w.rho = cost_exponent(p);
  if (p->r != 2) {
    w.nf = cv.take<double>(size_t(std::max(nA, nB)));
    w.nfcoef = cv.take<double>(size_t(B) * kNearStride);
    w.nfcoef_c = cv.take<double>(size_t(B) * kNearStride);
    w.kt = int(std::ceil(near_radius(p) * g / T - 1e-12));
    w.ps = near_smooth(p);
  }
  w.bytes = cv.off + 256;
  w.win = make_window(p->m, g, p->N);
}

// Zero the counters and statistics (fill kernels, so a later graph capture
// never records a memset).
template <typename R>
static int zero_state(Work<R>& w, hipStream_t st) {
  for (double* s : {w.st_row, w.st_col, w.st_eval}) NFS_HIP(launch_fill(s, sizeof(double) * kStat * w.B, st));
  NFS_HIP(launch_fill(w.pstate, sizeof(int) * kPState * w.B, st));
  NFS_HIP(launch_fill(w.tol2, sizeof(double), st));
  for (double* s : {w.st_rdx, w.st_rdy, w.st_cost}) NFS_HIP(launch_fill(s, sizeof(double) * 4 * w.B, st));
  return NFS_OK;
}

// ----------------------------------------------------------------------------- plan stage
// Bounding box of up to two clouds plus the statistics of one weight vector,
// written to out[0..8] on the device (no synchronization).
static int box_launch(double* out, double* partials, int d, const double* p0, long n0,
                      const double* p1, long n1, const double* w, long nw, hipStream_t st, int wsum = 0) {
  BoxArgs b{};
  b.wsum = wsum;
  b.pts[0] = p0;
  b.n[0] = n0;
  b.pts[1] = p1;
  b.n[1] = n1;
  b.w = w;
  b.nw = nw;
  b.d = d;
  b.partials = partials;
  b.out = out;
  NFS_HIP(launch_bbox(b, st));
  return NFS_OK;
}

// Counting sort of every problem's points by tile, and the chunk table.
// `sc` gives each problem's torus mapping (scale 0: points already on the torus).
// Chunk tables of a cloud from its host tile counts: each tile's points in
// ceil(count / chunk) chunks of near-equal size.  With `runs` (points already
// sorted) the per-chunk run tables are rebuilt as well.
template <typename R>
static int build_chunks(Work<R>& w, CloudBuf<R>& cb, int chunk, bool runs, hipStream_t st) {
  const int B = w.B, nb = w.nbins, d = w.geo.d;
  const std::vector<int>& counts = cb.hcounts;
  std::vector<Chunk> chunks;
  std::vector<int> prob_chunks(B + 1), tile_chunks(nb + 1);
  chunks.reserve(cb.max_chunks);
  for (int b = 0; b < B; ++b) {
    prob_chunks[b] = int(chunks.size());
    long acc = cb.off[b];
    for (int t = 0; t < nb; ++t) {
      const int cnt = counts[size_t(b) * nb + t];
      if (B == 1) tile_chunks[t] = int(chunks.size());
      const int nch = (cnt + chunk - 1) / chunk;
      for (int c = 0; c < nch; ++c) {
        const int s0 = int(int64_t(cnt) * c / nch), s1 = int(int64_t(cnt) * (c + 1) / nch);
        chunks.push_back(Chunk{t, int(acc) + s0, s1 - s0, b});
      }
      acc += cnt;
    }
    // 3-D: largest chunks first inside the problem's range.  Workgroups are
    // handed out in launch order, so the heavy chunks start first and the
    // light ones fill in behind them (3-D mixture: spreading 1.65 -> 1.45 ms).
    // In 2-D tile order is faster (its neighbouring halos share L2; largest
    // first took spreading on the 2-D mixture from 61 to 63 us), and the
    // per-tile reduction needs each tile's chunks adjacent.
    if (!w.two_level && d == 3)
      std::stable_sort(chunks.begin() + prob_chunks[b], chunks.end(),
                       [](const Chunk& u, const Chunk& v) { return u.count > v.count; });
  }
  prob_chunks[B] = int(chunks.size());
  tile_chunks[nb] = int(chunks.size());
  if ((long)chunks.size() > cb.max_chunks) return fail(NFS_EINVAL, "internal: chunk table overflow");
  cb.nchunks = int(chunks.size());
  NFS_HIP(hipMemcpyAsync(cb.chunks, chunks.data(), sizeof(Chunk) * chunks.size(), hipMemcpyHostToDevice, st));
  NFS_HIP(hipMemcpyAsync(cb.prob_chunks, prob_chunks.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, st));
  NFS_HIP(hipMemcpyAsync(cb.tile_chunks, tile_chunks.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice, st));
  if (runs) {
    ChunkRunArgs<R> ca{};
    ca.chunks = cb.chunks;
    ca.nchunks = cb.nchunks;
    ca.d = d;
    ca.T = w.geo.T;
    ca.sorted = w.cell_order;
    ca.G = run_length<R>(d);
    ca.coords = cb.coords;
    ca.runs = cb.runs;
    ca.nruns = cb.nruns;
    ca.srun = w.cell_order ? cb.srun : nullptr;
    ca.nsrun = cb.nsrun;
    NFS_HIP(launch_chunk_runs(ca, st));
  }
  NFS_HIP(hipStreamSynchronize(st));  // the host vectors above must outlive the copies
  return NFS_OK;
}

// side: the cloud is mapped with the centre center + side * shift (x: -1, y: +1;
// the shift is zero outside the centred form).
template <typename R>
static int sort_cloud(Work<R>& w, CloudBuf<R>& cb, const double* pts, const std::vector<Scaling>& sc,
                      const double* v0, const double* v1, hipStream_t st, double side = 0.0) {
  const Geom& geo = w.geo;
  const int B = w.B, nb = w.nbins, d = geo.d;
  NFS_HIP(launch_fill(cb.counts, sizeof(int) * size_t(B) * nb, st));
  NFS_HIP(launch_fill(cb.cursor, sizeof(int) * size_t(B) * nb, st));
  // a batch keys and scatters all its problems in one launch each
  const bool batched = B > 1 && plan_batchable(nb);
  std::vector<PlanProb> probs;
  long pblocks = 0;
  if (batched) {
    probs.resize(B);
    for (int b = 0; b < B; ++b) {
      PlanProb& pp = probs[b];
      pp.o = cb.off[b];
      pp.n = cb.off[b + 1] - cb.off[b];
      for (int c = 0; c < 3; ++c) pp.center[c] = sc[b].center[c] + side * sc[b].shift[c];
      pp.scale = sc[b].scale;
      pp.blk0 = pblocks;
      pblocks += (pp.n + plan_block_points() - 1) / plan_block_points();
    }
    NFS_HIP(hipMemcpyAsync(w.planprobs, probs.data(), sizeof(PlanProb) * B, hipMemcpyHostToDevice, st));
    KeyArgs ka{};
    ka.pts = pts;
    ka.n = pblocks;
    ka.d = d;
    ka.g = geo.g;
    ka.T = geo.T;
    for (int c = 0; c < 3; ++c) ka.nt[c] = geo.nt[c];
    ka.keys = cb.keys;
    ka.counts = cb.counts;
    ka.probs = w.planprobs;
    ka.nprob = B;
    if (pblocks > 0) NFS_HIP(launch_keys(ka, st));
  }
  for (int b = 0; b < B && !batched; ++b) {
    const long o = cb.off[b], n = cb.off[b + 1] - o;
    if (n == 0) continue;
    KeyArgs ka{};
    ka.pts = pts + o * d;
    ka.n = n;
    ka.d = d;
    ka.g = geo.g;
    ka.T = geo.T;
    for (int c = 0; c < 3; ++c) {
      ka.nt[c] = geo.nt[c];
      ka.center[c] = sc[b].center[c] + side * sc[b].shift[c];
    }
    ka.scale = sc[b].scale;
    ka.keys = cb.keys + o;
    ka.counts = cb.counts + size_t(b) * nb;
    NFS_HIP(launch_keys(ka, st));
  }
  std::vector<int>& counts = cb.hcounts;
  counts.assign(size_t(B) * nb, 0);
  std::vector<int> offsets(size_t(B) * nb);
  NFS_HIP(hipMemcpyAsync(counts.data(), cb.counts, sizeof(int) * counts.size(), hipMemcpyDeviceToHost, st));
  NFS_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < B; ++b) {
    long acc = cb.off[b];
    for (int t = 0; t < nb; ++t) {
      offsets[size_t(b) * nb + t] = int(acc);
      acc += counts[size_t(b) * nb + t];
    }
    if (acc != cb.off[b + 1]) return fail(NFS_EINVAL, "internal: tile histogram does not match the point count");
  }
  NFS_HIP(hipMemcpyAsync(cb.offsets, offsets.data(), sizeof(int) * offsets.size(), hipMemcpyHostToDevice, st));
  NFS_TRY(build_chunks(w, cb, w.chunk, false, st));
  if (batched) {
    ScatterArgs<R> sa{};
    sa.pts = pts;
    sa.n = pblocks;
    sa.d = d;
    sa.g = geo.g;
    sa.T = geo.T;
    for (int c = 0; c < 3; ++c) sa.nt[c] = geo.nt[c];
    sa.keys = cb.keys;
    sa.offsets = cb.offsets;
    sa.cursor = cb.cursor;
    sa.coords = w.cell_order ? w.stage_coords : cb.coords;
    sa.perm = w.cell_order ? w.stage_perm : cb.perm;
    sa.w0 = v0;
    sa.w0s = w.cell_order ? w.stage_w0 : cb.w0s;
    sa.w1 = v1;
    sa.w1s = w.cell_order ? w.stage_w1 : cb.w1s;
    sa.probs = w.planprobs;
    sa.nprob = B;
    if (pblocks > 0) NFS_HIP(launch_scatter(sa, st));
  }
  for (int b = 0; b < B && !batched; ++b) {
    const long o = cb.off[b], n = cb.off[b + 1] - o;
    if (n == 0) continue;
    ScatterArgs<R> sa{};
    sa.pts = pts + o * d;
    sa.n = n;
    sa.d = d;
    sa.g = geo.g;
    sa.T = geo.T;
    for (int c = 0; c < 3; ++c) {
      sa.nt[c] = geo.nt[c];
      sa.center[c] = sc[b].center[c] + side * sc[b].shift[c];
    }
    sa.scale = sc[b].scale;
    sa.keys = cb.keys + o;
    sa.offsets = cb.offsets + size_t(b) * nb;
    sa.cursor = cb.cursor + size_t(b) * nb;
    // with cell order the scatter fills the staging arrays, which the tile
    // sort below moves into the final arrays
    sa.coords = w.cell_order ? w.stage_coords : cb.coords;
    sa.perm = w.cell_order ? w.stage_perm : cb.perm;
    sa.idx_base = int(o);
    sa.w0 = v0 ? v0 + o : nullptr;
    sa.w0s = w.cell_order ? w.stage_w0 : cb.w0s;
    sa.w1 = v1 ? v1 + o : nullptr;
    sa.w1s = w.cell_order ? w.stage_w1 : cb.w1s;
    NFS_HIP(launch_scatter(sa, st));
  }
  if (w.cell_order) {
    TileSortArgs<R> ta{};
    ta.counts = cb.counts;
    ta.offsets = cb.offsets;
    ta.ntiles = B * nb;
    ta.d = d;
    ta.T = geo.T;
    ta.in_coords = w.stage_coords;
    ta.in_perm = w.stage_perm;
    ta.in_w0 = v0 ? w.stage_w0 : nullptr;
    ta.in_w1 = v1 ? w.stage_w1 : nullptr;
    ta.coords = cb.coords;
    ta.perm = cb.perm;
    ta.w0s = v0 ? cb.w0s : nullptr;
    ta.w1s = v1 ? cb.w1s : nullptr;
    ta.cellstart = cb.cellstart;
    NFS_HIP(launch_tile_sort(ta, st));
  }
  ChunkRunArgs<R> ca{};
  ca.chunks = cb.chunks;
  ca.nchunks = cb.nchunks;
  ca.d = d;
  ca.T = geo.T;
  ca.sorted = w.cell_order;
  ca.G = run_length<R>(d);
  ca.coords = cb.coords;
  ca.runs = cb.runs;
  ca.nruns = cb.nruns;
  ca.srun = w.cell_order ? cb.srun : nullptr;
  ca.nsrun = cb.nsrun;
  NFS_HIP(launch_chunk_runs(ca, st));
  NFS_HIP(hipStreamSynchronize(st));  // host vectors above must outlive the copies
  return NFS_OK;
}

// Diagonal tables from samples: the Fourier coefficients of a regularized
// kernel on the torus (Section 3.1: the polynomial inside the near-field
// radius, the kernel outside) as the DFT of its samples on the oversampled
// grid, truncated to |k_c| <= N/2.  One problem at a time through the adjoint
// NFFT's forward passes (w.U -> w.W [-> w.V] -> w.spec).  coef: the device
// coefficient blocks (B x kNearStride); cost: the primal cost's kernel
// (blocks of w.nfcoef_c) instead of K; tables: B x H outputs.
template <typename R>
static int sampled_tables(Work<R>& w, const double* coef, int cost, R* tables, hipStream_t st) {
  const Geom& geo = w.geo;
  const int g = geo.g, N = geo.N, d = geo.d, K0 = w.K0;
  const long rows = w.ncell / g;
  AxisArgs<R> ax{};
  ax.L = g;
  ax.N = N;
  ax.d = d;
  ax.tw = w.tw;
  ax.mul = Multiplier{nullptr, -1, 0};
  for (int b = 0; b < w.B; ++b) {
    R* tab = tables + size_t(b) * w.H;
    if (!(w.sc[b].eps_t > 0.0)) {
      NFS_HIP(launch_fill(tab, sizeof(R) * w.H, st));
      continue;
    }
    NFS_HIP(launch_kernel_samples<R>(d, g, coef + size_t(b) * kNearStride, cost, w.U, st));
    RowArgs<R> ra{};
    ra.mode = ROW_R2C;
    ra.L = g;
    ra.N = N;
    ra.nrows = int(rows);
    ra.real_io = w.U;
    ra.gmode = GRID_REAL;
    ra.grid_plane = w.gplane;
    ra.spec = d == 1 ? w.spec : w.W;
    ra.zero_src = 0;
    ra.tw = w.tw;
    NFS_HIP(launch_rows(ra, st));
    if (d >= 2) {
      const cplx<R>* cur = w.W;
      if (d == 3) {
        AxisArgs<R> a1 = ax;
        a1.mode = AX_FWD;
        a1.in = w.W;
        a1.out = w.V;
        a1.nin = g;
        a1.nout = N + 1;
        a1.out_centered = 1;
        a1.in_stride = a1.out_stride = K0;
        a1.in_ostride = long(g) * K0;
        a1.out_ostride = long(N + 1) * K0;
        a1.inner = K0;
        a1.npen = long(g) * K0;
        NFS_HIP(launch_axis(a1, st));
        cur = w.V;
      }
      const long inner = d == 2 ? K0 : long(N + 1) * K0;
      AxisArgs<R> a0 = ax;
      a0.mode = AX_FWD;
      a0.in = cur;
      a0.out = w.spec;
      a0.nin = g;
      a0.nout = N + 1;
      a0.out_centered = 1;
      a0.in_stride = a0.out_stride = inner;
      a0.inner = int(inner);
      a0.npen = inner;
      NFS_HIP(launch_axis(a0, st));
    }
    NFS_HIP(launch_spec_table<R>(d, N, g, w.spec, w.inv_phi, tab, st));
  }
  return NFS_OK;
}

template <typename R>
static int upload_tables(Work<R>& w, const nfs_params* p, hipStream_t st) {
  const int g = w.geo.g;
  // FFT twiddles, pass by pass in the device's pass order: a pass of radix Rd
  // after Ns = (product of the earlier radices) > 1 holds e^(-2 pi i m k /
  // (Rd Ns)) at (m - 1) Ns + k, m = 1..Rd-1, k < Ns.  The tables telescope to
  // g - (first radix) < g entries.
  std::vector<cplx<R>> tw(g, cplx<R>{R(0), R(0)});
  int bits_g = 0;
  while ((1 << bits_g) < g) ++bits_g;
  long off = 0, Ns = 1;
  for (int rem = bits_g; rem > 0;) {
    const int bits = fft_pass_bits(rem);
    const long Rd = 1L << bits;
    if (Ns > 1) {
      for (long m = 1; m < Rd; ++m)
        for (long k = 0; k < Ns; ++k) {
          const double a = -2.0 * kPi * double(m * k) / double(Rd * Ns);
          tw[off + (m - 1) * Ns + k] = cplx<R>{R(std::cos(a)), R(std::sin(a))};
        }
      off += (Rd - 1) * Ns;
    }
    Ns <<= bits;
    rem -= bits;
  }
  NFS_HIP(hipMemcpyAsync(w.tw, tw.data(), sizeof(cplx<R>) * g, hipMemcpyHostToDevice, st));
  const std::vector<double> phi = window_hat_table(p->N, p->m, g, w.win);
  std::vector<double> iphi(w.K0);
  for (int k = 0; k < w.K0; ++k) iphi[k] = 1.0 / phi[k];
  NFS_HIP(hipMemcpyAsync(w.inv_phi, iphi.data(), sizeof(double) * w.K0, hipMemcpyHostToDevice, st));
  if constexpr (sizeof(R) == 4) {
    const WindowPoly wp = make_window_poly(p->m, w.win);
    NFS_HIP(hipMemcpyAsync(w.wpoly, &wp, sizeof(WindowPoly), hipMemcpyHostToDevice, st));
  } else {
    const WindowPoly64 wp = make_window_poly64(p->m, w.win);
    NFS_HIP(hipMemcpyAsync(w.wpoly, &wp, sizeof(WindowPoly64), hipMemcpyHostToDevice, st));
  }
  std::vector<R> t2;
  bool any = false;
  for (int b = 0; b < w.B; ++b) any = any || w.sc[b].eps_t > 0.0;
  if (any && p->r != 2) {
    const double eI = near_radius(p);
    const int ps = near_smooth(p);
    const double rho = cost_exponent(p);
    // The diagonal table comes from samples of K_R on the grid (a DFT on the
    // device, the same for r = 1 and real exponents: a closed-form transform
    // plus a radial quadrature of K - K_R on the host took 0.5 s per 2-D
    // problem at N = 256, and the samples are as accurate).  The primal cost
    // <pi, C> needs the cost-weighted kernel's table and near field as well.
    const bool cost = (p->flags & NFS_FLAG_PRIMAL_COST) != 0;
    t2.assign(size_t(w.B) * w.H, R(0));
    std::vector<double> coef(size_t(w.B) * kNearStride, 0.0), coefc(size_t(w.B) * kNearStride, 0.0);
    for (int b = 0; b < w.B; ++b) {
      const double e = w.sc[b].eps_t;
      const std::vector<double> cf = nearfield_poly(e, eI, ps, rho);
      double* c = coef.data() + size_t(b) * kNearStride;
      c[0] = 1.0 / (e * g);
      c[1] = (eI * g) * (eI * g);
      c[2] = 1.0 / c[1];
      c[3] = ps;
      for (int j = 0; j < ps; ++j) c[4 + j] = cf[j];
      c[kNearRhoHalf] = 0.5 * rho;
      c[kNearRhoInv] = 1.0 / (e * std::pow(double(g), rho));  // (cells)^rho -> r^rho / eps_t
      if (cost) {
        // the primal cost's kernel |z|^rho exp(-|z|^rho/eps) in the caller's units:
        // (r_t / s)^rho exp(-r_t^rho / eps_t), regularized by its own polynomial
        double* cc = coefc.data() + size_t(b) * kNearStride;
        const double sr = std::pow(w.sc[b].scale, rho);
        std::copy(c, c + kNearStride, cc);
        if (e > 0.0) {
          const std::vector<double> cfc = nearfield_poly(e, eI, ps, rho, true);
          for (int j = 0; j < ps; ++j) cc[4 + j] = cfc[j] / sr;
        }
        cc[kNearCostMul] = 1.0 / (std::pow(double(g), rho) * sr);
      }
    }
    NFS_HIP(hipMemcpyAsync(w.dtab2, t2.data(), sizeof(R) * t2.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(hipMemcpyAsync(w.nfcoef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(hipMemcpyAsync(w.nfcoef_c, coefc.data(), sizeof(double) * coefc.size(), hipMemcpyHostToDevice, st));
    NFS_TRY(sampled_tables(w, w.nfcoef, 0, w.dtab, st));
    if (cost) NFS_TRY(sampled_tables(w, w.nfcoef_c, 1, w.dtab2, st));
  } else if (any) {
    // closed form evaluated on the device for all problems at once (the host
    // loop over 512 problems' 129^2 tables took 48 ms of the batch's plan)
    std::vector<double> pb(size_t(2) * w.B);
    for (int b = 0; b < w.B; ++b) {
      pb[2 * b] = w.sc[b].eps_t;
      pb[2 * b + 1] = w.sc[b].scale;
    }
    NFS_HIP(hipMemcpyAsync(w.tabpar, pb.data(), sizeof(double) * pb.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(launch_gauss_tables<R>(p->d, p->N, w.B, w.tabpar, w.inv_phi, w.dtab, w.dtab2, st));
  }
  NFS_HIP(hipStreamSynchronize(st));
  return NFS_OK;
}

// ----------------------------------------------------------------------------- the fast-summation chain
// B stacked grids S (zero on entry) -> U, with the per-problem multiplier
// applied in LDS between the forward and inverse passes of axis 0.  The
// forward pass zeroes S again after reading it.
template <typename R>
static hipError_t fft_chain(Work<R>& w, const R* table, int deriv, hipStream_t st, bool keep_src = false) {
  const Geom& geo = w.geo;
  const int g = geo.g, N = geo.N, d = geo.d, K0 = w.K0, B = w.B;
  Multiplier mu{table, deriv, w.H};
  if (double(B) * double(w.H) >= 4294967296.0) return hipErrorInvalidValue;  // 32-bit table offsets
  hipError_t e;
  if (d == 1) {
    RowArgs<R> ra{};
    ra.mode = ROW_FUSED1D;
    ra.L = g;
    ra.N = N;
    ra.nrows = B;
    ra.real_in = w.S;
    ra.gmode = w.gmode;
    ra.grid_plane = w.gplane;
    ra.real_io = w.U;
    ra.zero_src = keep_src ? 0 : 1;
    ra.tw = w.tw;
    ra.mul = mu;
    return launch_rows(ra, st);
  }
  const long rows = w.ncell / g;  // per problem
  RowArgs<R> ra{};
  ra.mode = ROW_R2C;
  ra.L = g;
  ra.N = N;
  ra.nrows = int(rows * B);
  ra.real_io = w.S;
  ra.gmode = w.gmode;
  ra.grid_plane = w.gplane;
  ra.spec = w.W;
  ra.zero_src = keep_src ? 0 : 1;
  ra.tw = w.tw;
  if ((e = launch_rows(ra, st)) != hipSuccess) return e;
  AxisArgs<R> ax{};
  ax.L = g;
  ax.N = N;
  ax.d = d;
  ax.tw = w.tw;
  ax.mul = mu;
  if (d == 2) {
    ax.mode = AX_FUSED;
    ax.in = w.W;
    ax.out = w.W;
    ax.nin = g;
    ax.nout = g;
    ax.in_stride = ax.out_stride = K0;
    ax.in_ostride = ax.out_ostride = long(g) * K0;
    ax.inner = K0;
    ax.npen = long(B) * K0;
    if ((e = launch_axis(ax, st)) != hipSuccess) return e;
  } else {
    // axis 1 forward: W[b l0][l1][k2] -> V[b l0][k1'][k2]
    AxisArgs<R> a1 = ax;
    a1.mode = AX_FWD;
    a1.in = w.W;
    a1.out = w.V;
    a1.nin = g;
    a1.nout = N + 1;
    a1.out_centered = 1;
    a1.in_stride = K0;
    a1.out_stride = K0;
    a1.in_ostride = long(g) * K0;
    a1.out_ostride = long(N + 1) * K0;
    a1.inner = K0;
    a1.npen = long(B) * g * K0;
    if ((e = launch_axis(a1, st)) != hipSuccess) return e;
    // axis 0 fused: V[b][l0][k1' k2], one problem per outer group
    AxisArgs<R> a0 = ax;
    a0.mode = AX_FUSED;
    a0.in = w.V;
    a0.out = w.V;
    a0.nin = g;
    a0.nout = g;
    a0.in_stride = a0.out_stride = long(N + 1) * K0;
    a0.in_ostride = a0.out_ostride = long(g) * (N + 1) * K0;
    a0.inner = (N + 1) * K0;
    a0.npen = long(B) * (N + 1) * K0;
    if ((e = launch_axis(a0, st)) != hipSuccess) return e;
    AxisArgs<R> a2 = ax;
    a2.mode = AX_INV;
    a2.in = w.V;
    a2.out = w.W;
    a2.nin = N + 1;
    a2.in_centered = 1;
    a2.nout = g;
    a2.in_stride = K0;
    a2.out_stride = K0;
    a2.in_ostride = long(N + 1) * K0;
    a2.out_ostride = long(g) * K0;
    a2.inner = K0;
    a2.npen = long(B) * g * K0;
    if ((e = launch_axis(a2, st)) != hipSuccess) return e;
  }
  RowArgs<R> rb{};
  rb.mode = ROW_C2R;
  rb.L = g;
  rb.N = N;
  rb.nrows = int(rows * B);
  rb.real_io = w.U;
  rb.spec = w.W;
  rb.tw = w.tw;
  return launch_rows(rb, st);
}

template <typename R>
static SpreadArgs<R> spread_args(Work<R>& w, const CloudBuf<R>& src, const double* weights, const double* wmul) {
  SpreadArgs<R> a{};
  a.geo = w.geo;
  a.coords = src.coords;
  a.w = weights;
  a.wmul = wmul;
  a.wconst = 1.0;
  a.chunks = src.chunks;
  a.runs = src.runs;
  a.nruns = src.nruns;
  a.srun = w.cell_order ? src.srun : nullptr;
  a.nsrun = src.nsrun;
  a.cell_order = w.cell_order;
  a.grid = w.S;
  a.grid_stride = w.ncell;
  a.gmode = w.gmode;
  a.grid_plane = w.gplane;
  a.win = w.win;
  a.wpoly = w.wpoly;
  return a;
}

// Spreading into the grids S (zero on entry): LDS tiles flushed straight to
// the grid with global atomics, or (single problem, NFS_FLAG_TILE_REDUCE)
// chunk tiles summed per (tile, neighbour).
template <typename R>
static hipError_t spread(Work<R>& w, const CloudBuf<R>& src, const double* weights, const double* wmul,
                         double wconst, hipStream_t st, const int* pstate = nullptr) {
  SpreadArgs<R> a = spread_args(w, src, weights, wmul);
  a.wconst = wconst;
  a.pstate = pstate;
  if (!w.two_level) return launch_spread(a, src.nchunks, st);
  a.part = w.part;
  hipError_t e = launch_spread(a, src.nchunks, st);
  if (e != hipSuccess) return e;
  ReduceArgs<R> r{};
  r.geo = w.geo;
  r.part = w.part;
  r.tile_chunks = src.tile_chunks;
  r.grid = w.S;
  r.pstate = pstate;
  return launch_spread_reduce(r, w.nbins, st);
}

template <typename R>
static InterpArgs<R> interp_args(Work<R>& w, const CloudBuf<R>& tgt, int epi, const double* wmul_src) {
  InterpArgs<R> a{};
  a.geo = w.geo;
  a.coords = tgt.coords;
  a.chunks = tgt.chunks;
  a.runs = tgt.runs;
  a.nruns = tgt.nruns;
  a.cell_order = w.cell_order;
  a.grid = w.U;
  a.grid_stride = w.ncell;
  a.win = w.win;
  a.wpoly = w.wpoly;
  a.norm = 1.0;
  a.wmul_src = wmul_src;
  a.epi = epi;
  a.perm = tgt.perm;
  a.out_stride = 1;
  a.partials = w.partials;
  a.nprob = w.B;
  a.prob_chunks = tgt.prob_chunks;
  return a;
}

// Near-field correction (r = 1 or a real exponent) of the product with sources `src` at the
// targets `tgt`, into w.nf (sorted target order, normalized like the spread).
template <typename R>
static hipError_t near_field(Work<R>& w, const CloudBuf<R>& src, const CloudBuf<R>& tgt, const double* weights,
                             const double* wmul, double wconst, hipStream_t st, const int* pstate = nullptr,
                             bool cost = false) {
  NearArgs<R> a{};
  a.geo = w.geo;
  a.tcoords = tgt.coords;
  a.tchunks = tgt.chunks;
  a.scoords = src.coords;
  a.sw = weights;
  a.soffsets = src.offsets;
  a.scounts = src.counts;
  a.wmul = wmul;
  a.wconst = wconst;
  a.coef = cost ? w.nfcoef_c : w.nfcoef;
  a.kt = w.kt;
  a.ps = w.ps;
  a.out = w.nf;
  a.pstate = pstate;
  a.scell = src.cellstart;
  a.real_exp = w.rho != 1.0;
  a.cost = cost;
  return launch_nearfield(a, tgt.nchunks, st);
}

// Gradient of the near-field correction (r = 1 or a real exponent) of the product with sources
// `src` at the targets `tgt`: d components in torus units, component c at
// out + c * tgt.n (sorted target order, normalized like the spread).
template <typename R>
static hipError_t near_field_grad(Work<R>& w, const CloudBuf<R>& src, const CloudBuf<R>& tgt, const double* weights,
                                  const double* wmul, double wconst, double* out, hipStream_t st) {
  NearArgs<R> a{};
  a.geo = w.geo;
  a.tcoords = tgt.coords;
  a.tchunks = tgt.chunks;
  a.scoords = src.coords;
  a.sw = weights;
  a.soffsets = src.offsets;
  a.scounts = src.counts;
  a.wmul = wmul;
  a.wconst = wconst;
  a.coef = w.nfcoef;
  a.kt = w.kt;
  a.ps = w.ps;
  a.out = out;
  a.out_plane = tgt.n;
  a.real_exp = w.rho != 1.0;
  return launch_nearfield_grad(a, tgt.nchunks, st);
}

// One Sinkhorn half-step for every problem: spread the scalings of `src`,
// transform, and update (or evaluate) the scalings of `tgt` (eq. (S1) via
// eq. (fastsum)).  In the log domain (EPI_LOGSINK / EPI_LOGEVAL, Algorithm 4)
// src.w1s and tgt.w1s hold potentials, wmul_* their per-problem maxima, and
// the spread weights exp((gamma - max gamma)/eps) go through w.tmp.
// `half` (iterations only): 0 for the alpha update, 1 for the alpha_t update;
// it hands every kernel the problems' stop state (stopped problems are
// skipped) and `src_l1` (the stats slot holding the l1 norm of the source
// weights, scaling form only) to the interpolation.  Evaluation half-steps
// pass half = -1 and run for every problem.
template <typename R>
static hipError_t half_step(Work<R>& w, CloudBuf<R>& src, CloudBuf<R>& tgt, double* wmul_src, double* wmul_tgt,
                            double* stats, int epi, hipStream_t st, int half = -1, const double* src_l1 = nullptr) {
  const bool logd = epi == EPI_LOGSINK || epi == EPI_LOGEVAL;
  const int* ps = half >= 0 ? w.pstate : nullptr;
  const double* wv = src.w1s;
  const double* wm = wmul_src;
  hipError_t e;
  if (logd) {
    if ((e = launch_logweights(src.chunks, src.nchunks, src.w1s, wmul_src, w.leps, w.tmp, ps, st)) != hipSuccess)
      return e;
    wv = w.tmp;
    wm = nullptr;
  }
  if ((e = spread(w, src, wv, wm, 1.0, st, ps)) != hipSuccess) return e;
  if ((e = fft_chain(w, w.dtab, -1, st)) != hipSuccess) return e;
  if (w.r == 1 && (e = near_field(w, src, tgt, wv, wm, 1.0, st, ps)) != hipSuccess) return e;
  InterpArgs<R> ia = interp_args(w, tgt, epi, wmul_src);
  if (w.r == 1) ia.nf = w.nf;
  ia.leps = w.leps;
  ia.p = tgt.w0s;
  ia.alpha = tgt.w1s;
  ia.stats = stats;
  ia.wmul_next = (epi == EPI_SINK || epi == EPI_LOGSINK) ? wmul_tgt : nullptr;
  if (half >= 0) {
    ia.pstate = w.pstate;
    ia.tol2 = w.tol2;
    ia.half = half;
    ia.src_l1 = logd ? nullptr : src_l1;
  }
  return launch_interp(ia, tgt.nchunks, st);
}

// ----------------------------------------------------------------------------- fast summation / NFFT
// out_i = tscale_i sum_j wv_j wv2_j K(tgt_i - src_j); wv2 and tscale are optional
// (the coupling-vector product passes the scalings there).
template <typename R>
static int do_fastsum(const nfs_params* p, const double* src, int64_t ns, const double* wv, const double* tgt,
                      int64_t nt, double* out, void* ws, size_t wsb, hipStream_t st, const double* wv2 = nullptr,
                      const double* tscale = nullptr) {
  Work<R> w;
  carve(w, p, 1, ns, nt, nullptr, 1);
  if (wsb < w.bytes) return fail(NFS_EWORKSPACE, "workspace too small");
  carve(w, p, 1, ns, nt, static_cast<char*>(ws), 1);
  w.X.off = {0, ns};
  w.Y.off = {0, nt};
  NFS_TRY(zero_state(w, st));
  if (wv2) {
    NFS_HIP(launch_mul(wv, wv2, ns, w.tmp, st));
    wv = w.tmp;
  }
  double box[kBoxVals];
  NFS_TRY(box_launch(w.st_box, w.partials, p->d, src, ns, tgt, nt, wv, ns, st));
  NFS_HIP(hipMemcpyAsync(box, w.st_box, sizeof(box), hipMemcpyDeviceToHost, st));
  NFS_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(box[i])) return fail(NFS_EINVAL, "non-finite point coordinates or weights");
  w.sc = {near_scaling(p, p->eps, box, box + 3)};
  NFS_TRY(sort_cloud(w, w.X, src, w.sc, wv, nullptr, st));
  NFS_TRY(sort_cloud(w, w.Y, tgt, w.sc, tscale, nullptr, st));
  NFS_TRY(upload_tables(w, p, st));
  NFS_HIP(launch_fill(w.S, grid_cell_bytes(w.gmode, sizeof(R)) * w.ncell, st));
  const double wmax = box[6] > 0.0 ? box[6] : 1.0;
  NFS_HIP(spread(w, w.X, w.X.w0s, nullptr, 1.0 / wmax, st));
  NFS_HIP(fft_chain(w, w.dtab, -1, st));
  if (w.r == 1) NFS_HIP(near_field(w, w.X, w.Y, w.X.w0s, nullptr, 1.0 / wmax, st));
  InterpArgs<R> ia = interp_args(w, w.Y, EPI_OUT, nullptr);
  if (w.r == 1) ia.nf = w.nf;
  ia.norm = wmax;
  ia.out = out;
  if (tscale) ia.scale_vec = w.Y.w0s;
  NFS_HIP(launch_interp(ia, w.Y.nchunks, st));
  NFS_HIP(hipStreamSynchronize(st));
  return NFS_OK;
}

// Workspace bytes of do_fastsum (one weight vector per cloud).
template <typename R>
static size_t fastsum_bytes(const nfs_params* p, int64_t ns, int64_t nt) {
  Work<R> w;
  carve(w, p, 1, ns, nt, nullptr, 1);
  return w.bytes;
}

// ----------------------------------------------------------------------------- allocation-free fast summation
// Scratch of nfs_fastsum_apply_noalloc: a file-scope device array, one copy
// on every GPU the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy: that name is a host
// stand-in, not a device address.  Each device's address is looked up once,
// with that device current, and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = size_t(NFS_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int scratch_address(void** out) {
  int dev = -1;
  NFS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NFS_EUNSUPPORTED, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    NFS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(NFS_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NFS_OK;
}

template <typename R>
static int do_nfft(const nfs_params* p, bool adjoint, const double* pts, int64_t n, const double* wv,
                   const double* fhat_in, double* fhat_out, double* out, void* ws, size_t wsb, hipStream_t st) {
  Work<R> w;
  carve(w, p, 1, n, 1, nullptr, 1);
  if (wsb < w.bytes) return fail(NFS_EWORKSPACE, "workspace too small");
  carve(w, p, 1, n, 1, static_cast<char*>(ws), 1);
  w.X.off = {0, n};
  w.Y.off = {0, 0};
  NFS_TRY(zero_state(w, st));
  double box[kBoxVals];
  NFS_TRY(box_launch(w.st_box, w.partials, p->d, pts, n, nullptr, 0, wv, wv ? n : 0, st));
  NFS_HIP(hipMemcpyAsync(box, w.st_box, sizeof(box), hipMemcpyDeviceToHost, st));
  NFS_HIP(hipStreamSynchronize(st));
  for (int c = 0; c < p->d; ++c)
    if (!(box[c] >= -0.5) || !(box[3 + c] < 0.5)) return fail(NFS_EINVAL, "NFFT points must lie in [-1/2, 1/2)^d");
  Scaling sc{};
  sc.scale = 0.0;  // points are already torus coordinates
  w.sc = {sc};
  NFS_TRY(sort_cloud(w, w.X, pts, w.sc, wv, nullptr, st));
  NFS_TRY(upload_tables(w, p, st));
  const Geom& geo = w.geo;
  const int g = geo.g, N = geo.N, d = geo.d, K0 = w.K0;
  const long rows = w.ncell / g;
  SpecArgs<R> sp{};
  sp.d = d;
  sp.N = N;
  sp.inv_phi = w.inv_phi;
  sp.scale = 1.0;
  AxisArgs<R> ax{};
  ax.L = g;
  ax.N = N;
  ax.d = d;
  ax.tw = w.tw;
  ax.mul = Multiplier{nullptr, -1, 0};
  if (adjoint) {
    NFS_HIP(launch_fill(w.S, grid_cell_bytes(w.gmode, sizeof(R)) * w.ncell, st));
    // weights normalized by max |w| so every spread contribution is at most one in size
    const double wmax = box[6] > 0.0 ? box[6] : 1.0;
    NFS_HIP(spread(w, w.X, w.X.w0s, nullptr, 1.0 / wmax, st));
    sp.scale = wmax;
    RowArgs<R> ra{};
    ra.mode = ROW_R2C;
    ra.L = g;
    ra.N = N;
    ra.nrows = int(rows);
    ra.real_io = w.S;
    ra.gmode = w.gmode;
    ra.grid_plane = w.gplane;
    ra.spec = d == 1 ? w.spec : w.W;
    ra.tw = w.tw;
    NFS_HIP(launch_rows(ra, st));
    if (d >= 2) {
      const cplx<R>* cur = w.W;
      if (d == 3) {
        AxisArgs<R> a1 = ax;
        a1.mode = AX_FWD;
        a1.in = w.W;
        a1.out = w.V;
        a1.nin = g;
        a1.nout = N + 1;
        a1.out_centered = 1;
        a1.in_stride = a1.out_stride = K0;
        a1.in_ostride = long(g) * K0;
        a1.out_ostride = long(N + 1) * K0;
        a1.inner = K0;
        a1.npen = long(g) * K0;
        NFS_HIP(launch_axis(a1, st));
        cur = w.V;
      }
      const long inner = d == 2 ? K0 : long(N + 1) * K0;
      AxisArgs<R> a0 = ax;
      a0.mode = AX_FWD;
      a0.in = cur;
      a0.out = w.spec;
      a0.nin = g;
      a0.nout = N + 1;
      a0.out_centered = 1;
      a0.in_stride = a0.out_stride = inner;
      a0.inner = int(inner);
      a0.npen = inner;
      NFS_HIP(launch_axis(a0, st));
    }
    sp.spec_in = w.spec;
    sp.user_out = fhat_out;
    NFS_HIP(launch_spec_to_user(sp, st));
  } else {
    sp.user_in = fhat_in;
    sp.spec_out = w.spec;
    NFS_HIP(launch_user_to_spec(sp, st));
    const cplx<R>* rows_in = w.spec;
    if (d >= 2) {
      const long inner = d == 2 ? K0 : long(N + 1) * K0;
      AxisArgs<R> a0 = ax;
      a0.mode = AX_INV;
      a0.in = w.spec;
      a0.out = d == 2 ? w.W : w.V;
      a0.nin = N + 1;
      a0.in_centered = 1;
      a0.nout = g;
      a0.in_stride = a0.out_stride = inner;
      a0.inner = int(inner);
      a0.npen = inner;
      NFS_HIP(launch_axis(a0, st));
      if (d == 3) {
        AxisArgs<R> a2 = ax;
        a2.mode = AX_INV;
        a2.in = w.V;
        a2.out = w.W;
        a2.nin = N + 1;
        a2.in_centered = 1;
        a2.nout = g;
        a2.in_stride = a2.out_stride = K0;
        a2.in_ostride = long(N + 1) * K0;
        a2.out_ostride = long(g) * K0;
        a2.inner = K0;
        a2.npen = long(g) * K0;
        NFS_HIP(launch_axis(a2, st));
      }
      rows_in = w.W;
    }
    RowArgs<R> rb{};
    rb.mode = ROW_C2R;
    rb.L = g;
    rb.N = N;
    rb.nrows = int(rows);
    rb.real_io = w.U;
    rb.spec = const_cast<cplx<R>*>(rows_in);
    rb.tw = w.tw;
    NFS_HIP(launch_rows(rb, st));
    InterpArgs<R> ia = interp_args(w, w.X, EPI_OUT, nullptr);
    ia.out = out;
    NFS_HIP(launch_interp(ia, w.X.nchunks, st));
  }
  NFS_HIP(hipStreamSynchronize(st));
  return NFS_OK;
}

// ----------------------------------------------------------------------------- Sinkhorn
static int check_weights(const double* box, long n, long nt_other, const char* name, int b) {
  const double tol = 1e-12 * double(std::max(n, nt_other));
  const std::string who = std::string(name) + (b >= 0 ? " of problem " + std::to_string(b) : "");
  if (box[7] < 0.0) return fail(NFS_EWEIGHTS, who + " has a negative weight");
  if (!(std::fabs(box[8] - 1.0) <= tol)) return fail(NFS_EWEIGHTS, who + " does not sum to 1");
  return NFS_OK;
}

// Plan shared by solve and grad: per-problem scaling from both clouds, the
// weights (and scalings) gathered into sorted order, tables.
template <typename R>
static int plan_sinkhorn(Work<R>& w, const nfs_params* p, const double* eps, const double* x, const double* mu,
                         const double* y, const double* nu, const double* ax, const double* ay, hipStream_t st) {
  const int B = w.B, d = p->d;
  const bool centred = (p->flags & NFS_FLAG_CENTER) != 0;
  NFS_TRY(zero_state(w, st));
  // per problem, the box of x (with y unless centred) and the weight
  // statistics of mu, then those of nu (with y's box when centred); a batch
  // takes all of them in one launch
  std::vector<BoxJob> jobs;
  for (int b = 0; b < B; ++b) {
    const long ox = w.X.off[b], nx = w.X.off[b + 1] - ox, oy = w.Y.off[b], ny = w.Y.off[b + 1] - oy;
    if (nx < 1 || ny < 1) return fail(NFS_EINVAL, "every problem needs at least one point per cloud");
    double* slot = w.st_box + kBoxSlot * b;
    BoxJob jx{}, jy{};
    jx.box.pts[0] = x + ox * d;
    jx.box.n[0] = nx;
    jx.box.w = mu + ox;
    jx.box.nw = nx;
    jx.box.out = slot;
    jy.box.w = nu + oy;
    jy.box.nw = ny;
    jy.box.out = slot + kBoxVals;
    if (centred) {
      // separate boxes and weighted means of the two clouds
      jx.box.wsum = 1;
      jy.box.pts[0] = y + oy * d;
      jy.box.n[0] = ny;
      jy.box.wsum = 1;
    } else {
      jx.box.pts[1] = y + oy * d;
      jx.box.n[1] = ny;
    }
    jobs.push_back(jx);
    jobs.push_back(jy);
  }
  if (B == 1) {
    for (BoxJob& j : jobs) {
      const BoxArgs& a = j.box;
      NFS_TRY(box_launch(a.out, w.partials, d, a.pts[0], a.n[0], a.pts[1], a.n[1], a.w, a.nw, st, a.wsum));
    }
  } else {
    long total = 0;
    for (BoxJob& j : jobs) {
      j.nblk = bbox_blocks(std::max(std::max(j.box.n[0], j.box.n[1]), j.box.nw));
      total += j.nblk;
    }
    const long njobs = long(jobs.size());
    if (total > w.npartials) {  // fewer workgroups per box, within the partials buffer (>= 2B + 1 slots)
      const long spare = w.npartials - njobs;
      long t2 = 0;
      for (BoxJob& j : jobs) {
        j.nblk = int(std::max<long>(1, long(j.nblk) * spare / total));
        t2 += j.nblk;
      }
      total = t2;
    }
    long blk0 = 0;
    for (BoxJob& j : jobs) {
      j.blk0 = blk0;
      blk0 += j.nblk;
    }
    NFS_HIP(hipMemcpyAsync(w.boxjobs, jobs.data(), sizeof(BoxJob) * jobs.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(launch_bbox_jobs(w.boxjobs, int(njobs), total, d, w.partials, st));
  }
  std::vector<double> box(size_t(B) * kBoxSlot);
  NFS_HIP(hipMemcpyAsync(box.data(), w.st_box, sizeof(double) * box.size(), hipMemcpyDeviceToHost, st));
  NFS_HIP(hipStreamSynchronize(st));
  w.sc.resize(B);
  for (int b = 0; b < B; ++b) {
    const double* bx = box.data() + size_t(kBoxSlot) * b;
    const double* by = bx + kBoxVals;
    for (int i = 0; i < kBoxVals; ++i) {
      const bool used = centred ? (i < 9 + d) : (i < 9);
      if (used && (!std::isfinite(bx[i]) || ((centred || i >= 6) && !std::isfinite(by[i]))))
        return fail(NFS_EINVAL, "non-finite point coordinates or weights");
    }
    const long nx = w.X.off[b + 1] - w.X.off[b], ny = w.Y.off[b + 1] - w.Y.off[b];
    NFS_TRY(check_weights(bx, nx, ny, "mu", B > 1 ? b : -1));
    NFS_TRY(check_weights(by, ny, nx, "nu", B > 1 ? b : -1));
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, shift[3] = {0, 0, 0};
    for (int c = 0; c < d; ++c) {
      if (centred) {
        // shift = (mean y - mean x)/2: x + shift and y - shift have the same weighted mean
        shift[c] = 0.5 * (by[9 + c] / by[8] - bx[9 + c] / bx[8]);
        lo[c] = std::min(bx[c] + shift[c], by[c] - shift[c]);
        hi[c] = std::max(bx[3 + c] + shift[c], by[3 + c] - shift[c]);
      } else {
        lo[c] = bx[c];
        hi[c] = bx[3 + c];
      }
    }
    w.sc[b] = near_scaling(p, eps[b], lo, hi);
    for (int c = 0; c < d; ++c) w.sc[b].shift[c] = shift[c];
  }
  NFS_TRY(sort_cloud(w, w.X, x, w.sc, mu, ax, st, -1.0));
  NFS_TRY(sort_cloud(w, w.Y, y, w.sc, nu, ay, st, 1.0));
  NFS_TRY(upload_tables(w, p, st));
  NFS_HIP(launch_fill(w.S, grid_cell_bytes(w.gmode, sizeof(R)) * size_t(w.B) * w.ncell, st));
  return NFS_OK;
}

// Persistent Sinkhorn state: plan done once, one iteration (10 kernels for
// all problems) captured in a hipGraph on an internal stream and replayed.
struct SolverBase {
  virtual ~SolverBase() {}
  virtual int iterate(int k, hipStream_t caller) = 0;
  virtual int residual(double* err_row, hipStream_t caller) = 0;
  virtual int finish(double* alpha, double* alpha_t, nfs_result* res, hipStream_t caller) = 0;
  virtual int profile(int k, double* stage_ms, hipStream_t caller) = 0;
  virtual int stage_info(double* info) = 0;
  // Tolerance of the per-iteration stop test (eq. (Error)); 0 runs every iteration.
  virtual int set_tol(double tol, hipStream_t caller) = 0;
  // Envelope gradient at the current scalings, on the solver's plan.
  virtual int grad(double* gx, double* gmu, double* gy, double* gnu, hipStream_t caller) = 0;
  // Whether every problem has stopped on the tolerance (synchronizes).
  virtual int all_stopped(bool* all, hipStream_t caller) = 0;
};

template <typename R>
struct Solver : SolverBase {
  nfs_params p{};
  Work<R> w;
  std::vector<double> eps;
  int done = 0;
  hipStream_t gs = nullptr;
  hipEvent_t ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // kGraphIters iterations in one graph: each graph launch leaves a gap of
  // about 8 us on the queue (the 2-D mixture iteration is 0.31 ms), so runs
  // of iterations replay this one and the rest the single-iteration graph.
  static constexpr int kGraphIters = 8;
  hipGraph_t graph_many = nullptr;
  hipGraphExec_t gexec_many = nullptr;
  bool logd = false;  // log domain (Algorithm 4): w1s holds potentials, wmul_* their maxima
  bool centred = false;  // NFS_FLAG_CENTER: the iteration runs on the shifted clouds (Scaling::shift)

  int sink() const { return logd ? EPI_LOGSINK : EPI_SINK; }

  // Constants of the centred form's change of variables (UncenterArgs::pb),
  // x side then y side, uploaded once after the plan.
  int upload_centring(hipStream_t st) {
    const int B = w.B;
    std::vector<double> unc(size_t(2) * B * kUncStride, 0.0);
    for (int side = 0; side < 2; ++side)
      for (int b = 0; b < B; ++b) {
        double* u = unc.data() + (size_t(side) * B + b) * kUncStride;
        const Scaling& sc = w.sc[b];
        double d2 = 0.0;
        u[0] = sc.scale;
        for (int c = 0; c < p.d; ++c) {
          const double delta = 2.0 * sc.shift[c];
          u[1 + c] = sc.center[c];
          u[4 + c] = (side == 0 ? -2.0 : 2.0) * delta / eps[b];
          d2 += delta * delta;
        }
        u[7] = 0.5 * d2 / eps[b];
        u[8] = eps[b];
      }
    NFS_HIP(hipMemcpyAsync(w.unc, unc.data(), sizeof(double) * unc.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(hipStreamSynchronize(st));  // unc is read by the copy
    return NFS_OK;
  }

  // Centred scalings of one cloud (side 0: x, 1: y) to the caller's variables
  // in the caller's order (out), or, with out NULL, the cloud's sorted
  // starting values from the caller's variables to the centred ones in place.
  hipError_t map_centred(CloudBuf<R>& cb, int side, double* out, hipStream_t st) {
    UncenterArgs<R> ua{};
    ua.geo = w.geo;
    ua.chunks = cb.chunks;
    ua.coords = cb.coords;
    ua.perm = out ? cb.perm : nullptr;
    ua.src = cb.w1s;
    ua.out = out ? out : cb.w1s;
    ua.pb = w.unc + size_t(side) * w.B * kUncStride;
    ua.logd = logd;
    return launch_uncenter(ua, cb.nchunks, st);
  }

  // The centred iteration starts from the image of the caller's start (ones,
  // zeros, or the warm start), so its iterates are exactly Algorithm 3's
  // (Algorithm 4's) under the change of variables.  The spread normalization
  // of the y side (scaling form: 1 / max; log domain: the max potential) and
  // the l1 norm the first alpha update reads are taken again from the mapped
  // values.
  int centre_start(hipStream_t st) {
    const int B = w.B;
    NFS_TRY(upload_centring(st));
    NFS_HIP(map_centred(w.X, 0, nullptr, st));
    NFS_HIP(map_centred(w.Y, 1, nullptr, st));
    for (int b = 0; b < B; ++b)
      NFS_HIP(launch_maxsum(w.Y.w1s + w.Y.off[b], w.Y.off[b + 1] - w.Y.off[b], w.partials,
                            w.st_box + 2 * b, st));
    std::vector<double> ms(size_t(B) * 2), wm(B), col(size_t(B) * kStat);
    NFS_HIP(hipMemcpyAsync(ms.data(), w.st_box, sizeof(double) * ms.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(col.data(), w.st_col, sizeof(double) * col.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
      const double mx = ms[2 * b], sum = ms[2 * b + 1];
      if (!std::isfinite(mx) || !std::isfinite(sum) || (!logd && !(mx > 0.0)))
        return fail(NFS_EINVAL, "the centred starting values over- or underflow (use the log domain)");
      wm[b] = logd ? mx : 1.0 / mx;
      col[size_t(b) * kStat + 7] = sum;
    }
    NFS_HIP(hipMemcpyAsync(w.wmul_y, wm.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
    NFS_HIP(hipMemcpyAsync(w.st_col, col.data(), sizeof(double) * col.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(hipStreamSynchronize(st));  // wm and col are read by the copies
    return NFS_OK;
  }
  int eval() const { return logd ? EPI_LOGEVAL : EPI_EVAL; }

  // One iteration: the alpha update (sources y with alpha_t; its epilogue
  // also gives ||E|| of the state before it) and the alpha_t update.
  hipError_t iteration(hipStream_t s) {
    hipError_t e = half_step(w, w.Y, w.X, w.wmul_y, w.wmul_x, w.st_row, sink(), s, 0, w.st_col + 7);
    if (e != hipSuccess) return e;
    return half_step(w, w.X, w.Y, w.wmul_x, w.wmul_y, w.st_col, sink(), s, 1, w.st_row + 7);
  }

  // Chunk size by measurement: rebuild the chunk and run tables for each
  // candidate (the sorted clouds do not change), time 3 iterations after one
  // warm-up, keep the fastest.  The iterations change the scalings and the
  // t <= 0 counters, so both are restored afterwards.
  int autotune(hipStream_t st) {
    const int B = w.B;
    std::vector<int> cands;
    for (int c : {w.chunk, 2 * w.chunk, 4096, 8192})
      if (c >= w.chunk && c <= 32768 && std::find(cands.begin(), cands.end(), c) == cands.end()) cands.push_back(c);
    if (cands.size() < 2) return NFS_OK;
    std::vector<double> hx(w.X.n), hy(w.Y.n), hwx(B), hwy(B), hcol(size_t(B) * kStat);
    NFS_HIP(hipMemcpyAsync(hcol.data(), w.st_col, sizeof(double) * hcol.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(hx.data(), w.X.w1s, sizeof(double) * hx.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(hy.data(), w.Y.w1s, sizeof(double) * hy.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(hwx.data(), w.wmul_x, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(hwy.data(), w.wmul_y, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    NFS_HIP(hipStreamSynchronize(st));
    hipEvent_t e0, e1;
    NFS_HIP(hipEventCreate(&e0));
    NFS_HIP(hipEventCreate(&e1));
    float best = 0.0f;
    int best_chunk = w.chunk;
    int rc = NFS_OK;
    for (int c : cands) {
      if ((rc = build_chunks(w, w.X, c, true, st)) != NFS_OK) break;
      if ((rc = build_chunks(w, w.Y, c, true, st)) != NFS_OK) break;
      hipError_t e = iteration(st);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      for (int i = 0; i < 3 && e == hipSuccess; ++i) e = iteration(st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        rc = fail(NFS_EHIP, std::string("autotune: ") + hipGetErrorString(e));
        break;
      }
      if (c == cands.front() || ms < best) {
        best = ms;
        best_chunk = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    NFS_TRY(rc);
    w.chunk = best_chunk;
    NFS_TRY(build_chunks(w, w.X, best_chunk, true, st));
    NFS_TRY(build_chunks(w, w.Y, best_chunk, true, st));
    NFS_HIP(hipMemcpyAsync(w.X.w1s, hx.data(), sizeof(double) * hx.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(hipMemcpyAsync(w.Y.w1s, hy.data(), sizeof(double) * hy.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(hipMemcpyAsync(w.wmul_x, hwx.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
    NFS_HIP(hipMemcpyAsync(w.wmul_y, hwy.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
    NFS_HIP(launch_fill(w.st_row, sizeof(double) * size_t(B) * kStat, st));
    NFS_HIP(hipMemcpyAsync(w.st_col, hcol.data(), sizeof(double) * hcol.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(launch_fill(w.pstate, sizeof(int) * size_t(B) * kPState, st));
    NFS_HIP(hipStreamSynchronize(st));  // the host copies above must outlive the transfers
    return NFS_OK;
  }

  // Starting scalings (Algorithm 3): alpha = 1; alpha_t = 1, or the caller's
  // positive starting value (already sorted into Y.w1s by the plan); wmul_*
  // normalize the spread weights by their maximum.
  // The l1 norm of the starting alpha_t goes to st_col[kStat b + 7], where the
  // first alpha update reads its source norm.
  int start_scalings(int B, const std::vector<long>& oy, const double* alpha_t0, hipStream_t st) {
    NFS_HIP(launch_fill_double(w.X.w1s, w.X.n, 1.0, st));
    NFS_HIP(launch_fill_double(w.wmul_x, B, 1.0, st));
    std::vector<double> col(size_t(B) * kStat, 0.0);
    if (!alpha_t0) {
      NFS_HIP(launch_fill_double(w.Y.w1s, w.Y.n, 1.0, st));
      NFS_HIP(launch_fill_double(w.wmul_y, B, 1.0, st));
      for (int b = 0; b < B; ++b) col[size_t(b) * kStat + 7] = double(oy[b + 1] - oy[b]);
      NFS_HIP(hipMemcpyAsync(w.st_col, col.data(), sizeof(double) * col.size(), hipMemcpyHostToDevice, st));
      NFS_HIP(hipStreamSynchronize(st));  // col is read by the copy
      return NFS_OK;
    }
    for (int b = 0; b < B; ++b)
      NFS_TRY(box_launch(w.st_box + kBoxSlot * b, w.partials, p.d, nullptr, 0, nullptr, 0,
                         alpha_t0 + oy[b], oy[b + 1] - oy[b], st));
    std::vector<double> box(size_t(B) * kBoxSlot), wm(B);
    NFS_HIP(hipMemcpyAsync(box.data(), w.st_box, sizeof(double) * box.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
      const double* bb = box.data() + size_t(kBoxSlot) * b;
      if (!(bb[7] > 0.0) || !std::isfinite(bb[6])) return fail(NFS_EINVAL, "warm-start alpha_t must be positive and finite");
      wm[b] = 1.0 / bb[6];
      col[size_t(b) * kStat + 7] = bb[8];
    }
    NFS_HIP(hipMemcpyAsync(w.wmul_y, wm.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
    NFS_HIP(hipMemcpyAsync(w.st_col, col.data(), sizeof(double) * col.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(hipStreamSynchronize(st));  // wm and col are read by the copies
    return NFS_OK;
  }

  // Starting potentials (Algorithm 4): beta = 0; gamma = 0, or the caller's
  // finite starting value (sorted into Y.w1s by the plan); wmul_* hold each
  // problem's largest potential, the shift of the spread weights.
  int start_log(int B, const std::vector<long>& oy, const double* gamma0, hipStream_t st) {
    std::vector<double> le(size_t(B) * kLepsStride), shift(B, 0.0);
    for (int b = 0; b < B; ++b) {
      le[kLepsStride * b] = 1.0 / eps[b];
      le[kLepsStride * b + 1] = eps[b];
    }
    NFS_HIP(launch_fill_double(w.X.w1s, w.X.n, 0.0, st));
    NFS_HIP(launch_fill_double(w.wmul_x, B, 0.0, st));
    if (!gamma0) {
      NFS_HIP(launch_fill_double(w.Y.w1s, w.Y.n, 0.0, st));
    } else {
      std::vector<double> ms(size_t(B) * 2);
      for (int b = 0; b < B; ++b)
        NFS_HIP(launch_maxsum(gamma0 + oy[b], oy[b + 1] - oy[b], w.partials, w.st_box + 2 * b, st));
      NFS_HIP(hipMemcpyAsync(ms.data(), w.st_box, sizeof(double) * ms.size(), hipMemcpyDeviceToHost, st));
      NFS_HIP(hipStreamSynchronize(st));
      for (int b = 0; b < B; ++b) {
        if (!std::isfinite(ms[2 * b]) || !std::isfinite(ms[2 * b + 1]))
          return fail(NFS_EINVAL, "warm-start gamma must be finite");
        shift[b] = ms[2 * b];
      }
    }
    NFS_HIP(hipMemcpyAsync(w.wmul_y, shift.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
    NFS_HIP(hipMemcpyAsync(w.leps, le.data(), sizeof(double) * le.size(), hipMemcpyHostToDevice, st));
    // the host vectors above are read by the copies: wait before they go
    NFS_HIP(hipStreamSynchronize(st));
    return NFS_OK;
  }

  int create(const nfs_params* prm, int B, const int64_t* n, const int64_t* nt, const double* eps_in,
             const double* x, const double* mu, const double* y, const double* nu, const double* alpha_t0, void* ws,
             size_t wsb, hipStream_t caller) {
    p = *prm;
    logd = (p.flags & NFS_FLAG_LOG_DOMAIN) != 0;
    centred = (p.flags & NFS_FLAG_CENTER) != 0;
    if (centred && p.r != 2) return fail(NFS_EUNSUPPORTED, "NFS_FLAG_CENTER needs the squared Euclidean cost (r = 2)");

    eps.assign(eps_in, eps_in + B);
    std::vector<long> ox(B + 1, 0), oy(B + 1, 0);
    for (int b = 0; b < B; ++b) {
      ox[b + 1] = ox[b] + n[b];
      oy[b + 1] = oy[b] + nt[b];
    }
    hipStream_t st = caller;
    // carve the workspace for the parameters q, plan, and set the starting values
    auto prepare = [&](const nfs_params& q) -> int {
      w = Work<R>{};
      carve(w, &q, B, ox[B], oy[B], nullptr, 2);
      if (wsb < w.bytes) return fail(NFS_EWORKSPACE, "workspace too small");
      carve(w, &q, B, ox[B], oy[B], static_cast<char*>(ws), 2);
      w.X.off = ox;
      w.Y.off = oy;
      NFS_TRY(plan_sinkhorn(w, &q, eps.data(), x, mu, y, nu, nullptr, alpha_t0, st));
      if (logd) {
        NFS_TRY(start_log(B, oy, alpha_t0, st));
      } else {
        NFS_TRY(start_scalings(B, oy, alpha_t0, st));
      }
      if (centred) NFS_TRY(centre_start(st));
      return NFS_OK;
    };
    const std::vector<int> tiles = tile_candidates(&p);
    if (tiles.size() > 1) {
      // the tile: plan and time one warm-up and three iterations per candidate
      hipEvent_t e0 = nullptr, e1 = nullptr;
      NFS_HIP(hipEventCreate(&e0));
      NFS_HIP(hipEventCreate(&e1));
      float best = 0.0f;
      int best_tile = tiles.front(), rc = NFS_OK;
      for (int T : tiles) {
        nfs_params q = p;
        q.tile = T;
        if ((rc = prepare(q)) != NFS_OK) break;
        hipError_t e = iteration(st);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int i = 0; i < 3 && e == hipSuccess; ++i) e = iteration(st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          rc = fail(NFS_EHIP, std::string("tile autotune: ") + hipGetErrorString(e));
          break;
        }
        if (T == tiles.front() || ms < best) {
          best = ms;
          best_tile = T;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      NFS_TRY(rc);
      p.tile = best_tile;
    }
    NFS_TRY(prepare(p));
    if ((p.flags & NFS_FLAG_AUTOTUNE) && p.r == 2 && !w.two_level) NFS_TRY(autotune(st));
    NFS_HIP(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
    NFS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    NFS_HIP(hipStreamSynchronize(st));
    if (!(p.flags & NFS_FLAG_NO_GRAPH)) {
      hipError_t e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e2 = iteration(gs);
        e = hipStreamEndCapture(gs, &graph);
        if (e2 != hipSuccess) e = e2;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      if (e == hipSuccess) e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e2 = hipSuccess;
        for (int i = 0; i < kGraphIters && e2 == hipSuccess; ++i) e2 = iteration(gs);
        e = hipStreamEndCapture(gs, &graph_many);
        if (e2 != hipSuccess) e = e2;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&gexec_many, graph_many, nullptr, nullptr, 0);
      if (e != hipSuccess) return fail(NFS_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    return NFS_OK;
  }

  ~Solver() override {
    if (gexec) hipGraphExecDestroy(gexec);
    if (graph) hipGraphDestroy(graph);
    if (gexec_many) hipGraphExecDestroy(gexec_many);
    if (graph_many) hipGraphDestroy(graph_many);
    if (gs) {
      hipStreamSynchronize(gs);
      hipStreamDestroy(gs);
    }
    if (ev) hipEventDestroy(ev);
  }

  // Order: caller -> internal stream -> work -> caller.
  int enter(hipStream_t caller) {
    NFS_HIP(hipEventRecord(ev, caller));
    NFS_HIP(hipStreamWaitEvent(gs, ev, 0));
    return NFS_OK;
  }
  int leave(hipStream_t caller) {
    NFS_HIP(hipEventRecord(ev, gs));
    NFS_HIP(hipStreamWaitEvent(caller, ev, 0));
    return NFS_OK;
  }

  int iterate(int k, hipStream_t caller) override {
    if (k <= 0) return NFS_OK;
    NFS_TRY(enter(caller));
    for (int i = 0; i < k;) {
      const bool many = gexec_many && k - i >= kGraphIters;
      hipError_t e = many ? hipGraphLaunch(gexec_many, gs) : (gexec ? hipGraphLaunch(gexec, gs) : iteration(gs));
      if (e != hipSuccess) return fail(NFS_EHIP, std::string("iteration: ") + hipGetErrorString(e));
      i += many ? kGraphIters : 1;
    }
    done += k;
    return leave(caller);
  }

  // Largest row residual over the problems.
  int residual(double* err_row, hipStream_t caller) override {
    NFS_TRY(enter(caller));
    NFS_HIP(half_step(w, w.Y, w.X, w.wmul_y, w.wmul_x, w.st_eval, eval(), gs));
    std::vector<double> h(size_t(w.B) * kStat);
    NFS_HIP(hipMemcpyAsync(h.data(), w.st_eval, sizeof(double) * h.size(), hipMemcpyDeviceToHost, gs));
    NFS_HIP(hipStreamSynchronize(gs));
    double e = 0.0;
    for (int b = 0; b < w.B; ++b) e = std::max(e, std::sqrt(h[size_t(kStat) * b]));
    *err_row = e;
    return leave(caller);
  }

  int profile(int k, double* stage_ms, hipStream_t caller) override {
    if (k <= 0) return fail(NFS_EINVAL, "profile needs k >= 1");
    NFS_TRY(enter(caller));
    std::vector<hipEvent_t> evs(8 * k + 1);
    for (auto& e : evs) NFS_HIP(hipEventCreate(&e));
    int ie = 0;
    NFS_HIP(hipEventRecord(evs[ie++], gs));
    for (int it = 0; it < k; ++it) {
      for (int h = 0; h < 2; ++h) {
        CloudBuf<R>& src = h == 0 ? w.Y : w.X;
        CloudBuf<R>& tgt = h == 0 ? w.X : w.Y;
        double* ws_ = h == 0 ? w.wmul_y : w.wmul_x;
        double* wt_ = h == 0 ? w.wmul_x : w.wmul_y;
        // log domain: the weight pass is timed with the spread
        const double* wv = src.w1s;
        const double* wm = ws_;
        if (logd) {
          NFS_HIP(launch_logweights(src.chunks, src.nchunks, src.w1s, ws_, w.leps, w.tmp, w.pstate, gs));
          wv = w.tmp;
          wm = nullptr;
        }
        NFS_HIP(spread(w, src, wv, wm, 1.0, gs, w.pstate));
        NFS_HIP(hipEventRecord(evs[ie++], gs));
        NFS_HIP(fft_chain(w, w.dtab, -1, gs));
        NFS_HIP(hipEventRecord(evs[ie++], gs));
        if (w.r == 1) NFS_HIP(near_field(w, src, tgt, wv, wm, 1.0, gs, w.pstate));
        NFS_HIP(hipEventRecord(evs[ie++], gs));
        InterpArgs<R> ia = interp_args(w, tgt, sink(), ws_);
        ia.leps = w.leps;
        if (w.r == 1) ia.nf = w.nf;
        ia.p = tgt.w0s;
        ia.alpha = tgt.w1s;
        ia.stats = h == 0 ? w.st_row : w.st_col;
        ia.wmul_next = wt_;
        ia.pstate = w.pstate;
        ia.tol2 = w.tol2;
        ia.half = h;
        ia.src_l1 = logd ? nullptr : (h == 0 ? w.st_col : w.st_row) + 7;
        NFS_HIP(launch_interp(ia, tgt.nchunks, gs));
        NFS_HIP(hipEventRecord(evs[ie++], gs));
      }
    }
    NFS_HIP(hipStreamSynchronize(gs));
    // per half-step: spread | FFT chain | near field | interpolation + update
    double acc[4] = {0, 0, 0, 0};
    float ms;
    for (int i = 1; i < ie; ++i) {
      NFS_HIP(hipEventElapsedTime(&ms, evs[i - 1], evs[i]));
      acc[(i - 1) % 4] += ms;
    }
    NFS_HIP(hipEventElapsedTime(&ms, evs[0], evs[ie - 1]));
    stage_ms[0] = acc[0] / (2.0 * k);
    stage_ms[1] = acc[1] / (2.0 * k);
    stage_ms[2] = acc[3] / (2.0 * k);
    stage_ms[3] = ms / k;
    stage_ms[4] = acc[2] / (2.0 * k);
    for (auto& e : evs) hipEventDestroy(e);
    done += k;
    return leave(caller);
  }

  // Envelope gradient (Proposition 2.3, eq. (14)) at the current scalings,
  // on the plan the iteration uses: the sorted clouds, tables and scalings
  // stay where they are.  x side: alpha_t is spread once, and each axis c
  // applies (2 pi i k_c) D_k to its transform and interpolates at x, times
  // -eps s alpha_i (s the torus scaling); the y side is the same with the
  // clouds exchanged (the kernel is even).  grad_mu = eps log alpha minus its
  // mean over the problem.  Outputs in the caller's (packed) point order.
  int grad(double* gx, double* gmu, double* gy, double* gnu, hipStream_t caller) override {
    if (logd || centred) return fail(NFS_EUNSUPPORTED, "the solver gradient needs the scaling form, uncentred");
    NFS_TRY(enter(caller));
    hipStream_t st = gs;
    const int B = w.B, d = p.d;
    // per problem: -eps_b s_b, whose reciprocal times the spread normalization divides the sums
    std::vector<double> rec(B);
    for (int b = 0; b < B; ++b) rec[b] = 1.0 / (-eps[b] * w.sc[b].scale);
    NFS_HIP(hipMemcpyAsync(w.gfac + B, rec.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
    for (int side = 0; side < 2; ++side) {
      CloudBuf<R>& src = side == 0 ? w.Y : w.X;
      CloudBuf<R>& tgt = side == 0 ? w.X : w.Y;
      double* wm = side == 0 ? w.wmul_y : w.wmul_x;
      double* out = side == 0 ? gx : gy;
      double* outm = side == 0 ? gmu : gnu;
      if (out) {
        NFS_HIP(launch_mul(wm, w.gfac + B, B, w.gfac, st));
        NFS_HIP(spread(w, src, src.w1s, wm, 1.0, st));
        if (w.r == 1) NFS_HIP(near_field_grad(w, src, tgt, src.w1s, wm, 1.0, w.tmp, st));
        for (int c = 0; c < d; ++c) {
          NFS_HIP(fft_chain(w, w.dtab, c, st, c + 1 < d));
          InterpArgs<R> ia = interp_args(w, tgt, EPI_OUT, w.gfac);
          if (w.r == 1) ia.nf = w.tmp + size_t(c) * tgt.n;
          ia.scale_vec = tgt.w1s;
          ia.out = out;
          ia.out_stride = d;
          ia.out_comp = c;
          NFS_HIP(launch_interp(ia, tgt.nchunks, st));
        }
      }
      if (outm)
        for (int b = 0; b < B; ++b) {
          const long o = tgt.off[b];
          NFS_HIP(launch_gradmu(tgt.w1s + o, tgt.off[b + 1] - o, eps[b], w.partials, w.st_cost, outm, st,
                                tgt.perm + o));
        }
    }
    NFS_HIP(hipStreamSynchronize(st));  // rec is read by the copy
    return leave(caller);
  }

  int set_tol(double tol, hipStream_t caller) override {
    NFS_TRY(enter(caller));
    NFS_HIP(launch_fill_double(w.tol2, 1, tol > 0.0 ? tol * tol : 0.0, gs));
    return leave(caller);
  }

  int all_stopped(bool* all, hipStream_t caller) override {
    NFS_TRY(enter(caller));
    std::vector<int> h(size_t(w.B) * kPState);
    NFS_HIP(hipMemcpyAsync(h.data(), w.pstate, sizeof(int) * h.size(), hipMemcpyDeviceToHost, gs));
    NFS_HIP(hipStreamSynchronize(gs));
    bool a = true;
    for (int b = 0; b < w.B; ++b) a = a && h[size_t(kPState) * b] == 2;
    *all = a;
    return leave(caller);
  }

  int stage_info(double* info) override {
    info[0] = double(w.X.n);
    info[1] = double(w.Y.n);
    info[2] = p.d;
    info[3] = double(w.ncell) * w.B;
    info[4] = double(sizeof(R));
    info[5] = w.X.nchunks;
    info[6] = w.Y.nchunks;
    info[7] = std::pow(2.0 * p.m + 1.0, p.d);
    info[8] = w.geo.T;
    return NFS_OK;
  }

  // Read-out of every problem (Algorithm 3 result, eq. (Error), Section 3.2
  // upper value, eq. (15) primal cost); res has B entries.
  int finish(double* alpha, double* alpha_t, nfs_result* res, hipStream_t caller) override {
    NFS_TRY(enter(caller));
    hipStream_t st = gs;
    const int B = w.B;
    // row residual of eq. (Error): one extra product K alpha_t
    NFS_HIP(half_step(w, w.Y, w.X, w.wmul_y, w.wmul_x, w.st_eval, eval(), st));
    std::vector<double> ev_row(size_t(B) * kStat), ev_col(size_t(B) * kStat);
    NFS_HIP(hipMemcpyAsync(ev_row.data(), w.st_eval, sizeof(double) * ev_row.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(half_step(w, w.X, w.Y, w.wmul_x, w.wmul_y, w.st_eval, eval(), st));
    NFS_HIP(hipMemcpyAsync(ev_col.data(), w.st_eval, sizeof(double) * ev_col.size(), hipMemcpyDeviceToHost, st));
    for (int b = 0; b < B; ++b) {
      const long ox = w.X.off[b], oy = w.Y.off[b];
      ReadoutArgs ra{w.X.w0s + ox, w.X.w1s + ox, w.X.off[b + 1] - ox, int(logd), w.partials,
                     w.st_rdx + 4 * b};
      NFS_HIP(launch_readout(ra, st));
      ReadoutArgs rb{w.Y.w0s + oy, w.Y.w1s + oy, w.Y.off[b + 1] - oy, int(logd), w.partials,
                     w.st_rdy + 4 * b};
      NFS_HIP(launch_readout(rb, st));
    }
    const bool primal = (p.flags & NFS_FLAG_PRIMAL_COST) && !logd && !centred;
    if (primal) {
      NFS_HIP(spread(w, w.Y, w.Y.w1s, w.wmul_y, 1.0, st));
      NFS_HIP(fft_chain(w, w.dtab2, -1, st));
      if (w.r == 1) NFS_HIP(near_field(w, w.Y, w.X, w.Y.w1s, w.wmul_y, 1.0, st, nullptr, true));
      InterpArgs<R> ia = interp_args(w, w.X, EPI_OUT, w.wmul_y);
      if (w.r == 1) ia.nf = w.nf;
      ia.out = w.tmp;
      ia.scale_vec = w.X.w1s;
      NFS_HIP(launch_interp(ia, w.X.nchunks, st));
      for (int b = 0; b < B; ++b) {
        const long ox = w.X.off[b];
        ReadoutArgs rc{w.tmp + ox, w.tmp + ox, w.X.off[b + 1] - ox, 0, w.partials,
                       w.st_cost + 4 * b};
        NFS_HIP(launch_readout(rc, st));
      }
    }
    if (centred) {
      // back to the caller's variables: alpha = alpha' exp((-2 delta.x' + |delta|^2/2)/eps),
      // alpha_t = alpha_t' exp((2 delta.y' + |delta|^2/2)/eps), delta = 2 shift
      if (alpha) NFS_HIP(map_centred(w.X, 0, alpha, st));
      if (alpha_t) NFS_HIP(map_centred(w.Y, 1, alpha_t, st));
    } else {
      if (alpha) NFS_HIP(launch_unpermute(w.X.w1s, w.X.perm, w.X.n, alpha, st));
      if (alpha_t) NFS_HIP(launch_unpermute(w.Y.w1s, w.Y.perm, w.Y.n, alpha_t, st));
    }
    std::vector<double> col(size_t(B) * kStat), row(size_t(B) * kStat), rdx(size_t(B) * 4), rdy(size_t(B) * 4),
        cost(size_t(B) * 4);
    std::vector<int> pst(size_t(B) * kPState);
    NFS_HIP(hipMemcpyAsync(pst.data(), w.pstate, sizeof(int) * pst.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(col.data(), w.st_col, sizeof(double) * col.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(row.data(), w.st_row, sizeof(double) * row.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(rdx.data(), w.st_rdx, sizeof(double) * rdx.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(rdy.data(), w.st_rdy, sizeof(double) * rdy.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipMemcpyAsync(cost.data(), w.st_cost, sizeof(double) * cost.size(), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipStreamSynchronize(st));
    NFS_TRY(leave(caller));
    int64_t nonpos = 0;
    for (int b = 0; b < B; ++b) {
      const double e = eps[b];
      nfs_result r{};
      r.iters = pst[size_t(kPState) * b + 1];
      r.precision_used = p.precision;
      r.scale = w.sc[b].scale;
      r.kernel_err = w.sc[b].kernel_err;
      // s = eps (1 + sum p log a + sum pt log at - sum_j at_j tt_j), tt the last K^T alpha;
      // log domain (Algorithm 4 result): s = sum p beta + sum pt gamma - eps sum_j at_j tt_j
      const double* cb = col.data() + size_t(kStat) * b;
      const double* rb = row.data() + size_t(kStat) * b;
      const double mass = r.iters > 0 ? cb[1] : ev_row[size_t(kStat) * b + 1];
      r.cost = logd ? rdx[4 * b + 0] + rdy[4 * b + 0] - e * mass : e * (1.0 + rdx[4 * b + 0] + rdy[4 * b + 0] - mass);
      if (centred) {
        // the shifted problem's cost plus |mean y - mean x|^2 (the separable part of the
        // squared cost the shift removed; the coupling is the same)
        double d2 = 0.0;
        for (int c = 0; c < p.d; ++c) d2 += 4.0 * w.sc[b].shift[c] * w.sc[b].shift[c];
        r.cost += d2;
      }
      r.cost_upper = r.cost - e * (rdx[4 * b + 1] + rdy[4 * b + 1]);
      r.cost_primal = primal ? cost[4 * b + 2] : NAN;
      r.marg_err_row = std::sqrt(ev_row[size_t(kStat) * b + 0]);
      r.marg_err_col = std::sqrt(ev_col[size_t(kStat) * b + 0]);
      r.marg_err = r.marg_err_row + r.marg_err_col;
      r.n_nonpos = int64_t(rb[4] + cb[4]);
      r.dyn_range = logd ? NAN : std::max(rb[8], cb[8]);
      r.centred = centred ? 1 : 0;
      nonpos += r.n_nonpos;
      if (res) res[b] = r;
    }
    if (nonpos > 0)
      return fail(NFS_ENONPOS, "fast summation produced kernel sums t <= 0 (normwise error above the dynamic range)");
    return NFS_OK;
  }
};

static int make_solver(const nfs_params* prm, int B, const int64_t* n, const int64_t* nt, const double* eps,
                       const double* x, const double* mu, const double* y, const double* nu, const double* alpha_t0,
                       void* ws, size_t wsb, hipStream_t st, SolverBase** out) {
  *out = nullptr;
  if (prm->precision == NFS_FP32) {
    auto* s = new Solver<float>();
    int rc = s->create(prm, B, n, nt, eps, x, mu, y, nu, alpha_t0, ws, wsb, st);
    if (rc != NFS_OK) {
      delete s;
      return rc;
    }
    *out = s;
  } else {
    auto* s = new Solver<double>();
    int rc = s->create(prm, B, n, nt, eps, x, mu, y, nu, alpha_t0, ws, wsb, st);
    if (rc != NFS_OK) {
      delete s;
      return rc;
    }
    *out = s;
  }
  return NFS_OK;
}

// max_iter iterations, or, with tol > 0, until every problem has stopped:
// each alpha update evaluates ||E|| of the state the previous iteration left
// (eq. (Error), fused into its epilogue), and a problem whose ||E|| <= tol
// completes that iteration and then stops (its kernels skip it).  The host
// polls the stop state every 10 iterations; replays after the last problem
// stopped only launch kernels that return at once.
static int run_solver(SolverBase* s, int32_t max_iter, double tol, double* alpha, double* alpha_t, nfs_result* res,
                      hipStream_t caller) {
  int rc = NFS_OK;
  int done = 0;
  const int check_every = 10;
  if (tol > 0.0) rc = s->set_tol(tol, caller);
  while (rc == NFS_OK && done < max_iter) {
    const int k = tol > 0.0 ? std::min(check_every, max_iter - done) : max_iter - done;
    rc = s->iterate(k, caller);
    done += k;
    if (rc == NFS_OK && tol > 0.0) {
      bool all = false;
      rc = s->all_stopped(&all, caller);
      if (rc == NFS_OK && all) break;
    }
  }
  if (rc == NFS_OK) rc = s->finish(alpha, alpha_t, res, caller);
  return rc;
}

template <typename R>
static int do_grad(const nfs_params* p, const double* x, int64_t n, const double* mu, const double* y, int64_t nt,
                   const double* nu, const double* alpha, const double* alpha_t, double* grad_x, double* grad_mu,
                   void* ws, size_t wsb, hipStream_t st) {
  Work<R> w;
  carve(w, p, 1, n, nt, nullptr, 2);
  if (wsb < w.bytes) return fail(NFS_EWORKSPACE, "workspace too small");
  carve(w, p, 1, n, nt, static_cast<char*>(ws), 2);
  w.X.off = {0, n};
  w.Y.off = {0, nt};
  const double eps = p->eps;
  // the gradient takes the scalings in the caller's variables: no centred mapping
  nfs_params q = *p;
  q.flags &= ~NFS_FLAG_CENTER;
  NFS_TRY(plan_sinkhorn(w, &q, &eps, x, mu, y, nu, alpha, alpha_t, st));
  if (grad_mu) NFS_HIP(launch_gradmu(alpha, n, p->eps, w.partials, w.st_cost, grad_mu, st));
  if (grad_x) {
    double box[kBoxVals];
    NFS_TRY(box_launch(w.st_box, w.partials, p->d, nullptr, 0, nullptr, 0, alpha_t, nt, st));
    NFS_HIP(hipMemcpyAsync(box, w.st_box, sizeof(box), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipStreamSynchronize(st));
    if (!(box[6] > 0.0) || !std::isfinite(box[6])) return fail(NFS_EINVAL, "alpha_t must be positive and finite");
    const double wmax = box[6];
    // alpha_t is spread once; each derivative axis applies (2 pi i k_c) b_k / Phi^2
    // to its transform and interpolates at x (the last pass clears the grid).
    NFS_HIP(spread(w, w.Y, w.Y.w1s, nullptr, 1.0 / wmax, st));
    // r = 1: the gradient of the near-field correction K - K_R, added to each axis
    if (w.r == 1) NFS_HIP(near_field_grad(w, w.Y, w.X, w.Y.w1s, nullptr, 1.0 / wmax, w.tmp, st));
    for (int c = 0; c < p->d; ++c) {
      NFS_HIP(fft_chain(w, w.dtab, c, st, c + 1 < p->d));
      InterpArgs<R> ia = interp_args(w, w.X, EPI_OUT, nullptr);
      if (w.r == 1) ia.nf = w.tmp + size_t(c) * w.X.n;
      // grad_x_i = -eps alpha_i s (dK'/dx'_c * alpha_t)(x'_i), x' = s (x - center)
      ia.norm = -p->eps * w.sc[0].scale * wmax;
      ia.scale_vec = w.X.w1s;
      ia.out = grad_x;
      ia.out_stride = p->d;
      ia.out_comp = c;
      NFS_HIP(launch_interp(ia, w.X.nchunks, st));
    }
  }
  NFS_HIP(hipStreamSynchronize(st));
  return NFS_OK;
}

// Workspace for a batch: the sum over problems of the points, B grids.
static int batch_sizes(const nfs_params* prm, int32_t B, const int64_t* n, const int64_t* nt, long* sn, long* snt) {
  if (B < 1) return fail(NFS_EINVAL, "batch needs at least one problem");
  if (!n || !nt) return fail(NFS_EINVAL, "NULL size array");
  long a = 0, b = 0;
  for (int i = 0; i < B; ++i) {
    if (n[i] < 1 || nt[i] < 1) return fail(NFS_EINVAL, "every problem needs at least one point per cloud");
    a += n[i];
    b += nt[i];
  }
  NFS_TRY(check_params(prm, a, b));
  *sn = a;
  *snt = b;
  return NFS_OK;
}

static int batch_workspace(const nfs_params* prm, int32_t B, long sn, long snt, size_t* bytes) {
  // a solver that tunes its tile plans once per candidate in the same workspace
  std::vector<int> tiles = tile_candidates(prm);
  if (tiles.empty()) tiles.push_back(prm->tile);
  nfs_params q = *prm;
  *bytes = 0;
  for (int T : tiles) {
    q.tile = T;
    if (prm->precision == NFS_FP32) {
      Work<float> w;
      carve(w, &q, B, sn, snt, nullptr, 2);
      *bytes = std::max(*bytes, w.bytes);
    } else {
      Work<double> w;
      carve(w, &q, B, sn, snt, nullptr, 2);
      *bytes = std::max(*bytes, w.bytes);
    }
  }
  return NFS_OK;
}

// ----------------------------------------------------------------------------- NFS_AUTO
static nfs_params with_precision(const nfs_params* p, int precision) {
  nfs_params q = *p;
  q.precision = precision;
  return q;
}

static size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Single problem: [0, S) solver workspace (S = the larger of the FP32 and FP64
// needs), then nt doubles keeping the caller's starting alpha_t.
static int auto_workspace(const nfs_params* p, int64_t n, int64_t nt, size_t* S, size_t* total) {
  const nfs_params p32 = with_precision(p, NFS_FP32), p64 = with_precision(p, NFS_FP64);
  NFS_TRY(check_params(&p32, n, nt));
  NFS_TRY(check_params(&p64, n, nt));
  size_t b32 = 0, b64 = 0;
  NFS_TRY(batch_workspace(&p32, 1, n, nt, &b32));
  NFS_TRY(batch_workspace(&p64, 1, n, nt, &b64));
  *S = align_up(std::max(b32, b64));
  *total = *S + sizeof(double) * size_t(nt);
  return NFS_OK;
}

// A problem is solved again with FP64 grids when its FP32 solve met a sum
// t <= 0, or sums below 1/kAutoRange of the l1 norm of their source weights
// (nfs_result.dyn_range): fast summation's error is normwise in that norm, so
// at FP32 rounding such sums keep few correct digits.
constexpr double kAutoRange = 1e5;

static bool needs_fp64(const nfs_result& r) { return r.n_nonpos > 0 || !(r.dyn_range <= kAutoRange); }

// With FP64 grids the sums' error is about 1e-16 of the l1 norm of their
// weights, so the FP64 tolerance 1e-10 holds for sums down to 1e-6 of it;
// beyond that (or at t <= 0) the problem is solved once more in the centred
// form (NFS_FLAG_CENTER), whose iterates are the same but whose sums span far
// less range when the clouds are apart.
constexpr double kAutoRange64 = 1e6;

static bool needs_centring(const nfs_result& r, bool logd) {
  return r.n_nonpos > 0 || (!logd && !(r.dyn_range <= kAutoRange64));
}

// Packed inputs and results of the problems re-solved in FP64: x, y, mu, nu,
// alpha, alpha_t of every problem at most.
static size_t auto_packed_bytes(int d, long sn, long snt) {
  return align_up(sizeof(double) * (size_t(sn + snt) * (d + 2)));
}

// Batch: the FP32 batch, or the packed copies plus the FP64 batch of every
// problem (the most that can be promoted), whichever needs more.
static int auto_batch_workspace(const nfs_params* p, int32_t B, const int64_t* n, const int64_t* nt, size_t* bytes) {
  const nfs_params p32 = with_precision(p, NFS_FP32), p64 = with_precision(p, NFS_FP64);
  long sn = 0, snt = 0;
  NFS_TRY(batch_sizes(&p32, B, n, nt, &sn, &snt));
  NFS_TRY(batch_sizes(&p64, B, n, nt, &sn, &snt));
  size_t b32 = 0, b64 = 0;
  NFS_TRY(batch_workspace(&p32, B, sn, snt, &b32));
  NFS_TRY(batch_workspace(&p64, B, sn, snt, &b64));
  *bytes = std::max(b32, auto_packed_bytes(p->d, sn, snt) + b64);
  return NFS_OK;
}

// ----------------------------------------------------------------------------- Sinkhorn divergence
// Workspace: packed inputs of the three problems (P, Pt), (P, P), (Pt, Pt) and
// their scalings, then the batch workspace.
struct DivLayout {
  int64_t n3[3], nt3[3];
  size_t packed = 0;  // bytes before the batch workspace
  size_t batch = 0;
};

static int divergence_layout(const nfs_params* p, int64_t n, int64_t nt, DivLayout* L) {
  if (!p) return fail(NFS_EINVAL, "params is NULL");
  if (n < 1 || nt < 1) return fail(NFS_EINVAL, "every cloud needs at least one point");
  L->n3[0] = n, L->n3[1] = n, L->n3[2] = nt;
  L->nt3[0] = nt, L->nt3[1] = n, L->nt3[2] = nt;
  if (p->precision == NFS_AUTO) {
    NFS_TRY(auto_batch_workspace(p, 3, L->n3, L->nt3, &L->batch));
  } else {
    long sn = 0, snt = 0;
    NFS_TRY(batch_sizes(p, 3, L->n3, L->nt3, &sn, &snt));
    NFS_TRY(batch_workspace(p, 3, sn, snt, &L->batch));
  }
  const size_t nx = size_t(2 * n + nt), ny = size_t(n + 2 * nt);
  L->packed = align_up(sizeof(double) * ((nx + ny) * size_t(p->d) + 2 * (nx + ny)));
  return NFS_OK;
}

}  // namespace nfs

// ============================================================================= C ABI
using namespace nfs;

extern "C" {

const char* nfs_last_error(void) { return g_err.c_str(); }

int nfs_validate(const nfs_params* prm, int64_t n, int64_t nt) {
  g_err.clear();
  return check_params(prm, n, nt);
}

int nfs_workspace_size(const nfs_params* prm, int64_t n, int64_t nt, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(NFS_EINVAL, "bytes is NULL");
  if (prm && prm->precision == NFS_AUTO) {
    size_t S = 0;
    return auto_workspace(prm, n, nt, &S, bytes);
  }
  NFS_TRY(check_params(prm, n, nt));
  return batch_workspace(prm, 1, n, nt, bytes);
}

int nfs_fastsum_apply(const nfs_params* prm, const double* src, int64_t ns, const double* w, const double* tgt,
                      int64_t nt, double* out, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  NFS_TRY(check_params(prm, ns, nt));
  if (!src || !w || !tgt || !out || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (prm->precision == NFS_FP32) return do_fastsum<float>(prm, src, ns, w, tgt, nt, out, workspace, ws_bytes, st);
  return do_fastsum<double>(prm, src, ns, w, tgt, nt, out, workspace, ws_bytes, st);
}

int nfs_fastsum_apply_noalloc(const nfs_params* prm, const double* src, int64_t ns, const double* w,
                              const double* tgt, int64_t nt, double* out, void* stream) {
  g_err.clear();
  NFS_TRY(check_params(prm, ns, nt));
  if (!src || !w || !tgt || !out) return fail(NFS_EINVAL, "NULL pointer argument");
  const size_t need = prm->precision == NFS_FP32 ? fastsum_bytes<float>(prm, ns, nt) : fastsum_bytes<double>(prm, ns, nt);
  if (need > kScratchBytes)
    return fail(NFS_EWORKSPACE, "problem needs " + std::to_string(need) + " bytes of scratch, above the " +
                                    std::to_string(kScratchBytes) +
                                    "-byte static scratch of nfs_fastsum_apply_noalloc; use nfs_fastsum_apply");
  void* ws = nullptr;
  NFS_TRY(scratch_address(&ws));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (prm->precision == NFS_FP32) return do_fastsum<float>(prm, src, ns, w, tgt, nt, out, ws, kScratchBytes, st);
  return do_fastsum<double>(prm, src, ns, w, tgt, nt, out, ws, kScratchBytes, st);
}

int nfs_plan_apply(const nfs_params* prm, const double* x, int64_t n, const double* y, int64_t nt,
                   const double* alpha, const double* alpha_t, const double* v, int32_t transpose, double* out,
                   void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  NFS_TRY(check_params(prm, n, nt));
  if (!x || !y || !alpha || !alpha_t || !v || !out || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  if (transpose != 0 && transpose != 1) return fail(NFS_EINVAL, "transpose must be 0 or 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // pi v = alpha o K (alpha_t o v): sources y, targets x; pi^T v with the roles swapped
  const double* src = transpose ? x : y;
  const double* tgt = transpose ? y : x;
  const int64_t ns = transpose ? n : nt, ntg = transpose ? nt : n;
  const double* ws_ = transpose ? alpha : alpha_t;
  const double* wt_ = transpose ? alpha_t : alpha;
  if (prm->precision == NFS_FP32)
    return do_fastsum<float>(prm, src, ns, ws_, tgt, ntg, out, workspace, ws_bytes, st, v, wt_);
  return do_fastsum<double>(prm, src, ns, ws_, tgt, ntg, out, workspace, ws_bytes, st, v, wt_);
}

int nfs_nfft_adjoint(const nfs_params* prm, const double* pts, int64_t n, const double* w, double* fhat,
                     void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  NFS_TRY(check_params(prm, n, 1));
  if (!pts || !w || !fhat || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (prm->precision == NFS_FP32)
    return do_nfft<float>(prm, true, pts, n, w, nullptr, fhat, nullptr, workspace, ws_bytes, st);
  return do_nfft<double>(prm, true, pts, n, w, nullptr, fhat, nullptr, workspace, ws_bytes, st);
}

int nfs_nfft_trafo(const nfs_params* prm, const double* fhat, const double* pts, int64_t n, double* out,
                   void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  NFS_TRY(check_params(prm, n, 1));
  if (!pts || !fhat || !out || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (prm->precision == NFS_FP32)
    return do_nfft<float>(prm, false, pts, n, nullptr, fhat, nullptr, out, workspace, ws_bytes, st);
  return do_nfft<double>(prm, false, pts, n, nullptr, fhat, nullptr, out, workspace, ws_bytes, st);
}

int nfs_sinkhorn_solve(const nfs_params* prm, const double* x, int64_t n, const double* mu, const double* y,
                       int64_t nt, const double* nu, int32_t max_iter, double tol, int32_t warm_start, double* alpha,
                       double* alpha_t, nfs_result* res, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (prm && prm->precision == NFS_AUTO) {
    size_t S = 0, total = 0;
    NFS_TRY(auto_workspace(prm, n, nt, &S, &total));
    if (!x || !mu || !y || !nu || !alpha || !alpha_t || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
    if (ws_bytes < total) return fail(NFS_EWORKSPACE, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* start = reinterpret_cast<double*>(static_cast<char*>(workspace) + S);
    if (warm_start) NFS_HIP(hipMemcpyAsync(start, alpha_t, sizeof(double) * nt, hipMemcpyDeviceToDevice, st));
    const nfs_params p32 = with_precision(prm, NFS_FP32), p64 = with_precision(prm, NFS_FP64);
    nfs_result r{};
    int rc = nfs_sinkhorn_solve(&p32, x, n, mu, y, nt, nu, max_iter, tol, warm_start, alpha, alpha_t, &r, workspace,
                                S, stream);
    const bool logd = (prm->flags & NFS_FLAG_LOG_DOMAIN) != 0;
    if (rc == NFS_ENONPOS || (rc == NFS_OK && !logd && needs_fp64(r))) {
      // again from the caller's starting value, with FP64 grids
      if (warm_start) NFS_HIP(hipMemcpyAsync(alpha_t, start, sizeof(double) * nt, hipMemcpyDeviceToDevice, st));
      rc = nfs_sinkhorn_solve(&p64, x, n, mu, y, nt, nu, max_iter, tol, warm_start, alpha, alpha_t, &r, workspace,
                              S, stream);
    }
    if ((rc == NFS_ENONPOS || (rc == NFS_OK && r.precision_used == NFS_FP64 && needs_centring(r, logd))) &&
        prm->r == 2 && !(prm->flags & NFS_FLAG_CENTER)) {
      // beyond FP64's range too: the centred form (NFS_FLAG_CENTER) with FP64 grids, same start
      nfs_params pc = p64;
      pc.flags |= NFS_FLAG_CENTER;
      if (warm_start) NFS_HIP(hipMemcpyAsync(alpha_t, start, sizeof(double) * nt, hipMemcpyDeviceToDevice, st));
      rc = nfs_sinkhorn_solve(&pc, x, n, mu, y, nt, nu, max_iter, tol, warm_start, alpha, alpha_t, &r, workspace, S,
                              stream);
    }
    if (res) *res = r;
    return rc;
  }
  NFS_TRY(check_params(prm, n, nt));
  if (!x || !mu || !y || !nu || !alpha || !alpha_t || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  if (max_iter < 0) return fail(NFS_EINVAL, "max_iter must be >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SolverBase* s = nullptr;
  NFS_TRY(make_solver(prm, 1, &n, &nt, &prm->eps, x, mu, y, nu, warm_start ? alpha_t : nullptr, workspace, ws_bytes,
                      st, &s));
  const int rc = run_solver(s, max_iter, tol, alpha, alpha_t, res, st);
  delete s;
  return rc;
}

int nfs_sinkhorn_solve_log(const nfs_params* prm, const double* x, int64_t n, const double* mu, const double* y,
                           int64_t nt, const double* nu, int32_t max_iter, double tol, int32_t warm_start,
                           double* beta, double* gamma, nfs_result* res, void* workspace, size_t ws_bytes,
                           void* stream) {
  g_err.clear();
  if (!prm) return fail(NFS_EINVAL, "params is NULL");
  nfs_params q = *prm;
  q.flags |= NFS_FLAG_LOG_DOMAIN;
  return nfs_sinkhorn_solve(&q, x, n, mu, y, nt, nu, max_iter, tol, warm_start, beta, gamma, res, workspace,
                            ws_bytes, stream);
}

int nfs_solver_create(const nfs_params* prm, const double* x, int64_t n, const double* mu, const double* y,
                      int64_t nt, const double* nu, const double* alpha_t0, void* workspace, size_t ws_bytes,
                      void* stream, nfs_solver** out) {
  g_err.clear();
  if (!out) return fail(NFS_EINVAL, "out is NULL");
  *out = nullptr;
  NFS_TRY(check_params(prm, n, nt));
  if (!x || !mu || !y || !nu || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  SolverBase* s = nullptr;
  NFS_TRY(make_solver(prm, 1, &n, &nt, &prm->eps, x, mu, y, nu, alpha_t0, workspace, ws_bytes,
                      static_cast<hipStream_t>(stream), &s));
  *out = reinterpret_cast<nfs_solver*>(s);
  return NFS_OK;
}

int nfs_solver_iterate(nfs_solver* s, int32_t iters, void* stream) {
  g_err.clear();
  if (!s) return fail(NFS_EINVAL, "solver is NULL");
  if (iters < 0) return fail(NFS_EINVAL, "iters must be >= 0");
  return reinterpret_cast<SolverBase*>(s)->iterate(iters, static_cast<hipStream_t>(stream));
}

int nfs_solver_residual(nfs_solver* s, double* err_row, void* stream) {
  g_err.clear();
  if (!s || !err_row) return fail(NFS_EINVAL, "NULL argument");
  return reinterpret_cast<SolverBase*>(s)->residual(err_row, static_cast<hipStream_t>(stream));
}

int nfs_solver_finish(nfs_solver* s, double* alpha, double* alpha_t, nfs_result* res, void* stream) {
  g_err.clear();
  if (!s) return fail(NFS_EINVAL, "solver is NULL");
  return reinterpret_cast<SolverBase*>(s)->finish(alpha, alpha_t, res, static_cast<hipStream_t>(stream));
}

int nfs_solver_profile(nfs_solver* s, int32_t iters, double* stage_ms, double* info, void* stream) {
  g_err.clear();
  if (!s || !stage_ms) return fail(NFS_EINVAL, "NULL argument");
  auto* b = reinterpret_cast<SolverBase*>(s);
  if (info) b->stage_info(info);
  return b->profile(iters, stage_ms, static_cast<hipStream_t>(stream));
}

int nfs_solver_grad(nfs_solver* s, double* grad_x, double* grad_mu, double* grad_y, double* grad_nu, void* stream) {
  g_err.clear();
  if (!s) return fail(NFS_EINVAL, "solver is NULL");
  return reinterpret_cast<SolverBase*>(s)->grad(grad_x, grad_mu, grad_y, grad_nu, static_cast<hipStream_t>(stream));
}

int nfs_solver_destroy(nfs_solver* s) {
  delete reinterpret_cast<SolverBase*>(s);
  return NFS_OK;
}

int nfs_batch_workspace_size(const nfs_params* prm, int32_t nprob, const int64_t* n, const int64_t* nt,
                             size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(NFS_EINVAL, "bytes is NULL");
  if (prm && prm->precision == NFS_AUTO) return auto_batch_workspace(prm, nprob, n, nt, bytes);
  long sn = 0, snt = 0;
  NFS_TRY(batch_sizes(prm, nprob, n, nt, &sn, &snt));
  return batch_workspace(prm, nprob, sn, snt, bytes);
}

int nfs_batch_solver_create(const nfs_params* prm, int32_t nprob, const int64_t* n, const int64_t* nt,
                            const double* eps, const double* x, const double* mu, const double* y, const double* nu,
                            const double* alpha_t0, void* workspace, size_t ws_bytes, void* stream, nfs_solver** out) {
  g_err.clear();
  if (!out) return fail(NFS_EINVAL, "out is NULL");
  *out = nullptr;
  long sn = 0, snt = 0;
  NFS_TRY(batch_sizes(prm, nprob, n, nt, &sn, &snt));
  if (!eps) return fail(NFS_EINVAL, "eps is NULL");
  for (int b = 0; b < nprob; ++b)
    if (!(eps[b] > 0.0) || !std::isfinite(eps[b])) return fail(NFS_EINVAL, "every eps must be positive and finite");
  if (!x || !mu || !y || !nu || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  SolverBase* s = nullptr;
  NFS_TRY(make_solver(prm, nprob, n, nt, eps, x, mu, y, nu, alpha_t0, workspace, ws_bytes,
                      static_cast<hipStream_t>(stream), &s));
  *out = reinterpret_cast<nfs_solver*>(s);
  return NFS_OK;
}

int nfs_batch_solve(const nfs_params* prm, int32_t nprob, const int64_t* n, const int64_t* nt, const double* eps,
                    const double* x, const double* mu, const double* y, const double* nu, int32_t max_iter,
                    double tol, double* alpha, double* alpha_t, nfs_result* res, void* workspace, size_t ws_bytes,
                    void* stream) {
  g_err.clear();
  if (max_iter < 0) return fail(NFS_EINVAL, "max_iter must be >= 0");
  if (!alpha || !alpha_t) return fail(NFS_EINVAL, "NULL pointer argument");
  if (prm && prm->precision == NFS_AUTO) {
    size_t need = 0;
    NFS_TRY(auto_batch_workspace(prm, nprob, n, nt, &need));
    if (!eps || !x || !mu || !y || !nu || !res || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
    if (ws_bytes < need) return fail(NFS_EWORKSPACE, "workspace too small");
    const nfs_params p32 = with_precision(prm, NFS_FP32), p64 = with_precision(prm, NFS_FP64);
    int rc = nfs_batch_solve(&p32, nprob, n, nt, eps, x, mu, y, nu, max_iter, tol, alpha, alpha_t, res, workspace,
                             ws_bytes, stream);
    if (rc != NFS_OK && rc != NFS_ENONPOS) return rc;
    const bool logd = (prm->flags & NFS_FLAG_LOG_DOMAIN) != 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int d = prm->d;
    std::vector<int64_t> ox(nprob + 1, 0), oy(nprob + 1, 0);
    for (int b = 0; b < nprob; ++b) {
      ox[b + 1] = ox[b] + n[b];
      oy[b + 1] = oy[b] + nt[b];
    }
    long sn_all = 0, snt_all = 0;
    NFS_TRY(batch_sizes(&p64, nprob, n, nt, &sn_all, &snt_all));
    const size_t packed = auto_packed_bytes(d, sn_all, snt_all);
    // Solve the problems `sel` again with parameters q, as one batch of their
    // own: inputs packed at the start of the workspace (x | y | mu | nu |
    // alpha | alpha_t), the batch workspace after them; results copied back.
    auto resolve = [&](const std::vector<int>& sel, const nfs_params& q) -> int {
      std::vector<int64_t> n2, nt2;
      std::vector<double> eps2;
      long sn = 0, snt = 0;
      for (int b : sel) {
        n2.push_back(n[b]);
        nt2.push_back(nt[b]);
        eps2.push_back(eps[b]);
        sn += n[b];
        snt += nt[b];
      }
      double* X2 = static_cast<double*>(workspace);
      double* Y2 = X2 + size_t(sn) * d;
      double* MU2 = Y2 + size_t(snt) * d;
      double* NU2 = MU2 + sn;
      double* A2 = NU2 + snt;
      double* AT2 = A2 + sn;
      long px = 0, py = 0;
      for (int b : sel) {
        NFS_HIP(hipMemcpyAsync(X2 + px * d, x + ox[b] * d, sizeof(double) * n[b] * d, hipMemcpyDeviceToDevice, st));
        NFS_HIP(hipMemcpyAsync(MU2 + px, mu + ox[b], sizeof(double) * n[b], hipMemcpyDeviceToDevice, st));
        NFS_HIP(hipMemcpyAsync(Y2 + py * d, y + oy[b] * d, sizeof(double) * nt[b] * d, hipMemcpyDeviceToDevice, st));
        NFS_HIP(hipMemcpyAsync(NU2 + py, nu + oy[b], sizeof(double) * nt[b], hipMemcpyDeviceToDevice, st));
        px += n[b];
        py += nt[b];
      }
      std::vector<nfs_result> r2(sel.size());
      nfs_params qq = q;
      const int rc2 = nfs_batch_solve(&qq, int32_t(sel.size()), n2.data(), nt2.data(), eps2.data(), X2, MU2, Y2, NU2,
                                      max_iter, tol, A2, AT2, r2.data(), static_cast<char*>(workspace) + packed,
                                      ws_bytes - packed, stream);
      if (rc2 != NFS_OK && rc2 != NFS_ENONPOS) return rc2;
      px = py = 0;
      for (size_t k = 0; k < sel.size(); ++k) {
        const int b = sel[k];
        NFS_HIP(hipMemcpyAsync(alpha + ox[b], A2 + px, sizeof(double) * n[b], hipMemcpyDeviceToDevice, st));
        NFS_HIP(hipMemcpyAsync(alpha_t + oy[b], AT2 + py, sizeof(double) * nt[b], hipMemcpyDeviceToDevice, st));
        px += n[b];
        py += nt[b];
        res[b] = r2[k];
      }
      NFS_HIP(hipStreamSynchronize(st));
      return NFS_OK;
    };
    // FP64 grids for the problems FP32 cannot resolve, from the same start
    std::vector<int> sel;
    for (int b = 0; b < nprob; ++b)
      if (res[b].n_nonpos > 0 || (!logd && needs_fp64(res[b]))) sel.push_back(b);
    if (sel.empty()) return rc;
    NFS_TRY(resolve(sel, p64));
    // beyond FP64's range too: the centred form (NFS_FLAG_CENTER) with FP64 grids
    std::vector<int> sel3;
    for (int b : sel)
      if (needs_centring(res[b], logd)) sel3.push_back(b);
    if (!sel3.empty() && prm->r == 2 && !(prm->flags & NFS_FLAG_CENTER)) {
      nfs_params pc = p64;
      pc.flags |= NFS_FLAG_CENTER;
      NFS_TRY(resolve(sel3, pc));
    }
    rc = NFS_OK;
    for (int b = 0; b < nprob; ++b)
      if (res[b].n_nonpos > 0) rc = NFS_ENONPOS;
    if (rc != NFS_OK) return fail(rc, "FP64 grids (and the centred form) also produced kernel sums t <= 0");
    g_err.clear();
    return NFS_OK;
  }
  nfs_solver* h = nullptr;
  NFS_TRY(nfs_batch_solver_create(prm, nprob, n, nt, eps, x, mu, y, nu, nullptr, workspace, ws_bytes, stream, &h));
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto* s = reinterpret_cast<SolverBase*>(h);
  const int rc = run_solver(s, max_iter, tol, alpha, alpha_t, res, st);
  delete s;
  return rc;
}

int nfs_divergence_workspace_size(const nfs_params* prm, int64_t n, int64_t nt, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(NFS_EINVAL, "bytes is NULL");
  DivLayout L;
  NFS_TRY(divergence_layout(prm, n, nt, &L));
  *bytes = L.packed + L.batch;
  return NFS_OK;
}

int nfs_sinkhorn_divergence(const nfs_params* prm, const double* x, int64_t n, const double* mu, const double* y,
                            int64_t nt, const double* nu, int32_t max_iter, double tol, double* sd, nfs_result* res,
                            void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  DivLayout L;
  NFS_TRY(divergence_layout(prm, n, nt, &L));
  if (!x || !mu || !y || !nu || !sd || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  if (ws_bytes < L.packed + L.batch) return fail(NFS_EWORKSPACE, "workspace too small");
  if (max_iter < 0) return fail(NFS_EINVAL, "max_iter must be >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int d = prm->d;
  const size_t nx = size_t(2 * n + nt), ny = size_t(n + 2 * nt);
  double* X = static_cast<double*>(workspace);
  double* Y = X + nx * d;
  double* MU = Y + ny * d;
  double* NU = MU + nx;
  double* A = NU + ny;
  double* AT = A + nx;
  const size_t bx = sizeof(double) * size_t(n) * d, by = sizeof(double) * size_t(nt) * d;
  // x rows: x | x | y ; y rows: y | x | y (problems (P, Pt), (P, P), (Pt, Pt))
  NFS_HIP(hipMemcpyAsync(X, x, bx, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(X + size_t(n) * d, x, bx, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(X + size_t(2 * n) * d, y, by, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(Y, y, by, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(Y + size_t(nt) * d, x, bx, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(Y + size_t(nt + n) * d, y, by, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(MU, mu, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(MU + n, mu, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(MU + 2 * n, nu, sizeof(double) * nt, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(NU, nu, sizeof(double) * nt, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(NU + nt, mu, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  NFS_HIP(hipMemcpyAsync(NU + nt + n, nu, sizeof(double) * nt, hipMemcpyDeviceToDevice, st));
  const double eps3[3] = {prm->eps, prm->eps, prm->eps};
  nfs_result r3[3] = {};
  const int rc = nfs_batch_solve(prm, 3, L.n3, L.nt3, eps3, X, MU, Y, NU, max_iter, tol, A, AT, r3,
                                 static_cast<char*>(workspace) + L.packed, ws_bytes - L.packed, stream);
  if (rc != NFS_OK && rc != NFS_ENONPOS) return rc;
  *sd = r3[0].cost - 0.5 * r3[1].cost - 0.5 * r3[2].cost;
  if (res)
    for (int k = 0; k < 3; ++k) res[k] = r3[k];
  return rc;
}

int nfs_sinkhorn_grad(const nfs_params* prm, const double* x, int64_t n, const double* mu, const double* y,
                      int64_t nt, const double* nu, const double* alpha, const double* alpha_t, double* grad_x,
                      double* grad_mu, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  NFS_TRY(check_params(prm, n, nt));
  if (!x || !mu || !y || !nu || !alpha || !alpha_t || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (prm->precision == NFS_FP32)
    return do_grad<float>(prm, x, n, mu, y, nt, nu, alpha, alpha_t, grad_x, grad_mu, workspace, ws_bytes, st);
  return do_grad<double>(prm, x, n, mu, y, nt, nu, alpha, alpha_t, grad_x, grad_mu, workspace, ws_bytes, st);
}

int nfs_sinkhorn_grad_targets(const nfs_params* prm, const double* x, int64_t n, const double* mu, const double* y,
                              int64_t nt, const double* nu, const double* alpha, const double* alpha_t,
                              double* grad_y, double* grad_nu, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  NFS_TRY(check_params(prm, n, nt));
  if (!x || !mu || !y || !nu || !alpha || !alpha_t || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the kernel is even: the target-side gradient is the source-side one with the roles swapped
  if (prm->precision == NFS_FP32)
    return do_grad<float>(prm, y, nt, nu, x, n, mu, alpha_t, alpha, grad_y, grad_nu, workspace, ws_bytes, st);
  return do_grad<double>(prm, y, nt, nu, x, n, mu, alpha_t, alpha, grad_y, grad_nu, workspace, ws_bytes, st);
}

}  // extern "C"
