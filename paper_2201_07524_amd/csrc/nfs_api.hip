// C ABI of the NFFT-boosted Sinkhorn library: argument checks, workspace
// layout, the plan stage (torus scaling, binning), the fast-summation chain
// and the Sinkhorn iteration (Algorithm 3) with hipGraph replay.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
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

static int check_params(const nfs_params* p, int64_t n, int64_t nt) {
  if (!p) return fail(NFS_EINVAL, "params is NULL");
  if (p->d < 1 || p->d > 3) return fail(NFS_EINVAL, "d must be 1, 2 or 3");
  if (p->r != 1 && p->r != 2) return fail(NFS_EUNSUPPORTED, "cost exponent r must be 1 or 2");
  if (p->r == 1) return fail(NFS_EUNSUPPORTED, "r = 1 (near-field regularization) is not available in this build");
  if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(NFS_EINVAL, "eps must be positive and finite");
  if (p->N < 4 || (p->N & 1)) return fail(NFS_EINVAL, "N must be even and >= 4");
  if (p->m < 2 || p->m > 8) return fail(NFS_EINVAL, "m must be in [2, 8]");
  if (!(p->sigma >= 1.0) || p->sigma > 16.0) return fail(NFS_EINVAL, "sigma must be in [1, 16]");
  if (p->precision != NFS_FP64 && p->precision != NFS_FP32) return fail(NFS_EINVAL, "precision must be NFS_FP64 or NFS_FP32");
  const int g = grid_size(p);
  if (g > 4096) return fail(NFS_EUNSUPPORTED, "grid size sigma*N above 4096 per dimension");
  if (p->tile < 0 || p->tile > 256) return fail(NFS_EINVAL, "tile must be in [0, 256]");
  if (p->chunk < 0 || p->chunk > (1 << 20)) return fail(NFS_EINVAL, "chunk must be in [0, 2^20]");
  if (n < 1 || nt < 1) return fail(NFS_EINVAL, "point counts must be >= 1");
  if (n > (int64_t(1) << 30) || nt > (int64_t(1) << 30)) return fail(NFS_EUNSUPPORTED, "point counts above 2^30");
  const double gd = std::pow(double(g), p->d);
  if (gd > double(1u << 30)) return fail(NFS_EUNSUPPORTED, "grid with more than 2^30 cells");
  const int T = p->tile ? p->tile : default_tile(p->d, p->precision);
  const int E = T + 2 * p->m + 1;
  const double tb = std::pow(double(E), p->d) * (p->precision == NFS_FP32 ? 4.0 : 8.0);
  if (tb > 160.0 * 1024.0) return fail(NFS_EINVAL, "LDS tile (tile + 2m + 1)^d exceeds 160 KiB; use a smaller tile");
  return NFS_OK;
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

template <typename R>
struct CloudBuf {
  long n = 0;
  R* coords = nullptr;
  int* perm = nullptr;
  int* keys = nullptr;
  int* counts = nullptr;
  int* offsets = nullptr;
  int* cursor = nullptr;
  Chunk* chunks = nullptr;
  int* tile_chunks = nullptr;  // nbins + 1: chunks of tile b are [tile_chunks[b], tile_chunks[b+1])
  long max_chunks = 0;
  int nchunks = 0;
  double* w0s = nullptr;  // sorted first vector (weights)
  double* w1s = nullptr;  // sorted second vector (scalings)
};

template <typename R>
struct Work {
  Geom geo{};
  WindowConst win{};
  int K0 = 0, nbins = 0, chunk = 0;
  long ncell = 0;
  CloudBuf<R> A, B;  // A: x / sources, B: y / targets
  bool two_level = false;  // chunk tiles + per-tile gather instead of global atomics
  R* part = nullptr;       // chunk tiles (two_level)
  long ecell = 0;          // values per chunk tile, E^d
  R* S = nullptr;    // spread grid
  R* U = nullptr;    // interpolation grid
  cplx<R>* W = nullptr;
  cplx<R>* V = nullptr;
  cplx<R>* spec = nullptr;
  cplx<R>* tw = nullptr;
  R* dtab = nullptr;
  R* dtab2 = nullptr;
  double* inv_phi = nullptr;
  double* partials = nullptr;
  unsigned* counters = nullptr;
  double* stats = nullptr;
  double* tmp = nullptr;
  size_t bytes = 0;
};

enum StatSlot : int {
  ST_ROW = 0, ST_COL = 8, ST_EVAL = 16, ST_RD_X = 24, ST_RD_Y = 28, ST_WMUL_X = 32, ST_WMUL_Y = 33,
  ST_BOX = 40, ST_BOX2 = 52, ST_LOGMEAN = 64, ST_MISC = 72, ST_TOTAL = 128
};
enum CounterSlot : int { CT_INTERP = 0, CT_BOX = 1, CT_RD = 2, CT_TOTAL = 16 };

template <typename R>
static void carve(Work<R>& w, const nfs_params* p, long nA, long nB, char* base, int kind_vectors) {
  Carver cv{base};
  const int d = p->d;
  const int g = grid_size(p);
  const int T = p->tile ? p->tile : default_tile(d, p->precision);
  const int chunk = p->chunk ? p->chunk : 1024;
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
  long ncell = 1;
  for (int c = 0; c < d; ++c) ncell *= g;
  w.ncell = ncell;
  auto cloud = [&](CloudBuf<R>& cb, long n, int nvec) {
    cb.n = n;
    cb.coords = cv.take<R>(size_t(n) * d);
    cb.perm = cv.take<int>(n);
    cb.keys = cv.take<int>(n);
    cb.counts = cv.take<int>(nbins);
    cb.offsets = cv.take<int>(nbins);
    cb.cursor = cv.take<int>(nbins);
    cb.max_chunks = n / chunk + std::min<long>(nbins, n) + 1;
    cb.chunks = cv.take<Chunk>(cb.max_chunks);
    cb.tile_chunks = cv.take<int>(nbins + 1);
    cb.w0s = nvec >= 1 ? cv.take<double>(n) : nullptr;
    cb.w1s = nvec >= 2 ? cv.take<double>(n) : nullptr;
  };
  cloud(w.A, nA, kind_vectors);
  cloud(w.B, nB, kind_vectors);
  long ecell = 1;
  for (int c = 0; c < d; ++c) ecell *= w.geo.E;
  w.ecell = ecell;
  long tcells = 1;
  for (int c = 0; c < d; ++c) tcells *= T;
  bool two = (p->flags & NFS_FLAG_TILE_REDUCE) && T >= p->m + 1 && (g % T) == 0 && tcells <= 2048;
  for (int c = 0; c < d; ++c) two = two && w.geo.nt[c] >= 3;
  w.two_level = two;
  w.part = two ? cv.take<R>(size_t(std::max(w.A.max_chunks, w.B.max_chunks)) * ecell) : nullptr;
  w.S = cv.take<R>(ncell);
  w.U = cv.take<R>(ncell);
  const long rows = ncell / g;
  w.W = cv.take<cplx<R>>(size_t(rows) * w.K0);
  w.V = d == 3 ? cv.take<cplx<R>>(size_t(g) * (p->N + 1) * w.K0) : nullptr;
  long spec_n = w.K0;
  for (int c = 0; c < d - 1; ++c) spec_n *= (p->N + 1);
  w.spec = cv.take<cplx<R>>(spec_n);
  w.tw = cv.take<cplx<R>>(g);
  long H = 1;
  for (int c = 0; c < d; ++c) H *= w.K0;
  w.dtab = cv.take<R>(H);
  w.dtab2 = cv.take<R>(H);
  w.inv_phi = cv.take<double>(w.K0);
  const long maxch = std::max(w.A.max_chunks, w.B.max_chunks);
  w.partials = cv.take<double>(size_t(std::max<long>(maxch, 1024)) * 9);
  w.counters = cv.take<unsigned>(CT_TOTAL);
  w.stats = cv.take<double>(ST_TOTAL);
  w.tmp = cv.take<double>(std::max(nA, nB) * std::max(d, 1));
  w.bytes = cv.off + 256;
  w.win = make_window(p->m, g, p->N);
}

// ----------------------------------------------------------------------------- plan stage
template <typename R>
static int sort_cloud(Work<R>& w, CloudBuf<R>& cb, const double* pts, const Scaling& sc, const double* v0,
                      const double* v1, hipStream_t st) {
  const Geom& geo = w.geo;
  NFS_HIP(launch_fill(cb.counts, sizeof(int) * w.nbins, st));
  NFS_HIP(launch_fill(cb.cursor, sizeof(int) * w.nbins, st));
  KeyArgs ka{};
  ka.pts = pts;
  ka.n = cb.n;
  ka.d = geo.d;
  ka.g = geo.g;
  ka.T = geo.T;
  for (int c = 0; c < 3; ++c) {
    ka.nt[c] = geo.nt[c];
    ka.center[c] = sc.center[c];
  }
  ka.scale = sc.scale;
  ka.keys = cb.keys;
  ka.counts = cb.counts;
  NFS_HIP(launch_keys(ka, st));
  std::vector<int> counts(w.nbins), offsets(w.nbins);
  NFS_HIP(hipMemcpyAsync(counts.data(), cb.counts, sizeof(int) * w.nbins, hipMemcpyDeviceToHost, st));
  NFS_HIP(hipStreamSynchronize(st));
  std::vector<Chunk> chunks;
  std::vector<int> tile_chunks(w.nbins + 1);
  chunks.reserve(cb.max_chunks);
  int acc = 0;
  for (int b = 0; b < w.nbins; ++b) {
    offsets[b] = acc;
    tile_chunks[b] = int(chunks.size());
    for (int s = 0; s < counts[b]; s += w.chunk) chunks.push_back(Chunk{b, acc + s, std::min(w.chunk, counts[b] - s), 0});
    acc += counts[b];
  }
  tile_chunks[w.nbins] = int(chunks.size());
  if ((long)chunks.size() > cb.max_chunks) return fail(NFS_EINVAL, "internal: chunk table overflow");
  cb.nchunks = int(chunks.size());
  NFS_HIP(hipMemcpyAsync(cb.offsets, offsets.data(), sizeof(int) * w.nbins, hipMemcpyHostToDevice, st));
  NFS_HIP(hipMemcpyAsync(cb.chunks, chunks.data(), sizeof(Chunk) * chunks.size(), hipMemcpyHostToDevice, st));
  NFS_HIP(hipMemcpyAsync(cb.tile_chunks, tile_chunks.data(), sizeof(int) * (w.nbins + 1), hipMemcpyHostToDevice, st));
  ScatterArgs<R> sa{};
  sa.pts = pts;
  sa.n = cb.n;
  sa.d = geo.d;
  sa.g = geo.g;
  sa.T = geo.T;
  for (int c = 0; c < 3; ++c) {
    sa.nt[c] = geo.nt[c];
    sa.center[c] = sc.center[c];
  }
  sa.scale = sc.scale;
  sa.keys = cb.keys;
  sa.offsets = cb.offsets;
  sa.cursor = cb.cursor;
  sa.coords = cb.coords;
  sa.perm = cb.perm;
  sa.w0 = v0;
  sa.w0s = cb.w0s;
  sa.w1 = v1;
  sa.w1s = cb.w1s;
  NFS_HIP(launch_scatter(sa, st));
  NFS_HIP(hipStreamSynchronize(st));  // host vectors above must outlive the copies
  return NFS_OK;
}

template <typename R>
static int upload_tables(Work<R>& w, const nfs_params* p, const Scaling& sc, hipStream_t st) {
  const int g = w.geo.g;
  std::vector<cplx<R>> tw(g);
  for (int j = 0; j < g; ++j) {
    const double a = -2.0 * kPi * double(j) / double(g);
    tw[j] = cplx<R>{R(std::cos(a)), R(std::sin(a))};
  }
  NFS_HIP(hipMemcpyAsync(w.tw, tw.data(), sizeof(cplx<R>) * g, hipMemcpyHostToDevice, st));
  std::vector<double> iphi(w.K0);
  for (int k = 0; k < w.K0; ++k) iphi[k] = 1.0 / window_hat(k, p->m, g, w.win);
  NFS_HIP(hipMemcpyAsync(w.inv_phi, iphi.data(), sizeof(double) * w.K0, hipMemcpyHostToDevice, st));
  std::vector<R> t1, t2;
  if (sc.eps_t > 0.0) {
    const int d = p->d;
    const double et = sc.eps_t;
    auto a = diag_table(d, p->N, p->m, g, w.win, [&](double k2) { return gauss_coeff(d, et, k2); });
    auto b = diag_table(d, p->N, p->m, g, w.win, [&](double k2) { return gauss_cost_coeff(d, et, k2); });
    t1.assign(a.begin(), a.end());
    t2.resize(b.size());
    const double inv_s2 = 1.0 / (sc.scale * sc.scale);
    for (size_t i = 0; i < b.size(); ++i) t2[i] = R(b[i] * inv_s2);
    NFS_HIP(hipMemcpyAsync(w.dtab, t1.data(), sizeof(R) * t1.size(), hipMemcpyHostToDevice, st));
    NFS_HIP(hipMemcpyAsync(w.dtab2, t2.data(), sizeof(R) * t2.size(), hipMemcpyHostToDevice, st));
  }
  NFS_HIP(hipStreamSynchronize(st));
  return NFS_OK;
}

// Bounding box of up to two clouds plus weight statistics of one vector.
static int box_stats(double* stats_dev, double* partials, unsigned* counter, int d, const double* p0, long n0,
                     const double* p1, long n1, const double* w, long nw, double host_out[9], hipStream_t st) {
  BoxArgs b{};
  b.pts[0] = p0;
  b.n[0] = n0;
  b.pts[1] = p1;
  b.n[1] = n1;
  b.w = w;
  b.nw = nw;
  b.d = d;
  b.partials = partials;
  b.counter = counter;
  b.out = stats_dev;
  NFS_HIP(launch_bbox(b, st));
  NFS_HIP(hipMemcpyAsync(host_out, stats_dev, sizeof(double) * 9, hipMemcpyDeviceToHost, st));
  NFS_HIP(hipStreamSynchronize(st));
  return NFS_OK;
}

// ----------------------------------------------------------------------------- the fast-summation chain
// grid S (spread, zero on entry) -> U, with the multiplier applied in LDS.
// S is left zero for the next spread.
template <typename R>
static hipError_t fft_chain(Work<R>& w, const R* table, int deriv, hipStream_t st) {
  const Geom& geo = w.geo;
  const int g = geo.g, N = geo.N, d = geo.d, K0 = w.K0;
  Multiplier mu{table, deriv};
  hipError_t e;
  if (d == 1) {
    RowArgs<R> ra{};
    ra.mode = ROW_FUSED1D;
    ra.L = g;
    ra.N = N;
    ra.nrows = 1;
    ra.real_in = w.S;
    ra.real_io = w.U;
    ra.zero_src = 1;
    ra.tw = w.tw;
    ra.mul = mu;
    return launch_rows(ra, st);
  }
  const long rows = w.ncell / g;
  RowArgs<R> ra{};
  ra.mode = ROW_R2C;
  ra.L = g;
  ra.N = N;
  ra.nrows = int(rows);
  ra.real_io = w.S;
  ra.spec = w.W;
  ra.zero_src = 1;
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
    ax.in_ostride = ax.out_ostride = 0;
    ax.inner = K0;
    ax.npen = K0;
    if ((e = launch_axis(ax, st)) != hipSuccess) return e;
  } else {
    // axis 1 forward: W[l0][l1][k2] -> V[l0][k1'][k2]
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
    a1.npen = long(g) * K0;
    if ((e = launch_axis(a1, st)) != hipSuccess) return e;
    AxisArgs<R> a0 = ax;
    a0.mode = AX_FUSED;
    a0.in = w.V;
    a0.out = w.V;
    a0.nin = g;
    a0.nout = g;
    a0.in_stride = a0.out_stride = long(N + 1) * K0;
    a0.in_ostride = a0.out_ostride = 0;
    a0.inner = (N + 1) * K0;
    a0.npen = long(N + 1) * K0;
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
    a2.npen = long(g) * K0;
    if ((e = launch_axis(a2, st)) != hipSuccess) return e;
  }
  RowArgs<R> rb{};
  rb.mode = ROW_C2R;
  rb.L = g;
  rb.N = N;
  rb.nrows = int(rows);
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
  a.grid = w.S;
  a.win = w.win;
  return a;
}

// Spreading into the grid S (zero on entry; the forward FFT pass zeroes it
// again after reading): either chunk tiles summed per (tile, neighbour) or LDS
// tiles flushed straight to the grid with global atomics.
template <typename R>
static hipError_t spread(Work<R>& w, const CloudBuf<R>& src, const double* weights, const double* wmul,
                         double wconst, hipStream_t st) {
  SpreadArgs<R> a = spread_args(w, src, weights, wmul);
  a.wconst = wconst;
  if (!w.two_level) return launch_spread(a, src.nchunks, st);
  a.part = w.part;
  hipError_t e = launch_spread(a, src.nchunks, st);
  if (e != hipSuccess) return e;
  ReduceArgs<R> r{};
  r.geo = w.geo;
  r.part = w.part;
  r.tile_chunks = src.tile_chunks;
  r.grid = w.S;
  return launch_spread_reduce(r, w.nbins, st);
}

template <typename R>
static InterpArgs<R> interp_args(Work<R>& w, const CloudBuf<R>& tgt, int epi, const double* wmul_src) {
  InterpArgs<R> a{};
  a.geo = w.geo;
  a.coords = tgt.coords;
  a.chunks = tgt.chunks;
  a.grid = w.U;
  a.win = w.win;
  a.norm = 1.0;
  a.wmul_src = wmul_src;
  a.epi = epi;
  a.perm = tgt.perm;
  a.out_stride = 1;
  a.partials = w.partials;
  a.counter = w.counters + CT_INTERP;
  return a;
}

// One Sinkhorn half-step: spread the scalings of `src`, transform, and update
// (or evaluate) the scalings of `tgt` (eq. (S1) via eq. (fastsum)).
template <typename R>
static hipError_t half_step(Work<R>& w, CloudBuf<R>& src, CloudBuf<R>& tgt, double* wmul_src, double* wmul_tgt,
                            double* stats, int epi, hipStream_t st) {
  hipError_t e;
  if ((e = spread(w, src, src.w1s, wmul_src, 1.0, st)) != hipSuccess) return e;
  if ((e = fft_chain(w, w.dtab, -1, st)) != hipSuccess) return e;
  InterpArgs<R> ia = interp_args(w, tgt, epi, wmul_src);
  ia.p = tgt.w0s;
  ia.alpha = tgt.w1s;
  ia.stats = stats;
  ia.wmul_next = epi == EPI_SINK ? wmul_tgt : nullptr;
  return launch_interp(ia, tgt.nchunks, st);
}

// ----------------------------------------------------------------------------- entry point bodies
template <typename R>
static int do_fastsum(const nfs_params* p, const double* src, int64_t ns, const double* wv, const double* tgt,
                      int64_t nt, double* out, void* ws, size_t wsb, hipStream_t st) {
  Work<R> w;
  carve(w, p, ns, nt, nullptr, 1);
  if (wsb < w.bytes) return fail(NFS_EWORKSPACE, "workspace too small");
  carve(w, p, ns, nt, static_cast<char*>(ws), 1);
  NFS_HIP(launch_fill(w.counters, sizeof(unsigned) * CT_TOTAL, st));
  NFS_HIP(launch_fill(w.stats, sizeof(double) * ST_TOTAL, st));
  double box[9];
  NFS_TRY(box_stats(w.stats + ST_BOX, w.partials, w.counters + CT_BOX, p->d, src, ns, tgt, nt, wv, ns, box, st));
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(box[i])) return fail(NFS_EINVAL, "non-finite point coordinates or weights");
  Scaling sc = choose_scaling(p->d, p->r, p->eps, p->N, box, box + 3);
  NFS_TRY(sort_cloud(w, w.A, src, sc, wv, nullptr, st));
  NFS_TRY(sort_cloud(w, w.B, tgt, sc, nullptr, nullptr, st));
  NFS_TRY(upload_tables(w, p, sc, st));
  NFS_HIP(launch_fill(w.S, sizeof(R) * w.ncell, st));
  const double wmax = box[6] > 0.0 ? box[6] : 1.0;
  NFS_HIP(spread(w, w.A, w.A.w0s, nullptr, 1.0 / wmax, st));
  NFS_HIP(fft_chain(w, w.dtab, -1, st));
  InterpArgs<R> ia = interp_args(w, w.B, EPI_OUT, nullptr);
  ia.norm = wmax;
  ia.out = out;
  NFS_HIP(launch_interp(ia, w.B.nchunks, st));
  NFS_HIP(hipStreamSynchronize(st));
  return NFS_OK;
}

template <typename R>
static int do_nfft(const nfs_params* p, bool adjoint, const double* pts, int64_t n, const double* wv,
                   const double* fhat_in, double* fhat_out, double* out, void* ws, size_t wsb, hipStream_t st) {
  Work<R> w;
  carve(w, p, n, 1, nullptr, 1);
  if (wsb < w.bytes) return fail(NFS_EWORKSPACE, "workspace too small");
  carve(w, p, n, 1, static_cast<char*>(ws), 1);
  NFS_HIP(launch_fill(w.counters, sizeof(unsigned) * CT_TOTAL, st));
  double box[9];
  NFS_TRY(box_stats(w.stats + ST_BOX, w.partials, w.counters + CT_BOX, p->d, pts, n, nullptr, 0, wv, wv ? n : 0,
                    box, st));
  for (int c = 0; c < p->d; ++c)
    if (!(box[c] >= -0.5) || !(box[3 + c] < 0.5)) return fail(NFS_EINVAL, "NFFT points must lie in [-1/2, 1/2)^d");
  Scaling sc{};
  sc.scale = 0.0;  // points are already torus coordinates
  NFS_TRY(sort_cloud(w, w.A, pts, sc, wv, nullptr, st));
  NFS_TRY(upload_tables(w, p, sc, st));
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
  ax.mul = Multiplier{nullptr, -1};
  if (adjoint) {
    NFS_HIP(launch_fill(w.S, sizeof(R) * w.ncell, st));
    // weights normalized by max |w| so every spread contribution is at most one in size
    const double wmax = box[6] > 0.0 ? box[6] : 1.0;
    NFS_HIP(spread(w, w.A, w.A.w0s, nullptr, 1.0 / wmax, st));
    sp.scale = wmax;
    RowArgs<R> ra{};
    ra.mode = ROW_R2C;
    ra.L = g;
    ra.N = N;
    ra.nrows = int(rows);
    ra.real_io = w.S;
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
    InterpArgs<R> ia = interp_args(w, w.A, EPI_OUT, nullptr);
    ia.out = out;
    NFS_HIP(launch_interp(ia, w.A.nchunks, st));
  }
  NFS_HIP(hipStreamSynchronize(st));
  return NFS_OK;
}

static int check_weights(const double box[9], long n, long nt_other, const char* name) {
  const double tol = 1e-12 * double(std::max(n, nt_other));
  if (box[7] < 0.0) return fail(NFS_EWEIGHTS, std::string(name) + " has a negative weight");
  if (!(std::fabs(box[8] - 1.0) <= tol)) return fail(NFS_EWEIGHTS, std::string(name) + " does not sum to 1");
  return NFS_OK;
}

struct SolveCtx {
  Scaling sc;
  double box_x[9], box_y[9];
};

// Plan shared by solve and grad: scaling from both clouds, sorting with the
// weights (and scalings) gathered into sorted order, tables.
template <typename R>
static int plan_sinkhorn(Work<R>& w, const nfs_params* p, const double* x, long n, const double* mu, const double* y,
                         long nt, const double* nu, const double* ax, const double* ay, SolveCtx& ctx,
                         hipStream_t st) {
  NFS_HIP(launch_fill(w.counters, sizeof(unsigned) * CT_TOTAL, st));
  NFS_HIP(launch_fill(w.stats, sizeof(double) * ST_TOTAL, st));
  NFS_TRY(box_stats(w.stats + ST_BOX, w.partials, w.counters + CT_BOX, p->d, x, n, y, nt, mu, n, ctx.box_x, st));
  NFS_TRY(box_stats(w.stats + ST_BOX2, w.partials, w.counters + CT_BOX, p->d, nullptr, 0, nullptr, 0, nu, nt,
                    ctx.box_y, st));
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(ctx.box_x[i]) || !std::isfinite(ctx.box_y[i]))
      return fail(NFS_EINVAL, "non-finite point coordinates or weights");
  NFS_TRY(check_weights(ctx.box_x, n, nt, "mu"));
  NFS_TRY(check_weights(ctx.box_y, nt, n, "nu"));
  ctx.sc = choose_scaling(p->d, p->r, p->eps, p->N, ctx.box_x, ctx.box_x + 3);
  NFS_TRY(sort_cloud(w, w.A, x, ctx.sc, mu, ax, st));
  NFS_TRY(sort_cloud(w, w.B, y, ctx.sc, nu, ay, st));
  NFS_TRY(upload_tables(w, p, ctx.sc, st));
  NFS_HIP(launch_fill(w.S, sizeof(R) * w.ncell, st));
  return NFS_OK;
}

// Persistent Sinkhorn state: plan done once, one iteration captured in a
// hipGraph on an internal stream and replayed; read-out on demand.
struct SolverBase {
  virtual ~SolverBase() {}
  virtual int iterate(int k, hipStream_t caller) = 0;
  virtual int residual(double* err_row, hipStream_t caller) = 0;
  virtual int finish(double* alpha, double* alpha_t, nfs_result* res, hipStream_t caller) = 0;
  virtual int profile(int k, double* stage_ms, hipStream_t caller) = 0;
  virtual int stage_info(double* info) = 0;
};

template <typename R>
struct Solver : SolverBase {
  nfs_params p{};
  Work<R> w;
  SolveCtx ctx{};
  long n = 0, nt = 0;
  int done = 0;
  hipStream_t gs = nullptr;
  hipEvent_t ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  double* stats() { return w.stats; }
  double* wmul_x() { return w.stats + ST_WMUL_X; }
  double* wmul_y() { return w.stats + ST_WMUL_Y; }

  hipError_t iteration(hipStream_t s) {
    hipError_t e = half_step(w, w.B, w.A, wmul_y(), wmul_x(), stats() + ST_ROW, EPI_SINK, s);
    if (e != hipSuccess) return e;
    return half_step(w, w.A, w.B, wmul_x(), wmul_y(), stats() + ST_COL, EPI_SINK, s);
  }

  int create(const nfs_params* prm, const double* x, long n_, const double* mu, const double* y, long nt_,
             const double* nu, const double* alpha_t0, void* ws, size_t wsb, hipStream_t caller) {
    p = *prm;
    n = n_;
    nt = nt_;
    carve(w, &p, n, nt, nullptr, 2);
    if (wsb < w.bytes) return fail(NFS_EWORKSPACE, "workspace too small");
    carve(w, &p, n, nt, static_cast<char*>(ws), 2);
    hipStream_t st = caller;
    NFS_TRY(plan_sinkhorn(w, &p, x, n, mu, y, nt, nu, nullptr, alpha_t0, ctx, st));
    NFS_HIP(launch_fill_double(w.A.w1s, n, 1.0, st));
    if (!alpha_t0) {
      NFS_HIP(launch_fill_double(w.B.w1s, nt, 1.0, st));
      NFS_HIP(launch_fill_double(wmul_y(), 1, 1.0, st));
    } else {
      double box[9];
      NFS_TRY(box_stats(stats() + ST_MISC, w.partials, w.counters + CT_BOX, p.d, nullptr, 0, nullptr, 0, alpha_t0,
                        nt, box, st));
      if (!(box[7] > 0.0) || !std::isfinite(box[6]))
        return fail(NFS_EINVAL, "warm-start alpha_t must be positive and finite");
      NFS_HIP(launch_fill_double(wmul_y(), 1, 1.0 / box[6], st));
    }
    NFS_HIP(launch_fill_double(wmul_x(), 1, 1.0, st));
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
      if (e != hipSuccess) return fail(NFS_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    return NFS_OK;
  }

  ~Solver() override {
    if (gexec) hipGraphExecDestroy(gexec);
    if (graph) hipGraphDestroy(graph);
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
    for (int i = 0; i < k; ++i) {
      hipError_t e = gexec ? hipGraphLaunch(gexec, gs) : iteration(gs);
      if (e != hipSuccess) return fail(NFS_EHIP, std::string("iteration: ") + hipGetErrorString(e));
    }
    done += k;
    return leave(caller);
  }

  int residual(double* err_row, hipStream_t caller) override {
    NFS_TRY(enter(caller));
    NFS_HIP(half_step(w, w.B, w.A, wmul_y(), wmul_x(), stats() + ST_EVAL, EPI_EVAL, gs));
    double h[4];
    NFS_HIP(hipMemcpyAsync(h, stats() + ST_EVAL, sizeof(h), hipMemcpyDeviceToHost, gs));
    NFS_HIP(hipStreamSynchronize(gs));
    *err_row = std::sqrt(h[0]);
    return leave(caller);
  }

  // Per-stage device times with events between the kernels of `k` iterations
  // (direct launches on the internal stream, no graph).  stage_ms receives the
  // average per launch of: [0] spread, [1] FFT chain, [2] interpolation + update,
  // [3] whole iteration.
  int profile(int k, double* stage_ms, hipStream_t caller) override {
    if (k <= 0) return fail(NFS_EINVAL, "profile needs k >= 1");
    NFS_TRY(enter(caller));
    std::vector<hipEvent_t> evs(8 * k + 1);
    for (auto& e : evs) NFS_HIP(hipEventCreate(&e));
    int ie = 0;
    NFS_HIP(hipEventRecord(evs[ie++], gs));
    for (int it = 0; it < k; ++it) {
      for (int h = 0; h < 2; ++h) {
        CloudBuf<R>& src = h == 0 ? w.B : w.A;
        CloudBuf<R>& tgt = h == 0 ? w.A : w.B;
        double* ws_ = h == 0 ? wmul_y() : wmul_x();
        double* wt_ = h == 0 ? wmul_x() : wmul_y();
        NFS_HIP(spread(w, src, src.w1s, ws_, 1.0, gs));
        NFS_HIP(hipEventRecord(evs[ie++], gs));
        NFS_HIP(fft_chain(w, w.dtab, -1, gs));
        NFS_HIP(hipEventRecord(evs[ie++], gs));
        InterpArgs<R> ia = interp_args(w, tgt, EPI_SINK, ws_);
        ia.p = tgt.w0s;
        ia.alpha = tgt.w1s;
        ia.stats = stats() + (h == 0 ? ST_ROW : ST_COL);
        ia.wmul_next = wt_;
        NFS_HIP(launch_interp(ia, tgt.nchunks, gs));
        NFS_HIP(hipEventRecord(evs[ie++], gs));
        ie++;  // keep 4 slots per half-step (last unused)
      }
    }
    NFS_HIP(hipStreamSynchronize(gs));
    double acc[3] = {0, 0, 0};
    float ms;
    int prev = 0;
    ie = 1;
    for (int it = 0; it < k; ++it)
      for (int h = 0; h < 2; ++h) {
        for (int s = 0; s < 3; ++s) {
          NFS_HIP(hipEventElapsedTime(&ms, evs[prev], evs[ie]));
          acc[s] += ms;
          prev = ie;
          ++ie;
        }
        ++ie;
      }
    NFS_HIP(hipEventElapsedTime(&ms, evs[0], evs[prev]));
    for (int s = 0; s < 3; ++s) stage_ms[s] = acc[s] / (2.0 * k);
    stage_ms[3] = ms / k;
    for (auto& e : evs) hipEventDestroy(e);
    done += k;
    return leave(caller);
  }

  // Sizes that set the algorithmic traffic: [0] n, [1] nt, [2] d, [3] grid cells,
  // [4] bytes per grid cell, [5] chunks of x, [6] chunks of y, [7] taps per point.
  int stage_info(double* info) override {
    info[0] = double(n);
    info[1] = double(nt);
    info[2] = p.d;
    info[3] = double(w.ncell);
    info[4] = double(sizeof(R));
    info[5] = w.A.nchunks;
    info[6] = w.B.nchunks;
    info[7] = std::pow(2.0 * p.m + 1.0, p.d);
    return NFS_OK;
  }

  int finish(double* alpha, double* alpha_t, nfs_result* res, hipStream_t caller) override {
    NFS_TRY(enter(caller));
    hipStream_t st = gs;
    double* S = stats();
    // row residual of eq. (Error): one extra product K alpha_t
    NFS_HIP(half_step(w, w.B, w.A, wmul_y(), wmul_x(), S + ST_EVAL, EPI_EVAL, st));
    double ev_row[8];
    NFS_HIP(hipMemcpyAsync(ev_row, S + ST_EVAL, sizeof(ev_row), hipMemcpyDeviceToHost, st));
    NFS_HIP(half_step(w, w.A, w.B, wmul_x(), wmul_y(), S + ST_EVAL, EPI_EVAL, st));
    ReadoutArgs ra{w.A.w0s, w.A.w1s, n, w.partials, w.counters + CT_RD, S + ST_RD_X};
    NFS_HIP(launch_readout(ra, st));
    ReadoutArgs rb{w.B.w0s, w.B.w1s, nt, w.partials, w.counters + CT_RD, S + ST_RD_Y};
    NFS_HIP(launch_readout(rb, st));
    if (p.flags & NFS_FLAG_PRIMAL_COST) {
      NFS_HIP(spread(w, w.B, w.B.w1s, wmul_y(), 1.0, st));
      NFS_HIP(fft_chain(w, w.dtab2, -1, st));
      InterpArgs<R> ia = interp_args(w, w.A, EPI_OUT, wmul_y());
      ia.out = w.tmp;
      ia.scale_vec = w.A.w1s;
      NFS_HIP(launch_interp(ia, w.A.nchunks, st));
      ReadoutArgs rc2{w.tmp, w.tmp, n, w.partials, w.counters + CT_RD, S + ST_MISC + 8};
      NFS_HIP(launch_readout(rc2, st));
    }
    if (alpha) NFS_HIP(launch_unpermute(w.A.w1s, w.A.perm, n, alpha, st));
    if (alpha_t) NFS_HIP(launch_unpermute(w.B.w1s, w.B.perm, nt, alpha_t, st));
    double hs[ST_TOTAL];
    NFS_HIP(hipMemcpyAsync(hs, S, sizeof(hs), hipMemcpyDeviceToHost, st));
    NFS_HIP(hipStreamSynchronize(st));
    NFS_TRY(leave(caller));
    const double eps = p.eps;
    nfs_result r{};
    r.iters = done;
    r.precision_used = p.precision;
    r.scale = ctx.sc.scale;
    r.kernel_err = ctx.sc.kernel_err;
    // s = eps (1 + sum p log a + sum pt log at - sum_j at_j tt_j), tt the last K^T alpha
    const double mass = done > 0 ? hs[ST_COL + 1] : ev_row[1];
    r.cost = eps * (1.0 + hs[ST_RD_X + 0] + hs[ST_RD_Y + 0] - mass);
    r.cost_upper = r.cost - eps * (hs[ST_RD_X + 1] + hs[ST_RD_Y + 1]);
    r.cost_primal = (p.flags & NFS_FLAG_PRIMAL_COST) ? hs[ST_MISC + 8 + 2] : NAN;
    r.marg_err_row = std::sqrt(ev_row[0]);
    r.marg_err_col = std::sqrt(hs[ST_EVAL + 0]);
    r.marg_err = r.marg_err_row + r.marg_err_col;
    r.n_nonpos = int64_t(hs[ST_ROW + 4] + hs[ST_COL + 4]);
    if (res) *res = r;
    if (r.n_nonpos > 0)
      return fail(NFS_ENONPOS, "fast summation produced kernel sums t <= 0 (normwise error above the dynamic range)");
    return NFS_OK;
  }
};

static int make_solver(const nfs_params* prm, const double* x, int64_t n, const double* mu, const double* y,
                       int64_t nt, const double* nu, const double* alpha_t0, void* ws, size_t wsb, hipStream_t st,
                       SolverBase** out) {
  *out = nullptr;
  if (prm->precision == NFS_FP32) {
    auto* s = new Solver<float>();
    int rc = s->create(prm, x, n, mu, y, nt, nu, alpha_t0, ws, wsb, st);
    if (rc != NFS_OK) {
      delete s;
      return rc;
    }
    *out = s;
  } else {
    auto* s = new Solver<double>();
    int rc = s->create(prm, x, n, mu, y, nt, nu, alpha_t0, ws, wsb, st);
    if (rc != NFS_OK) {
      delete s;
      return rc;
    }
    *out = s;
  }
  return NFS_OK;
}

static int do_solve(const nfs_params* p, const double* x, int64_t n, const double* mu, const double* y, int64_t nt,
                    const double* nu, int32_t max_iter, double tol, int32_t warm, double* alpha, double* alpha_t,
                    nfs_result* res, void* ws, size_t wsb, hipStream_t caller) {
  SolverBase* s = nullptr;
  NFS_TRY(make_solver(p, x, n, mu, y, nt, nu, warm ? alpha_t : nullptr, ws, wsb, caller, &s));
  int rc = NFS_OK;
  int done = 0;
  const int check_every = 10;
  while (rc == NFS_OK && done < max_iter) {
    const int k = tol > 0.0 ? std::min(check_every, max_iter - done) : max_iter - done;
    rc = s->iterate(k, caller);
    done += k;
    if (rc == NFS_OK && tol > 0.0) {
      double e = 0.0;
      rc = s->residual(&e, caller);
      if (rc == NFS_OK && e <= tol) break;
    }
  }
  if (rc == NFS_OK) rc = s->finish(alpha, alpha_t, res, caller);
  delete s;
  return rc;
}

template <typename R>
static int do_grad(const nfs_params* p, const double* x, int64_t n, const double* mu, const double* y, int64_t nt,
                   const double* nu, const double* alpha, const double* alpha_t, double* grad_x, double* grad_mu,
                   void* ws, size_t wsb, hipStream_t st) {
  Work<R> w;
  carve(w, p, n, nt, nullptr, 2);
  if (wsb < w.bytes) return fail(NFS_EWORKSPACE, "workspace too small");
  carve(w, p, n, nt, static_cast<char*>(ws), 2);
  SolveCtx ctx;
  NFS_TRY(plan_sinkhorn(w, p, x, n, mu, y, nt, nu, alpha, alpha_t, ctx, st));
  if (grad_mu) NFS_HIP(launch_gradmu(alpha, n, p->eps, w.partials, w.counters + CT_RD, w.stats + ST_LOGMEAN, grad_mu, st));
  if (grad_x) {
    double box[9];
    NFS_TRY(box_stats(w.stats + ST_MISC, w.partials, w.counters + CT_BOX, p->d, nullptr, 0, nullptr, 0, alpha_t, nt,
                      box, st));
    if (!(box[6] > 0.0) || !std::isfinite(box[6])) return fail(NFS_EINVAL, "alpha_t must be positive and finite");
    const double wmax = box[6];
    // The spectrum of the spread alpha_t is formed once per derivative axis;
    // each pass applies (2 pi i k_c) b_k / Phi^2 and interpolates at x.
    for (int c = 0; c < p->d; ++c) {
      NFS_HIP(spread(w, w.B, w.B.w1s, nullptr, 1.0 / wmax, st));
      NFS_HIP(fft_chain(w, w.dtab, c, st));
      InterpArgs<R> ia = interp_args(w, w.A, EPI_OUT, nullptr);
      // grad_x_i = -eps alpha_i s (dK'/dx'_c * alpha_t)(x'_i), x' = s (x - center)
      ia.norm = -p->eps * ctx.sc.scale * wmax;
      ia.scale_vec = w.A.w1s;
      ia.out = grad_x;
      ia.out_stride = p->d;
      ia.out_comp = c;
      NFS_HIP(launch_interp(ia, w.A.nchunks, st));
    }
  }
  NFS_HIP(hipStreamSynchronize(st));
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
  NFS_TRY(check_params(prm, n, nt));
  if (!bytes) return fail(NFS_EINVAL, "bytes is NULL");
  if (prm->precision == NFS_FP32) {
    Work<float> w;
    carve(w, prm, n, nt, nullptr, 2);
    *bytes = w.bytes;
  } else {
    Work<double> w;
    carve(w, prm, n, nt, nullptr, 2);
    *bytes = w.bytes;
  }
  return NFS_OK;
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
  NFS_TRY(check_params(prm, n, nt));
  if (!x || !mu || !y || !nu || !alpha || !alpha_t || !workspace) return fail(NFS_EINVAL, "NULL pointer argument");
  if (max_iter < 0) return fail(NFS_EINVAL, "max_iter must be >= 0");
  return do_solve(prm, x, n, mu, y, nt, nu, max_iter, tol, warm_start, alpha, alpha_t, res, workspace, ws_bytes,
                  static_cast<hipStream_t>(stream));
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
  NFS_TRY(make_solver(prm, x, n, mu, y, nt, nu, alpha_t0, workspace, ws_bytes, static_cast<hipStream_t>(stream), &s));
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

int nfs_solver_destroy(nfs_solver* s) {
  delete reinterpret_cast<SolverBase*>(s);
  return NFS_OK;
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

}  // extern "C"
