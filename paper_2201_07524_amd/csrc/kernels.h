// Kernel argument structs and launcher declarations (host side of the kernels).
#pragma once

#include "common.h"

namespace nfs {

enum Epilogue : int {
  EPI_OUT = 0,   // out[perm[q]*stride + comp] = t * scale_vec[q]
  EPI_SINK = 1,  // alpha[q] = p[q]/t with the residual of the old alpha[q], and the reductions
                 // below (Algorithm 3 half-step)
  EPI_EVAL = 2,  // residual sum (alpha[q] t - p[q])^2 only, no update
  // Log domain (Algorithm 4): alpha[] holds potentials beta, the source side's
  // weights were exp((gamma - shift)/eps) with shift = wmul_src[prob], so the
  // kernel sum is t = exp(shift/eps - 1/2) S with S the interpolated value.
  EPI_LOGSINK = 3,  // beta[q] = eps (log p[q] - log S + 1) - shift, mass and max reductions
  EPI_LOGEVAL = 4,  // residual sum (exp((beta[q] + shift)/eps - 1) S - p[q])^2 only, no update
};

// Per-problem constants of the log domain: leps[2 b] = 1/eps_b, leps[2 b + 1] = eps_b.
constexpr int kLepsStride = 2;

// Per-problem statistics of a half-step (doubles, stride kStat), written by
// the last workgroup of the problem's interpolation:
//   [0] sum (alpha_old t - p)^2: the squared residual of eq. (Error) of the
//       state before the update (the row term at an alpha update, the column
//       term at an alpha_t update)
//   [1] sum alpha_new t (mass; EPI_EVAL: sum alpha_old t)
//   [2] max alpha_new (EPI_EVAL: max alpha_old; log domain: max potential)
//   [3] count of sums t <= 0 or non-finite in this launch, [4] running count
//   [5] min t, [6] max t over targets of positive weight
//   [7] sum |alpha_new| (the l1 norm of the next half-step's source weights)
//   [8] running max of ||w||_1 / min t, w the source weights (scaling form:
//       the dynamic range the sums had to resolve)
constexpr int kStat = 16;
// Per-problem state of a solve (ints, stride kPState): [0] 0 running, 1 the
// alpha update found ||E|| <= tol for the state before it, 2 stopped (every
// kernel of an iteration skips the problem); [1] iterations completed.
constexpr int kPState = 2;

// Format of the spread grid S, written by the spreading flush and read by
// the forward row pass: R values summed with float atomics (GRID_REAL), or
// the exact integer sums of the LDS tiles' fixed-point words (int64 atomics,
// so S does not depend on the order of the flushes): GRID_FIX64 one word per
// cell in units of 2^-32, GRID_FIX128 two planes (2^-30, then 2^-60 units,
// the second `grid_plane` words after the first).
enum GridMode : int { GRID_REAL = 0, GRID_FIX64 = 1, GRID_FIX128 = 2 };
// Mode of the spreading kernel for this geometry and value type (two_level:
// the per-tile reduction, which sums R values).
int spread_grid_mode(const Geom& geo, int rbytes, bool two_level);
// Bytes per grid cell of S in that mode.
inline size_t grid_cell_bytes(int mode, size_t rbytes) {
  return mode == GRID_FIX128 ? 16 : (mode == GRID_FIX64 ? 8 : rbytes);
}

template <typename R>
struct SpreadArgs {
  Geom geo;
  const R* coords;       // sorted tile-local coordinates, n x d
  const double* w;       // sorted weights
  const double* wmul;    // per-problem multiplier of the weights, indexed by chunk.prob (nullable)
  double wconst;         // host constant multiplier of the weights
  const Chunk* chunks;
  const int* runs;       // run table of each chunk (offsets from the chunk's start)
  const int* nruns;      // per chunk: full runs, single points
  // Spreading's own run table (nullable; cell order only): every cell's points
  // in ceil(c / G) runs, the last one partial.  Entries are offset | (count - 1) << 16:
  // groups of four same-cell runs, then same-cell pairs, then the remaining runs.
  // nsrun: 3 per chunk (quad entries, pair entries, solo runs).
  const int* srun;
  const int* nsrun;
  int cell_order;        // points sorted by cell inside each tile
  R* grid;               // problem p's g^d grid at cell p*grid_stride, zero on entry, in the format gmode
  long grid_stride;
  int gmode;             // GridMode of grid (GRID_REAL when part is set)
  long grid_plane;       // GRID_FIX128: words between the two planes
  const int* pstate;     // nullable: chunks of problems in state 2 are skipped
  R* part;               // non-null: store each chunk's padded tile here instead of flushing
  WindowConst win;
  const void* __restrict__ wpoly;   // window polynomials: WindowPoly::c (FP32) or WindowPoly64::c (FP64)
};

// Sum of the padded chunk tiles into the grid: one workgroup per (tile, neighbour)
// sums the overlap of that neighbour's chunks and adds it to the grid with
// at most 3^d atomic adds per cell (the grid must be zero on entry).
template <typename R>
struct ReduceArgs {
  Geom geo;
  const R* part;           // chunk tiles, E^d values each
  const int* tile_chunks;  // nbins + 1 offsets into the chunk list (chunks are sorted by tile)
  R* grid;
  const int* pstate;       // nullable: nothing to do when the (single) problem is in state 2
};
template <typename R>
hipError_t launch_spread_reduce(const ReduceArgs<R>& a, int nbins, hipStream_t st);

template <typename R>
struct InterpArgs {
  Geom geo;
  const R* coords;
  const Chunk* chunks;
  const int* runs;          // run table of each chunk (offsets from the chunk's start)
  const int* nruns;         // per chunk: full runs, single points
  int cell_order;           // points sorted by cell inside each tile
  const R* grid;            // problem p's grid at grid + p*grid_stride
  long grid_stride;
  WindowConst win;
  const void* __restrict__ wpoly;   // window polynomials: WindowPoly::c (FP32) or WindowPoly64::c (FP64)
  double norm;              // constant factor of the result
  const double* wmul_src;   // the result is divided by wmul_src[prob] (nullable); log domain:
                            // the source potentials' shift
  const double* leps;       // log domain constants (EPI_LOGSINK / EPI_LOGEVAL)
  int epi;
  // EPI_OUT
  const int* perm;
  double* out;
  int out_stride;
  int out_comp;
  const double* scale_vec;  // sorted per-point factor (nullable)
  const double* nf;         // sorted per-target near-field sum added before scaling (nullable)
  // EPI_SINK / EPI_EVAL
  const double* p;
  double* alpha;
  double* partials;         // kRedVals doubles per chunk
  int nprob;                // problems B
  const int* prob_chunks;   // B + 1: chunks of problem p are [prob_chunks[p], prob_chunks[p+1])
  double* stats;            // per problem, stride kStat (layout above)
  double* wmul_next;        // per problem, receives 1/max alpha (log domain: max beta) (nullable)
  const double* src_l1;     // nullable: per problem (stride kStat) the l1 norm of the source weights
  int* pstate;              // nullable: per problem (stride kPState); stopped problems are skipped
  const double* tol2;       // with pstate: squared tolerance on the residual (<= 0: never stop)
  int half;                 // with pstate: 0 alpha update (residual checked), 1 alpha_t update
};

// Near-field correction for r = 1 and real exponents rho (kernel
// exp(-|z|^rho/eps) regularized inside |z| < eps_I by an even polynomial): for
// every target,
//   out[q] = sum_{sources j within eps_I} w_j wm (K - K_R)(x_q - y_j),
// over the sources of the (2 kt + 1)^d neighbour tiles.  Per-problem constants
// (stride kNearStride doubles): [0] 1/(eps_t g) (cell distance -> r/eps),
// [1] eps_I^2 in cells^2, [2] 1/eps_I^2 in cells^-2, [3] p, [4 + j] c_j (j < p <= 16),
// [kNearRhoHalf] rho/2, [kNearRhoInv] 1/(eps_t g^rho) ((cell distance)^rho -> r^rho/eps).
// NearArgs::real_exp selects K = exp(-(r2 cells)^(rho/2) [kNearRhoInv]); else rho = 1.
// NearArgs::cost selects the primal cost's kernel c K instead, c = |x - y|^rho in
// the caller's units: K_c = (r2 cells)^(rho/2) [kNearCostMul] exp(-(r2 cells)^(rho/2)
// [kNearRhoInv]) with [kNearCostMul] = 1/(g s)^rho (s the torus scale) and the c_j
// of its own regularizing polynomial (a second coefficient block), any rho.
constexpr int kNearStride = 24;
constexpr int kNearRhoHalf = 20;
constexpr int kNearRhoInv = 21;
constexpr int kNearCostMul = 22;
// Exponent forms of the near-field kernels (template parameter FORM).
constexpr int kNearR1 = 0;    // exp(-r/eps)
constexpr int kNearReal = 1;  // exp(-r^rho/eps)
constexpr int kNearCost = 2;  // r^rho exp(-r^rho/eps), scaled to the caller's cost units
template <typename R>
struct NearArgs {
  Geom geo;
  const R* tcoords;
  const Chunk* tchunks;
  const R* scoords;
  const double* sw;
  const int* soffsets;  // B x nbins: first sorted source of each tile
  const int* scounts;   // B x nbins
  const double* wmul;   // per problem (nullable)
  double wconst;
  const double* coef;   // B x kNearStride
  int kt;
  int ps;               // polynomial terms p
  double* out;
  long out_plane;       // gradient: entries between the components of out
  const int* pstate;    // nullable: targets of problems in state 2 are skipped
  const int* scell;     // nullable: per source tile the cell starts (TileSortArgs::cellstart);
                        // with it only the source cells within eps_I of each wave's targets are read
  int real_exp;         // kernel exp(-|z|^rho/eps) with the real rho of coef (else rho = 1)
  int cost;             // the primal cost's kernel |z|^rho exp(-|z|^rho/eps) (coef: its own block)
};
template <typename R>
hipError_t launch_nearfield(const NearArgs<R>& a, int nchunks, hipStream_t st);
// Gradient of the same near-field sum at the targets, d components in torus
// units: out[c * out_plane + q] (q in sorted target order).
template <typename R>
hipError_t launch_nearfield_grad(const NearArgs<R>& a, int nchunks, hipStream_t st);

template <typename R>
hipError_t launch_spread(const SpreadArgs<R>& a, int nchunks, hipStream_t st);
template <typename R>
hipError_t launch_interp(const InterpArgs<R>& a, int nchunks, hipStream_t st);

// ----------------------------------------------------------------------------- FFT
// Spectral multiplier applied inside the axis-0 pass: value(k) = Dtab[|k0|,|k1|,|k2|]
// (table of extent H = N/2+1 per dimension, row-major), optionally times
// i 2 pi k_c for the derivative axis c (deriv < 0: none).
struct Multiplier {
  const void* tab;   // R table, (N/2+1)^d entries per problem
  int deriv;         // -1 or derivative axis
  long tab_stride;   // entries between the tables of consecutive problems
};

// FFT pass plan for a length 2^rem: radix-4 passes while two or more bits
// remain, then one radix-2 pass.  The device passes and the host twiddle
// table (pass tables of (radix - 1) Ns entries, end to end) both follow it.
__host__ __device__ inline int fft_pass_bits(int rem) { return rem >= 2 ? 2 : rem; }

enum RowMode : int { ROW_R2C = 0, ROW_C2R = 1, ROW_FUSED1D = 2 };
enum AxisMode : int { AX_FWD = 0, AX_INV = 1, AX_FUSED = 2 };

template <typename R>
struct RowArgs {
  int mode;
  int L;            // grid size g (FFT length)
  int N;
  int nrows;        // number of real rows
  R* real_io;       // R2C: input rows (zeroed after reading if zero_src); C2R/FUSED1D: output rows
  const R* real_in; // FUSED1D input row
  int gmode;        // R2C / FUSED1D input: GridMode of the spread grid
  long grid_plane;  // GRID_FIX128: words between its two planes
  cplx<R>* spec;    // R2C: output [nrows][K0]; C2R: input [nrows][K0]
  int zero_src;
  const cplx<R>* tw;  // pass twiddle tables (fft_pass_bits), L entries
  int tw_lds;       // set by the launcher: twiddles staged in LDS
  Multiplier mul;   // FUSED1D only
};

template <typename R>
struct AxisArgs {
  int mode;
  int L, N, d;
  const cplx<R>* in;
  cplx<R>* out;
  int nin, in_centered;    // entries along the axis; centered: entry e <-> k = e - N/2
  int nout, out_centered;
  long in_stride, out_stride;     // element stride along the axis
  long in_ostride, out_ostride;   // stride between outer pencil groups
  int inner;                      // pencils per outer group (contiguous)
  long npen;                      // total pencils
  const cplx<R>* tw;
  int tw_lds;          // set by the launcher: twiddles staged in LDS
  Multiplier mul;                 // FUSED: applied between forward and inverse; INV: applied on load
  int apply_mul;
};

template <typename R>
hipError_t launch_rows(const RowArgs<R>& a, hipStream_t st);
template <typename R>
hipError_t launch_axis(const AxisArgs<R>& a, hipStream_t st);

// ----------------------------------------------------------------------------- plan / misc
// out[kBoxVals]: min_c (c < 3), max_c, max |w|, min w, sum w, then, with
// wsum set (w the weights of pts[0], nw = n[0]), sum_i w_i pts[0][i][c].
constexpr int kBoxVals = 12;
struct BoxArgs {
  const double* pts[2];
  long n[2];
  const double* w;    // optional weights (for max |w|, min w, sum w)
  long nw;
  int d;
  int wsum;
  double* partials;   // kBoxVals per block, up to 1024 blocks
  double* out;
};
hipError_t launch_bbox(const BoxArgs& a, hipStream_t st);
// Many boxes in one launch (the per-problem boxes of a batched plan): box j
// is jobs[j] (its partials and d ignored) over workgroups [blk0[j], blk0[j] +
// nblk[j]) of the launch, nblocks in all; partials holds kBoxVals per
// workgroup of the launch.
struct BoxJob {
  BoxArgs box;
  long blk0;
  int nblk;
};
// Workgroups per box: about eight values per thread, at most 1024.
int bbox_blocks(long n);
hipError_t launch_bbox_jobs(const BoxJob* jobs, int njobs, long nblocks, int d, double* partials, hipStream_t st);

// Scalings between the centred form and the caller's variables: with x'
// the mapped point (torus coordinate tau, x' = center + tau/scale) and
// lf = (sign 2 delta . x' + |delta|^2/2)/eps (delta = 2 shift), the caller's
// scaling is the centred one times exp(lf) (potentials: plus eps lf).
// perm set: out[perm[q]] = src[q] exp(lf), the read-out in the caller's
// order; perm NULL: out[q] = src[q] exp(-lf) in sorted order (the start of
// the centred iteration from the caller's start; out may be src).  One
// workgroup per chunk.
template <typename R>
struct UncenterArgs {
  Geom geo;
  const Chunk* chunks;
  const R* coords;       // sorted tile-local coordinates
  const int* perm;
  const double* src;     // sorted scalings (potentials when logd)
  double* out;
  const double* pb;      // per problem (stride kUncStride): scale, center[3], coef[3] = sign 2 delta/eps, cst, eps
  int logd;
};
constexpr int kUncStride = 10;
template <typename R>
hipError_t launch_uncenter(const UncenterArgs<R>& a, int nchunks, hipStream_t st);

struct KeyArgs {
  const double* pts;
  long n;
  int d, g, T;
  int nt[3];
  double center[3];
  double scale;       // torus coordinate = scale*(x - center); scale = 0: points already on the torus
  int* keys;
  int* counts;        // histogram per tile
  // Batched form (probs non-null, one launch for all problems of a plan):
  // pts, keys are the cloud's arrays, counts (and the scatter's offsets and
  // cursor) hold nbins entries per problem, and problem b's points, mapping
  // and first workgroup come from probs[b] (n, center, scale unused).
  const struct PlanProb* probs;
  int nprob;
};
// One problem of a batched plan launch: its points [o, o + n) of the cloud,
// its torus mapping, and the first of the ceil(n / plan_block_points())
// workgroups that take its points.
struct PlanProb {
  long o, n;
  double center[3];
  double scale;
  long blk0;
};
// Points per workgroup of the key and scatter kernels; whether a grid of
// nbins tiles takes their batched form.
long plan_block_points();
bool plan_batchable(int nbins);
hipError_t launch_keys(const KeyArgs& a, hipStream_t st);

template <typename R>
struct ScatterArgs {
  const double* pts;
  long n;
  int d, g, T;
  int nt[3];
  double center[3];
  double scale;
  const int* keys;
  const int* offsets;  // per tile: global first position
  int* cursor;
  R* coords;          // sorted tile-local coordinates (global positions)
  int* perm;          // sorted -> original index (global)
  int idx_base;       // added to the local point index when writing perm
  const double* w0;   // optional gathered vectors (nullable)
  double* w0s;
  const double* w1;
  double* w1s;
  const PlanProb* probs;  // batched form, as in KeyArgs (idx_base then unused)
  int nprob;
};
template <typename R>
hipError_t launch_scatter(const ScatterArgs<R>& a, hipStream_t st);

// Cell sort of every tile: one workgroup per (problem, tile) moves the tile's
// points from the staging arrays (as left by the scatter) to the final arrays
// in increasing order of their cell inside the tile (T^d <= kSortBins cells).
constexpr int kSortBins = 4096;
template <typename R>
struct TileSortArgs {
  const int* counts;    // B x nbins points per tile
  const int* offsets;   // B x nbins first position of each tile
  int ntiles;           // B x nbins
  int d, T;
  R* in_coords;         // staging, n x d (also the scratch of the in-cell ordering)
  int* in_perm;
  double* in_w0;        // nullable
  double* in_w1;        // nullable
  R* coords;
  int* perm;
  double* w0s;          // nullable
  double* w1s;          // nullable
  int* cellstart;       // nullable: B x nbins x (T^d + 1) first position of each cell,
                        // relative to the tile's first point (the last entry is the count)
};
template <typename R>
hipError_t launch_tile_sort(const TileSortArgs<R>& a, hipStream_t st);

// Run table of every chunk.  When the points are in cell order (sorted = 1),
// each cell's points in the chunk
// form full runs of G = run_length(d) and c mod G single points; otherwise
// every point is a single point.  For the chunk starting at `start`,
// runs[start + r] is the offset (from `start`) of the first point of entry r:
// nruns[2 chunk] full runs come first, then nruns[2 chunk + 1] single points.
template <typename R>
struct ChunkRunArgs {
  const Chunk* chunks;
  int nchunks;
  int d, T;
  int sorted;
  int G;
  const R* coords;
  int* runs;
  int* nruns;
  int* srun;    // nullable (cell order only): spreading's run table, see SpreadArgs::srun
  int* nsrun;   // 3 per chunk: quad entries, pair entries, solo runs
};
template <typename R>
hipError_t launch_chunk_runs(const ChunkRunArgs<R>& a, hipStream_t st);

hipError_t launch_fill(void* p, size_t bytes, hipStream_t st);
hipError_t launch_fill_double(double* p, long n, double v, hipStream_t st);
hipError_t launch_unpermute(const double* src_sorted, const int* perm, long n, double* dst, hipStream_t st);

// Tables of the fused diagonal of the Gaussian kernel (r = 2) over |k_c| =
// 0..N/2 per axis (extent H = (N/2+1)^d, row-major) for every problem.  The
// periodized Gaussian of torus temperature e (period 1) has the Fourier
// coefficient prod_c sqrt(pi e) exp(-pi^2 e k_c^2) (Poisson summation); with
// the window transform Phi (inv_phi = 1/Phi):
//   kernel: D(k) = prod_c f(k_c),  f(k) = sqrt(pi e) exp(-pi^2 e k^2) hw(k) / Phi(k)^2
//   cost:   C(k) = D(k) (d e / 2 - pi^2 e^2 |k|^2) / s^2
//           (the coefficients of |z|^2 exp(-|z|^2/e), back in the caller's units)
// hw = 1/2 on |k_c| = N/2: the symmetric form of the real part of the sum over
// I_N.  Problem b: pb[2b] = e, pb[2b + 1] = scale s (e <= 0 leaves zeros); its
// tables start at b H.  Evaluated in FP64, stored as R.
template <typename R>
hipError_t launch_gauss_tables(int d, int N, int B, const double* pb, const double* inv_phi, R* kernel, R* cost,
                               hipStream_t st);

// Diagonal table of a real cost exponent rho (r = 0), in two steps around a
// forward FFT of the grid.  kernel_samples: out[l] = K_R at the grid node l
// (row-major, g per axis, last axis fastest) on the torus, taken at the
// nearest image of the origin, from a near-field coefficient block cf
// (NearArgs::coef layout): the even polynomial inside (cf[1] = (eps_I g)^2
// squared cells) and exp(-r2^(rho/2) cf[kNearRhoInv]) outside (cost: the primal
// cost's kernel r2^(rho/2) cf[kNearCostMul] exp(-r2^(rho/2) cf[kNearRhoInv]), with
// the polynomial of the cost block inside); r2 in squared
// cells.  spec_table: from the forward spectrum of those samples (the row
// transform's k = 0..N/2 on the last axis, centered k = -N/2..N/2 on the
// others, as the adjoint NFFT leaves it), tab[i] = Re(spec) hw / (g^d prod_c
// Phi(k_c)^2) over |k_c| = 0..N/2 (extent (N/2+1)^d, row-major), the same
// table as the Gaussian's.  Evaluated in FP64, stored as R.
template <typename R>
hipError_t launch_kernel_samples(int d, int g, const double* cf, int cost, R* out, hipStream_t st);
template <typename R>
hipError_t launch_spec_table(int d, int N, int g, const cplx<R>* spec, const double* inv_phi, R* tab, hipStream_t st);

// readout: over sorted arrays, out[0] += sum a*log(b) (a>0), out[1] += sum a*log(a), out[2] += sum a
struct ReadoutArgs {
  const double* a;
  const double* b;
  long n;
  int logv;  // b holds potentials: sum a b instead of sum a log b
  double* partials;   // 3 per block, 256 blocks
  double* out;
};
hipError_t launch_readout(const ReadoutArgs& a, hipStream_t st);

// Log-domain weights of a sorted cloud, one workgroup per chunk:
//   out[q] = exp((pot[q] - shift[prob]) / eps_prob), prob = chunks[blockIdx].prob,
// in [0, 1] when shift is the problem's largest potential (-inf gives 0).
// Chunks of problems in state 2 of pstate (nullable) are skipped.
hipError_t launch_logweights(const Chunk* chunks, int nchunks, const double* pot, const double* shift,
                             const double* leps, double* out, const int* pstate, hipStream_t st);

// out[i] = a[i] * b[i], i < n.
hipError_t launch_mul(const double* a, const double* b, long n, double* out, hipStream_t st);

// out[0] = max v, out[1] = sum v (non-finite if any entry is), over n values.
hipError_t launch_maxsum(const double* v, long n, double* partials, double* out, hipStream_t st);

// grad_mu: out[i] = eps*log(alpha[i]) - shift (out[perm[i]] with perm), with shift = eps*mean(log alpha)
// over the n entries (zero scalings count as log 0 = 0: weight zero, see Proposition 2.3)
hipError_t launch_gradmu(const double* alpha, long n, double eps, double* partials,
                         double* mean_out, double* grad_mu, hipStream_t st, const int* perm = nullptr);

// NFFT spectrum conversion between user layout (full I_N, complex FP64) and
// the internal half spectrum (R), with deconvolution by 1/Phi.
template <typename R>
struct SpecArgs {
  int d, N;
  const cplx<R>* spec_in;  // internal -> user
  cplx<R>* spec_out;       // user -> internal
  const double* user_in;
  double* user_out;
  const double* inv_phi;   // N/2+1 entries: 1/Phi(|k|)
  double scale;            // internal -> user: factor applied to the output
};
template <typename R>
hipError_t launch_spec_to_user(const SpecArgs<R>& a, hipStream_t st);
template <typename R>
hipError_t launch_user_to_spec(const SpecArgs<R>& a, hipStream_t st);

}  // namespace nfs
