/*
 * nfs.h - C ABI of the MI355X (gfx950) NFFT-boosted Sinkhorn library.
 *
 * The library solves the entropy-regularized optimal transport problem between
 * two discrete measures P = sum_i p_i delta_{x_i} and Pt = sum_j pt_j delta_{y_j}
 * on R^d (Definition 2.2, eqs. (Sinkhorn), (SD1)-(SD2)) with Sinkhorn's scaling
 * iteration (Algorithm 1), where both Gibbs-kernel products
 *
 *     t_i  = sum_j alpha_t_j exp(-|x_i - y_j|^r / eps)      (eq. (matexp))
 *     tt_j = sum_i alpha_i   exp(-|x_i - y_j|^r / eps)      (eq. (matexpt))
 *
 * are evaluated by NFFT fast summation (Section 3.1, eq. (fastsum)), i.e. the
 * NFFT-accelerated Sinkhorn algorithm (Algorithm 3).
 *
 * Notation: the paper writes the kernel as exp(-lambda d^r).  This ABI uses the
 * temperature eps = 1/lambda, so K = exp(-c/eps).
 *
 * Conventions shared by every entry point
 *   - Arrays named as points, weights, scalings and outputs are DEVICE
 *     pointers, caller-owned, contiguous, FP64.  Points are point-major:
 *     x[i*d + c].
 *   - `workspace` is a caller-allocated device buffer of at least the size
 *     that nfs_workspace_size() reports for the same call; the library
 *     allocates no device memory itself.  Its contents on entry are ignored
 *     and on return are unspecified.
 *   - All device work is ordered on `stream` (a hipStream_t, 0 = the null
 *     stream).  Calls return after the plan stage has synchronized `stream`
 *     once; entry points that return host scalars synchronize it again at
 *     the end.  Device outputs are complete when the call returns.
 *   - Return value 0 (NFS_OK) on success, otherwise one of the NFS_E* codes;
 *     nfs_last_error() then gives a message (thread-local).  Outputs are
 *     undefined on error.  No exception crosses the ABI.
 *   - Calls on distinct workspaces may run concurrently on distinct streams.
 */
#ifndef NFS_H
#define NFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define NFS_OK 0
#define NFS_EINVAL 1        /* bad d, r, N, m, sigma, eps, size, null pointer */
#define NFS_EWEIGHTS 2      /* negative weight or |sum - 1| > 1e-12 * max(n, nt) */
#define NFS_ENONPOS 3       /* a kernel sum t <= 0 or non-finite during the solve */
#define NFS_EUNSUPPORTED 4  /* option outside what the library implements */
#define NFS_EHIP 5          /* HIP runtime error */
#define NFS_EWORKSPACE 6    /* workspace smaller than nfs_workspace_size() */

/* Grid / FFT / window precision.  Scalings and reductions are always FP64.
 * NFS_AUTO is accepted by the solve calls only (nfs_sinkhorn_solve,
 * nfs_batch_solve, and the workspace sizes for them): the problem is solved
 * with FP32 grids, and every problem whose solve met a kernel sum t <= 0 or a
 * non-finite one (the FP32 dynamic-range floor of fast summation) is solved
 * again from its starting value with FP64 grids.  nfs_result.precision_used
 * reports the grid precision of the returned result. */
#define NFS_FP64 0
#define NFS_FP32 1
#define NFS_AUTO 2

/* flags */
#define NFS_FLAG_NO_GRAPH 1      /* launch the iteration kernels directly, no hipGraph replay */
#define NFS_FLAG_PRIMAL_COST 2   /* also evaluate <pi, C> (one extra fast summation with the
                                    kernel c K; for r = 1 and real exponents its table comes
                                    from samples of its own regularized form at plan time, and
                                    the extra sum has its own near field) */
#define NFS_FLAG_TILE_REDUCE 4   /* spread: store each chunk's LDS tile and sum the tiles per
                                    (tile, neighbour) instead of flushing LDS tiles straight
                                    into the grid with global atomics (the default) */
#define NFS_FLAG_AUTOTUNE 16     /* solver handles (and the solves built on them), r = 2 only: the
                                    spreading tile and bin sizes by measurement.  With tile = 0,
                                    plan and time a warm-up and three iterations at half, one and
                                    two times the default tile (those whose LDS tile fits) and keep
                                    the fastest; then time a few iterations at each candidate chunk
                                    size (the points a workgroup takes: the default, twice it, 4096,
                                    8192) and keep the fastest.  The starting values are restored
                                    before the first iteration; nfs_workspace_size() covers every
                                    candidate tile */
#define NFS_FLAG_CENTER 32       /* solve calls, r = 2: the centred form.  For the squared cost,
                                    |x - y|^2 = |x' - y'|^2 - 2 delta.(x' - y') + |delta|^2 with
                                    x' = x + delta/2, y' = y - delta/2 and delta = mean_nu y -
                                    mean_mu x; the middle term is separable, so the coupling of the
                                    shifted clouds (equal weighted means) is the same and the
                                    scalings differ by factors exp(-/+2 delta.x'/eps).  The
                                    iteration runs on the shifted clouds from alpha_t' = 1, where
                                    the scalings (hence the sums the fast summation must resolve)
                                    have far less dynamic range when the clouds are apart; the
                                    result is mapped back: cost + |delta|^2, scalings times those
                                    factors (potentials plus eps times their logs).  Starting from
                                    alpha_t' = 1 is Algorithm 3 from alpha_t = exp((2 delta.y' +
                                    |delta|^2/2)/eps).  No warm start, no primal cost (NaN) */
#define NFS_FLAG_LOG_DOMAIN 8    /* solve in potentials (Algorithm 4): the alpha / alpha_t arguments
                                    of the solve, batch and solver calls hold beta / gamma instead,
                                    with alpha = exp(beta/eps - 1/2), alpha_t = exp(gamma/eps - 1/2);
                                    NFS_FLAG_PRIMAL_COST is ignored (cost_primal = NaN) */

typedef struct nfs_params {
  int32_t d;          /* dimension, 1..3 */
  int32_t r;          /* cost exponent: 2 -> c = |x-y|^2; 1 -> c = |x-y| (near-field corrected,
                         Remark 3.2); 0 -> the real exponent rexp */
  double eps;         /* temperature > 0; K = exp(-c/eps) (the paper's 1/lambda) */
  int32_t N;          /* bandwidth per dimension: I_N = {-N/2..N/2-1}^d, even, >= 4 */
  int32_t m;          /* window cutoff: 2m+1 grid taps per dimension, 2 <= m <= 8 */
  double sigma;       /* oversampling: grid g = sigma*N rounded up to a power of two, g >= N + 2 */
  int32_t precision;  /* NFS_FP64, NFS_FP32, or NFS_AUTO (solve calls only) */
  int32_t tile;       /* grid cells per bin side (0 = default for d) */
  int32_t chunk;      /* max points per workgroup chunk, 0..32768 (0 = default: for r = 2, 1536
                         (FP32, d = 2) or 4096 (FP32, d = 3), 4096 for clouds with more than 8
                         points per grid cell and n >= 200 * 4096; else 1024) */
  int32_t flags;      /* NFS_FLAG_* */
  double eps_I;       /* r = 0, 1: near-field radius times N on the period-1 torus (0 = default 4);
                         the radius must fit in 2 kt + 1 tiles, kt = ceil(eps_I sigma / tile) */
  int32_t p_smooth;   /* r = 0, 1: derivatives matched by the inner polynomial (0 = default 8, max 16) */
  int32_t reserved;
  double rexp;        /* r = 0: real cost exponent in (1, 4], not 2: c = |x-y|^rexp (Definition 2.1
                         with real r).  Treated as r = 1 is: the kernel exp(-|z|^rexp/eps) is
                         replaced inside |z| < eps_I by the even polynomial matching its first
                         p_smooth - 1 derivatives at eps_I (Section 3.1), the Fourier
                         coefficients of the regularized kernel come from its samples on the
                         oversampled grid, and the near field adds K - K_R.  The gradients
                         use grad c = rexp |x-y|^(rexp-2) (x-y).  Ignored
                         unless r = 0 */
} nfs_params;

typedef struct nfs_result {
  double cost;          /* s_{r;lambda;NFFT} (Algorithm 3 result) */
  double cost_upper;    /* cost + eps*(H(P) + H(Pt)) (Section 3.2) */
  double cost_primal;   /* <pi, C> = sum alpha_i K_ij c_ij alpha_t_j, if NFS_FLAG_PRIMAL_COST */
  double marg_err;      /* ||E|| of eq. (Error) after the last iteration (row + column) */
  double marg_err_row;  /* ||alpha o (K alpha_t) - p||_2 (one extra kernel product) */
  double marg_err_col;  /* ||alpha_t o (K^T alpha) - pt||_2 */
  double scale;         /* s: points were mapped to the torus as s*(x - center) */
  double kernel_err;    /* a-priori bound on the kernel approximation (periodization/truncation) */
  int32_t iters;        /* iterations done (one = alpha update then alpha_t update) */
  int32_t precision_used;
  int64_t n_nonpos;     /* number of kernel sums t <= 0 or non-finite seen */
  double dyn_range;     /* largest ratio ||w||_1 / min_i t_i over the solve's half-steps, w the
                           source weights of the sums t (Algorithm 3 only; NaN in the log
                           domain, infinite once a sum t <= 0 was seen): the dynamic range
                           the fast sums had to resolve, as their error is normwise in
                           ||w||_1 */
  int32_t centred;      /* 1 if the result comes from the centred form (NFS_FLAG_CENTER) */
  int32_t reserved;
} nfs_result;

/* Message for the last error on this thread ("" if none). */
const char* nfs_last_error(void);

/* CPU-only argument check of params and sizes (no device access). */
int nfs_validate(const nfs_params* prm, int64_t n, int64_t nt);

/* Workspace bytes needed by fastsum_apply / sinkhorn_solve / sinkhorn_grad for
 * clouds of n sources and nt targets (or n x-points and nt y-points). */
int nfs_workspace_size(const nfs_params* prm, int64_t n, int64_t nt, size_t* bytes);

/*
 * Fast summation (Section 3.1, eq. (fastsum)):
 *   out_i = sum_j w_j exp(-|tgt_i - src_j|^r / eps),  i < nt.
 * src: ns x d, w: ns (any sign), tgt: nt x d, out: nt.  ns, nt >= 1.
 */
int nfs_fastsum_apply(const nfs_params* prm, const double* src, int64_t ns, const double* w,
                      const double* tgt, int64_t nt, double* out,
                      void* workspace, size_t ws_bytes, void* stream);

/*
 * Allocation-free variant of nfs_fastsum_apply, for callers that cannot
 * allocate device memory or pass a workspace: code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * result, layout and errors as nfs_fastsum_apply, without the workspace: its
 * scratch is a static device array of NFS_NOALLOC_SCRATCH_BYTES bytes that the
 * library holds on every GPU it runs on until the process ends.  The call
 * allocates no device memory (no hipMalloc/hipFree, no allocating library
 * call).  A problem whose scratch need exceeds the limit (the need is at
 * most what nfs_workspace_size() reports for the same sizes, e.g. about
 * 24 MiB for 1e5 + 1e5 points at d = 2, N = 512, FP32) returns
 * NFS_EWORKSPACE before any device work.  Every call on one GPU shares that
 * GPU's array: calls that overlap in time on one GPU (from several host
 * threads or on several streams) race and give undefined results; calls on
 * one stream, or on different GPUs, do not.
 */
#define NFS_NOALLOC_SCRATCH_BYTES (64u << 20)
int nfs_fastsum_apply_noalloc(const nfs_params* prm, const double* src, int64_t ns, const double* w,
                              const double* tgt, int64_t nt, double* out, void* stream);

/*
 * Adjoint NFFT, the inner sum of eq. (fastsum) for real weights, on the
 * period-1 torus: fhat_k = sum_j w_j exp(-2 pi i k.y_j), k in I_N.
 * pts: n x d with every coordinate in [-1/2, 1/2); fhat: N^d complex values,
 * interleaved (re, im), row-major with index (k_0 + N/2, ..., k_{d-1} + N/2).
 */
int nfs_nfft_adjoint(const nfs_params* prm, const double* pts, int64_t n, const double* w,
                     double* fhat, void* workspace, size_t ws_bytes, void* stream);

/*
 * NFFT, the outer sum of eq. (fastsum): out_i = Re sum_{k in I_N} fhat_k exp(2 pi i k.x_i).
 * fhat layout as in nfs_nfft_adjoint; pts in [-1/2, 1/2)^d; out: n reals.
 */
int nfs_nfft_trafo(const nfs_params* prm, const double* fhat, const double* pts, int64_t n,
                   double* out, void* workspace, size_t ws_bytes, void* stream);

/*
 * NFFT-accelerated Sinkhorn (Algorithm 3).  x: n x d with weights mu (sum 1,
 * >= 0); y: nt x d with weights nu.  Runs max_iter iterations (alpha update,
 * then alpha_t update, eq. (S1)); if tol > 0 it stops early once ||E|| <= tol,
 * checked every 10 iterations with one extra kernel product.
 *   alpha   (n):  out, final scalings alpha.
 *   alpha_t (nt): in = starting value when warm_start != 0 (else ones), out = final alpha_t.
 *   res: host pointer, filled on success.
 */
int nfs_sinkhorn_solve(const nfs_params* prm, const double* x, int64_t n, const double* mu,
                       const double* y, int64_t nt, const double* nu,
                       int32_t max_iter, double tol, int32_t warm_start,
                       double* alpha, double* alpha_t, nfs_result* res,
                       void* workspace, size_t ws_bytes, void* stream);

/*
 * NFFT-accelerated log-domain Sinkhorn (Algorithm 4): the same iteration in
 * the dual potentials, which stay finite where the scalings over- or
 * underflow.  Equals nfs_sinkhorn_solve with NFS_FLAG_LOG_DOMAIN set.
 * Potentials enter the fast sums as exp(gamma_j/eps - 1/2) and the update is
 * beta_i = eps (log mu_i - log t_i) + eps/2.  The printed update lacks the
 * eps/2; with it the iterates are those of Algorithm 3, and the Algorithm 4
 * result s = sum mu beta + sum nu gamma - eps sum_j t_j exp(gamma_j/eps - 1/2)
 * equals the Algorithm 3 result.  Each half-step spreads exp((gamma - max
 * gamma)/eps) in [0, 1] and returns max beta for the next one.
 *   beta  (n):  out, final potentials beta (-inf where mu_i = 0).
 *   gamma (nt): in = starting value when warm_start != 0 (finite; else
 *               zeros, as in the paper), out = final gamma.
 *   res: as nfs_sinkhorn_solve, with cost the Algorithm 4 result; cost_primal
 *        is NaN.
 * Same workspace size, precision (NFS_AUTO included) and errors as
 * nfs_sinkhorn_solve; NFS_EINVAL for a non-finite gamma start.
 */
int nfs_sinkhorn_solve_log(const nfs_params* prm, const double* x, int64_t n, const double* mu,
                           const double* y, int64_t nt, const double* nu,
                           int32_t max_iter, double tol, int32_t warm_start,
                           double* beta, double* gamma, nfs_result* res,
                           void* workspace, size_t ws_bytes, void* stream);

/*
 * Persistent solver handle for the same iteration (Algorithm 3): the plan
 * (torus scaling, binning, coefficient tables) is done once by create, which
 * also records one iteration in a hipGraph on an internal stream; iterate
 * replays it.  Device work of every call is ordered after earlier work on
 * `stream`, and later work on `stream` waits for it.  The handle keeps
 * pointers into `workspace`, which must stay allocated and untouched until
 * destroy.  alpha_t0 (nullable, nt) is the starting value of alpha_t.
 */
typedef struct nfs_solver nfs_solver;
int nfs_solver_create(const nfs_params* prm, const double* x, int64_t n, const double* mu,
                      const double* y, int64_t nt, const double* nu, const double* alpha_t0,
                      void* workspace, size_t ws_bytes, void* stream, nfs_solver** out);
/* Runs `iters` more iterations (alpha update, then alpha_t update). */
int nfs_solver_iterate(nfs_solver* s, int32_t iters, void* stream);
/* Row residual ||alpha o (K alpha_t) - p||_2 of the current state (one extra
 * kernel product); synchronizes and writes the host scalar *err_row. */
int nfs_solver_residual(nfs_solver* s, double* err_row, void* stream);
/* Read-out: final scalings in the caller's point order (either may be NULL)
 * and the result struct, as nfs_sinkhorn_solve.  The solver stays usable. */
int nfs_solver_finish(nfs_solver* s, double* alpha, double* alpha_t, nfs_result* res, void* stream);
/* Runs `iters` iterations with direct launches and events between kernels;
 * stage_ms[5] receives the average device time per launch of spreading, of
 * the FFT chain, of interpolation with the scaling update, of one whole
 * iteration, and of the near-field sum (r = 1; about 0 for r = 2).  info (nullable, 9 doubles): n, nt, d, grid cells, bytes per grid
 * value, chunks of x, chunks of y, taps per point, tile size T. */
int nfs_solver_profile(nfs_solver* s, int32_t iters, double* stage_ms, double* info, void* stream);
/* Envelope gradient of the cost at the solver's current scalings (as
 * nfs_sinkhorn_grad and nfs_sinkhorn_grad_targets; Proposition 2.3, eq. (14)),
 * on the solver's own plan: no re-sort, no new tables.  grad_x (n x d),
 * grad_mu (n), grad_y (nt x d), grad_nu (nt), in the caller's point order
 * (for a batch solver, packed by problem, each problem's weight gradient
 * centred over that problem); any may be NULL.  The log domain and the
 * centred form return NFS_EUNSUPPORTED.  The scalings are not
 * changed, so iterate may continue afterwards. */
int nfs_solver_grad(nfs_solver* s, double* grad_x, double* grad_mu, double* grad_y, double* grad_nu, void* stream);
int nfs_solver_destroy(nfs_solver* s);

/*
 * Batched form (the project's own): nprob independent problems that share d,
 * r, N, m, sigma, precision, tile and chunk (prm->eps is ignored; eps[b] is
 * problem b's temperature).  Points and weights are packed in problem order:
 * problem b's x points are rows [sum_{c<b} n[c], sum_{c<=b} n[c]) of x (and
 * of mu and alpha), likewise y, nu, alpha_t with nt.  n, nt, eps: host arrays.
 * Every stage of an iteration is one kernel launch over all problems and one
 * iteration of all problems is captured in one hipGraph.  res: host array of
 * nprob results.  A solver made by nfs_batch_solver_create is driven with the
 * nfs_solver_* calls above (nfs_solver_finish then fills nprob results and
 * nfs_solver_residual returns the largest residual over the problems).
 */
int nfs_batch_workspace_size(const nfs_params* prm, int32_t nprob, const int64_t* n, const int64_t* nt,
                             size_t* bytes);
int nfs_batch_solver_create(const nfs_params* prm, int32_t nprob, const int64_t* n, const int64_t* nt,
                            const double* eps, const double* x, const double* mu, const double* y,
                            const double* nu, const double* alpha_t0, void* workspace, size_t ws_bytes,
                            void* stream, nfs_solver** out);
int nfs_batch_solve(const nfs_params* prm, int32_t nprob, const int64_t* n, const int64_t* nt,
                    const double* eps, const double* x, const double* mu, const double* y,
                    const double* nu, int32_t max_iter, double tol, double* alpha, double* alpha_t,
                    nfs_result* res, void* workspace, size_t ws_bytes, void* stream);

/*
 * Sinkhorn divergence (Remark on entropy bias and Sinkhorn divergence,
 * Section 2.2; its NFFT form in Section 3.2):
 *   sd = s(P, Pt) - s(P, P)/2 - s(Pt, Pt)/2,
 * each s the Algorithm 3 result after max_iter iterations from the default
 * start (tol > 0: stop early per problem as in nfs_sinkhorn_solve).  The three
 * problems run as one batch (batched form) from inputs packed into the
 * workspace; prm->precision may be NFS_AUTO.  *sd: host scalar.  res
 * (nullable, host array of 3): results of (P, Pt), (P, P), (Pt, Pt).  Returns
 * NFS_ENONPOS (with *sd set) when a kernel sum t <= 0 remains.
 */
int nfs_divergence_workspace_size(const nfs_params* prm, int64_t n, int64_t nt, size_t* bytes);
int nfs_sinkhorn_divergence(const nfs_params* prm, const double* x, int64_t n, const double* mu,
                            const double* y, int64_t nt, const double* nu, int32_t max_iter, double tol,
                            double* sd, nfs_result* res, void* workspace, size_t ws_bytes, void* stream);

/*
 * Gradient of the Sinkhorn cost at given scalings (alpha, alpha_t), by the
 * envelope theorem applied to the dual (Proposition 2.3, eq. (14)):
 *   grad_x[i]  = sum_j pi_ij grad_x c(x_i, y_j) = -eps alpha_i (grad K * alpha_t)(x_i)   (n x d)
 *   grad_mu[i] = eps log alpha_i - mean_k(eps log alpha_k)                               (n)
 * with the kernel gradient summed by fast summation (coefficients 2 pi i k b_k
 * of the regularized kernel); for r = 1 (grad_x c = (x - y)/|x - y|, zero
 * where points coincide) and a real exponent rexp (grad_x c = rexp |x - y|^(rexp-2)
 * (x - y)) the gradient of the near-field correction K - K_R is added by
 * direct sums over the pairs closer than eps_I.  Either output may be NULL.
 */
int nfs_sinkhorn_grad(const nfs_params* prm, const double* x, int64_t n, const double* mu,
                      const double* y, int64_t nt, const double* nu,
                      const double* alpha, const double* alpha_t,
                      double* grad_x, double* grad_mu,
                      void* workspace, size_t ws_bytes, void* stream);

/*
 * Target side of the same gradient (the kernel is even, so this is the
 * computation above with the roles of the two clouds exchanged):
 *   grad_y[j]  = sum_i pi_ij grad_y c(x_i, y_j) = -eps alpha_t_j (grad K * alpha)(y_j)   (nt x d)
 *   grad_nu[j] = eps log alpha_t_j - mean_k(eps log alpha_t_k)                            (nt)
 * Same arguments, workspace size and errors as nfs_sinkhorn_grad.  Either
 * output may be NULL.
 */
int nfs_sinkhorn_grad_targets(const nfs_params* prm, const double* x, int64_t n, const double* mu,
                              const double* y, int64_t nt, const double* nu,
                              const double* alpha, const double* alpha_t,
                              double* grad_y, double* grad_nu,
                              void* workspace, size_t ws_bytes, void* stream);

/*
 * Product of the coupling pi = diag(alpha) K diag(alpha_t) (eq. (pi*)) with a
 * vector, by one fast summation, without forming pi (the product the paper's
 * remark on the optimal transition matrix leaves out):
 *   transpose = 0: v (nt) -> out (n),  out = alpha o K (alpha_t o v);
 *   transpose = 1: v (n)  -> out (nt), out = alpha_t o K^T (alpha o v).
 * alpha, alpha_t: scalings as returned by nfs_sinkhorn_solve (not potentials).
 * Workspace: nfs_workspace_size(prm, n, nt).  NFS_EINVAL for a NULL pointer or
 * transpose not in {0, 1}.  r = 1 includes the near field.
 */
int nfs_plan_apply(const nfs_params* prm, const double* x, int64_t n, const double* y, int64_t nt,
                   const double* alpha, const double* alpha_t, const double* v, int32_t transpose,
                   double* out, void* workspace, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NFS_H */
