"""Dense FP64 Sinkhorn (Algorithm 1) with the read-outs of Algorithm 3.

Test infrastructure only (see ``oracle/__init__.py``).

Notation.  The paper writes the Gibbs kernel as k = exp(-lambda d^r) with a
large lambda meaning weak regularization.  Here ``eps`` is the temperature,
eps = 1/lambda, so k = exp(-c/eps) with c = |x - y|^r.  Every formula below is
the paper's with 1/lambda replaced by eps.
"""
import numpy as np


def cost_matrix(x, y, r):
    """c_ij = ||x_i - y_j||^r with the Euclidean norm (Definition 2.1, eq. (dist))."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    if y.ndim == 1:
        y = y[:, None]
    diff = x[:, None, :] - y[None, :, :]
    dist = np.sqrt(np.sum(diff * diff, axis=-1))
    return dist ** r


def gibbs_kernel(x, y, r, eps):
    """k_ij = exp(-c_ij / eps) (Section 2.2, the Gibbs kernel k = exp(-lambda d^r))."""
    return np.exp(-cost_matrix(x, y, r) / eps)


def xlogy(a, b):
    """a*log(b) with the convention 0*log(0) = 0 used for zero weights."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.zeros(np.broadcast(a, b).shape)
    nz = a != 0
    out[nz] = a[nz] * np.log(b[nz])
    return out


def entropy(p):
    """H(P) = -sum p_i log p_i (Lemma 2.1)."""
    return -float(np.sum(xlogy(p, p)))


def kl(a, b):
    """Kullback-Leibler divergence sum a_i log(a_i/b_i) (Section 2, Notations)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nz = a > 0
    return float(np.sum(a[nz] * np.log(a[nz] / b[nz])))


def dual_value(K, alpha, alpha_t, p, pt, eps):
    """Dual function of Proposition 2.3, eq. (14), with 1/lambda = eps.

    d = eps + eps*sum p log alpha + eps*sum pt log alpha_t - eps*alpha^T K alpha_t.
    """
    return (eps + eps * float(np.sum(xlogy(p, alpha)))
            + eps * float(np.sum(xlogy(pt, alpha_t)))
            - eps * float(alpha @ (K @ alpha_t)))


def _safe_div(num, den):
    out = np.zeros_like(num)
    nz = num != 0
    out[nz] = num[nz] / den[nz]
    return out


def sinkhorn(K, p, pt, iters, alpha_t0=None, eps=None, record=False):
    """Algorithm 1 (Sinkhorn's algorithm) for a fixed number of iterations.

    One iteration is the odd half-step (update alpha from alpha_t, eq. (S1)
    left) followed by the even half-step (update alpha_t from alpha, eq. (S1)
    right, with the target weights pt).  Both scalings start at one
    (eq. (MatrixK_sin_div)); ``alpha_t0`` replaces the starting alpha_t (the
    algorithm's "starting value" input, used for warm restarts).  A point of
    weight zero gets scaling zero.

    Returns a dict with the final scalings, the last products t = K alpha_t and
    tt = K^T alpha that produced them, and, when ``record`` is set and ``eps``
    given, the dual value and the Kullback-Leibler term of every half-step
    (Lemma 2.4).
    """
    K = np.asarray(K, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    pt = np.asarray(pt, dtype=np.float64)
    n, nt = K.shape
    alpha = np.ones(n)
    alpha_t = np.ones(nt) if alpha_t0 is None else np.array(alpha_t0, dtype=np.float64)
    hist = []
    t = tt = None
    for _ in range(iters):
        # odd half-step: row sums of pi = diag(alpha) K diag(alpha_t) before the update
        t = K @ alpha_t
        if record:
            hist.append(dict(kind="row", kl=kl(p, alpha * t),
                             dual_before=dual_value(K, alpha, alpha_t, p, pt, eps)))
        alpha = _safe_div(p, t)
        if record:
            hist[-1]["dual_after"] = dual_value(K, alpha, alpha_t, p, pt, eps)
        # even half-step: column sums before the update
        tt = K.T @ alpha
        if record:
            hist.append(dict(kind="col", kl=kl(pt, alpha_t * tt),
                             dual_before=dual_value(K, alpha, alpha_t, p, pt, eps)))
        alpha_t = _safe_div(pt, tt)
        if record:
            hist[-1]["dual_after"] = dual_value(K, alpha, alpha_t, p, pt, eps)
    return dict(alpha=alpha, alpha_t=alpha_t, t=t, tt=tt, hist=hist)


def sinkhorn_to_tolerance(K, p, pt, tol, max_iter=100000):
    """Algorithm 1 with its stopping rule ||E|| <= tol (eq. (Error)).

    After each full iteration the column residual is zero, so ||E|| is the row
    residual ||alpha o (K alpha_t) - p||.
    """
    alpha = np.ones(K.shape[0])
    alpha_t = np.ones(K.shape[1])
    for it in range(1, max_iter + 1):
        alpha = _safe_div(p, K @ alpha_t)
        tt = K.T @ alpha
        alpha_t = _safe_div(pt, tt)
        err = float(np.linalg.norm(alpha * (K @ alpha_t) - p))
        if err <= tol:
            return dict(alpha=alpha, alpha_t=alpha_t, tt=tt, iters=it, err=err)
    return dict(alpha=alpha, alpha_t=alpha_t, tt=tt, iters=max_iter, err=err)


def cost_readout(alpha, alpha_t, tt, p, pt, eps):
    """Result of Algorithm 3: s = eps + eps*sum p log alpha + eps*sum pt log alpha_t
    - eps*sum_j tt_j alpha_t_j, with tt the last product K^T alpha."""
    return (eps + eps * float(np.sum(xlogy(p, alpha)))
            + eps * float(np.sum(xlogy(pt, alpha_t)))
            - eps * float(np.sum(tt * alpha_t)))


def cost_upper_bound(s, p, pt, eps):
    """Upper ERW value of Section 3.2: s + (H(P) + H(Pt))/lambda."""
    return s + eps * (entropy(p) + entropy(pt))


def primal_cost(K, C, alpha, alpha_t):
    """<pi, C> = sum_ij alpha_i k_ij c_ij alpha_t_j (eq. (15) with pi of eq. (pi*))."""
    return float(alpha @ ((K * C) @ alpha_t))


def marginal_errors(K, alpha, alpha_t, p, pt):
    """Both terms of the residual of eq. (Error), Euclidean norm."""
    pi_row = alpha * (K @ alpha_t)
    pi_col = alpha_t * (K.T @ alpha)
    return float(np.linalg.norm(pi_row - p)), float(np.linalg.norm(pi_col - pt))


def transport_plan(K, alpha, alpha_t):
    """pi = diag(alpha) k diag(alpha_t) (eq. (pi*)); dense, small problems only."""
    return alpha[:, None] * K * alpha_t[None, :]


def envelope_gradient(x, y, K, alpha, alpha_t, r, eps):
    """Gradient of s with respect to the source positions and weights.

    Differentiating the dual (eq. (14)) at fixed scalings (envelope theorem):
      d s / d x_i  = sum_j pi_ij grad_x c(x_i, y_j),
      d s / d p_i  = eps log alpha_i, projected onto sum = 0 (the weights live
                     on the probability simplex).
    For r = 2, grad_x c = 2 (x_i - y_j); for r = 1 it is the unit vector
    (x_i - y_j)/|x_i - y_j| (zero where the points coincide); for a real
    r > 1, r |x_i - y_j|^(r - 2) (x_i - y_j) (zero where they coincide).
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    if y.ndim == 1:
        y = y[:, None]
    pi = transport_plan(K, alpha, alpha_t)
    diff = x[:, None, :] - y[None, :, :]
    if r == 2:
        g = 2.0 * diff
    elif r == 1:
        nrm = np.sqrt(np.sum(diff * diff, axis=-1, keepdims=True))
        g = np.where(nrm > 0, diff / np.where(nrm > 0, nrm, 1.0), 0.0)
    elif r > 1:
        nrm = np.sqrt(np.sum(diff * diff, axis=-1, keepdims=True))
        g = np.where(nrm > 0, r * np.where(nrm > 0, nrm, 1.0) ** (r - 2) * diff, 0.0)
    else:
        raise ValueError("r must be 1, 2 or a real exponent above 1")
    grad_x = np.einsum("ij,ijc->ic", pi, g)
    gmu = eps * np.where(alpha > 0, np.log(np.where(alpha > 0, alpha, 1.0)), 0.0)
    grad_mu = gmu - gmu.mean()
    return grad_x, grad_mu


def envelope_gradient_targets(x, y, K, alpha, alpha_t, r, eps):
    """Gradient of s with respect to the target positions and weights, by the
    same envelope argument on eq. (14):
      d s / d y_j  = sum_i pi_ij grad_y c(x_i, y_j),
      d s / d pt_j = eps log alpha_t_j, projected onto sum = 0.
    For r = 2, grad_y c = 2 (y_j - x_i); for r = 1, (y_j - x_i)/|y_j - x_i|;
    for a real r > 1, r |y_j - x_i|^(r - 2) (y_j - x_i).
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    if y.ndim == 1:
        y = y[:, None]
    pi = transport_plan(K, alpha, alpha_t)
    diff = y[None, :, :] - x[:, None, :]
    if r == 2:
        g = 2.0 * diff
    elif r == 1:
        nrm = np.sqrt(np.sum(diff * diff, axis=-1, keepdims=True))
        g = np.where(nrm > 0, diff / np.where(nrm > 0, nrm, 1.0), 0.0)
    elif r > 1:
        nrm = np.sqrt(np.sum(diff * diff, axis=-1, keepdims=True))
        g = np.where(nrm > 0, r * np.where(nrm > 0, nrm, 1.0) ** (r - 2) * diff, 0.0)
    else:
        raise ValueError("r must be 1, 2 or a real exponent above 1")
    grad_y = np.einsum("ij,ijc->jc", pi, g)
    gnu = eps * np.where(alpha_t > 0, np.log(np.where(alpha_t > 0, alpha_t, 1.0)), 0.0)
    grad_nu = gnu - gnu.mean()
    return grad_y, grad_nu


def plan_apply(K, alpha, alpha_t, v, transpose=False):
    """Product of the coupling pi = diag(alpha) k diag(alpha_t) (eq. (pi*))
    with a vector: pi v (n values), or pi^T v (nt values) when ``transpose``."""
    pi = transport_plan(K, alpha, alpha_t)
    return pi.T @ v if transpose else pi @ v


def solve(x, p, y, pt, r, eps, iters, alpha_t0=None):
    """Convenience wrapper: Algorithm 1 for ``iters`` iterations plus every read-out.

    Returns the scalings, the cost s (Algorithm 3 result), the upper value,
    the primal cost <pi, C>, and the residual of eq. (Error) after the last
    iteration (the row term needs one extra product K alpha_t).
    """
    C = cost_matrix(x, y, r)
    K = np.exp(-C / eps)
    out = sinkhorn(K, p, pt, iters, alpha_t0=alpha_t0)
    a, at, tt = out["alpha"], out["alpha_t"], out["tt"]
    s = cost_readout(a, at, tt, p, pt, eps)
    e_row, e_col = marginal_errors(K, a, at, p, pt)
    return dict(alpha=a, alpha_t=at, tt=tt, cost=s,
                cost_upper=cost_upper_bound(s, p, pt, eps),
                cost_primal=primal_cost(K, C, a, at),
                marg_err=e_row + e_col, marg_err_row=e_row, marg_err_col=e_col)


def sinkhorn_divergence(x, p, y, pt, r, eps, iters):
    """Sinkhorn divergence sd(P, Pt) = s(P, Pt) - s(P, P)/2 - s(Pt, Pt)/2
    (Remark on entropy bias and Sinkhorn divergence, Section 2.2; its NFFT form
    in Section 3.2), each s the Algorithm 3 result after ``iters`` iterations
    of Algorithm 1 from the default start.  Returns sd and the three costs."""
    s_xy = solve(x, p, y, pt, r, eps, iters)["cost"]
    s_xx = solve(x, p, x, p, r, eps, iters)["cost"]
    s_yy = solve(y, pt, y, pt, r, eps, iters)["cost"]
    return dict(sd=s_xy - 0.5 * s_xx - 0.5 * s_yy, cost_xy=s_xy, cost_xx=s_xx, cost_yy=s_yy)


# ---------------------------------------------------------------------------
# Log-domain Sinkhorn (Algorithm 2, dense; Algorithm 4 computes the same sums
# by fast summation).
#
# Reading.  Both algorithms enter the potentials into the sums through
# exp(gamma_j/eps - 1/2) and exp(beta_i/eps - 1/2), and their result is the
# dual of eq. (14) in potentials,
#   s = sum p beta + sum pt gamma - eps sum_ij exp((beta_i + gamma_j - c_ij)/eps - 1).
# That dual is maximized over beta_i exactly when
#   exp(beta_i/eps - 1/2) sum_j k_ij exp(gamma_j/eps - 1/2) = p_i,
# i.e. beta_i = eps (log p_i - log t_i) + eps/2.  The printed updates omit the
# eps/2; with it, alpha = exp(beta/eps - 1/2) and alpha_t = exp(gamma/eps - 1/2)
# are exactly the scalings of Algorithm 1 and the printed result equals the
# Algorithm 3 result.  Without it, the iterates reach a plan of mass e^{-1/2}
# and the result formula is off by a multiple of eps.
# ---------------------------------------------------------------------------
def _logsumexp(z, axis):
    """log sum exp(z) along ``axis``, shifted by the maximum (the log-sum-exp
    step the log-domain algorithm relies on); -inf where every entry is -inf."""
    m = np.max(z, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        return np.squeeze(m, axis=axis) + np.log(np.sum(np.exp(z - m), axis=axis))


def _log_or_neg_inf(p):
    with np.errstate(divide="ignore"):
        return np.where(p > 0, np.log(np.where(p > 0, p, 1.0)), -np.inf)


def log_dual_value(C, beta, gamma, p, pt, eps):
    """Dual of eq. (14) in potentials (the result of Algorithm 2):
    sum p beta + sum pt gamma - eps sum_ij exp((beta_i + gamma_j - c_ij)/eps - 1)."""
    z = (beta[:, None] + gamma[None, :] - C) / eps - 1.0
    mass = float(np.exp(_logsumexp(z.ravel(), axis=0)))
    return (float(np.sum(p[p > 0] * beta[p > 0])) + float(np.sum(pt[pt > 0] * gamma[pt > 0]))
            - eps * mass)


def log_plan_marginals(C, beta, gamma, eps):
    """Row and column sums of pi_ij = exp((beta_i + gamma_j - c_ij)/eps - 1)."""
    z = (beta[:, None] + gamma[None, :] - C) / eps - 1.0
    return np.exp(_logsumexp(z, axis=1)), np.exp(_logsumexp(z, axis=0))


def sinkhorn_log(C, p, pt, eps, iters, gamma0=None, record=False):
    """Algorithm 2 (log-domain stabilized Sinkhorn) for a fixed number of
    iterations, with the reading above for the update.

    Potentials start at zero (gamma0 replaces the starting gamma).  One
    iteration is the odd half-step
        log t_i = LSE_j (gamma_j/eps - 1/2 - c_ij/eps),
        beta_i  = eps (log p_i - log t_i) + eps/2,
    then the even half-step with the roles of (beta, p) and (gamma, pt)
    swapped.  A zero weight gives the potential -inf.  Returns the potentials,
    log tt of the last even half-step and, with ``record``, the dual before
    and after every half-step with the Kullback-Leibler term of Lemma 2.4.
    """
    C = np.asarray(C, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    pt = np.asarray(pt, dtype=np.float64)
    n, nt = C.shape
    beta = np.zeros(n)
    gamma = np.zeros(nt) if gamma0 is None else np.array(gamma0, dtype=np.float64)
    logp, logpt = _log_or_neg_inf(p), _log_or_neg_inf(pt)
    hist = []
    logt = logtt = None
    for _ in range(iters):
        logt = _logsumexp((gamma[None, :] - C) / eps - 0.5, axis=1)
        if record:
            rows, _ = log_plan_marginals(C, beta, gamma, eps)
            hist.append(dict(kind="row", kl=kl(p, rows), dual_before=log_dual_value(C, beta, gamma, p, pt, eps)))
        beta = eps * (logp - logt) + 0.5 * eps
        if record:
            hist[-1]["dual_after"] = log_dual_value(C, beta, gamma, p, pt, eps)
        logtt = _logsumexp((beta[:, None] - C) / eps - 0.5, axis=0)
        if record:
            _, cols = log_plan_marginals(C, beta, gamma, eps)
            hist.append(dict(kind="col", kl=kl(pt, cols), dual_before=log_dual_value(C, beta, gamma, p, pt, eps)))
        gamma = eps * (logpt - logtt) + 0.5 * eps
        if record:
            hist[-1]["dual_after"] = log_dual_value(C, beta, gamma, p, pt, eps)
    return dict(beta=beta, gamma=gamma, logt=logt, logtt=logtt, hist=hist)


def solve_log(x, p, y, pt, r, eps, iters, gamma0=None):
    """Algorithm 2 for ``iters`` iterations plus its read-outs.

    cost: sum p beta + sum pt gamma - eps sum_j tt_j exp(gamma_j/eps - 1/2)
    with tt the last even half-step's sums (the result of Algorithm 4);
    cost_upper: cost + eps (H(p) + H(pt)) (Section 3.2);
    marg_err_row / marg_err_col: the two norms of eq. (Error) for the plan
    exp((beta_i + gamma_j - c_ij)/eps - 1).
    """
    p = np.asarray(p, dtype=np.float64)
    pt = np.asarray(pt, dtype=np.float64)
    C = cost_matrix(x, y, r)
    out = sinkhorn_log(C, p, pt, eps, iters, gamma0=gamma0)
    beta, gamma = out["beta"], out["gamma"]
    if iters > 0:
        mass = float(np.sum(np.exp(out["logtt"] + gamma / eps - 0.5)))
    else:
        mass = float(np.sum(log_plan_marginals(C, beta, gamma, eps)[0]))
    s = float(np.sum(p[p > 0] * beta[p > 0])) + float(np.sum(pt[pt > 0] * gamma[pt > 0])) - eps * mass
    rows, cols = log_plan_marginals(C, beta, gamma, eps)
    e_row = float(np.linalg.norm(rows - p))
    e_col = float(np.linalg.norm(cols - pt))
    return dict(beta=beta, gamma=gamma, cost=s, cost_upper=cost_upper_bound(s, p, pt, eps),
                marg_err_row=e_row, marg_err_col=e_col, marg_err=e_row + e_col)
