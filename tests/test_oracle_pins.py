"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with a retyping of itself: each checks a
closed form, an identity of the paper's lemmas, a special case with a textbook
answer, or a brute-force evaluation of a different formula.  A dropped term,
a wrong sign, a swapped weight vector or a transposed kernel in the oracle
fails at least one of them (see test_planted_mistakes_are_caught).
"""
import math

import numpy as np
import pytest

from oracle import direct, ndft
from oracle import sinkhorn_dense as sd
from paper_2201_07524_amd import workloads


def _cloud(n, d, seed, scale=0.2):
    return np.random.default_rng(seed).uniform(-scale, scale, size=(n, d))


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("r", [1, 2])
@pytest.mark.parametrize("eps", [0.01, 0.3])
def test_single_point_cost_equals_ground_cost(r, eps):
    """n = nt = 1: the only coupling is the product, and the Algorithm 3 result
    s = eps(1 + log a + log at - at*tt) reduces to c(x, y) exactly."""
    x = np.array([[0.1, -0.2]])
    y = np.array([[-0.05, 0.07]])
    out = sd.solve(x, np.ones(1), y, np.ones(1), r, eps, iters=3)
    c = np.linalg.norm(x - y) ** r
    assert abs(out["cost"] - c) <= 1e-14 * max(1.0, c)
    assert abs(out["cost_primal"] - c) <= 1e-14 * max(1.0, c)


@pytest.mark.parametrize("eps", [0.02, 0.5])
def test_coincident_support_closed_form(eps):
    """All points at one location: c = 0, pi = p pt^T, and
    s = 0 - eps*H(pi) = -eps (H(p) + H(pt)) (Definition 2.2)."""
    n, nt = 7, 5
    x = np.tile([[0.3, -0.1]], (n, 1))
    y = np.tile([[0.3, -0.1]], (nt, 1))
    p = workloads.dirichlet_weights(n, 1)
    pt = workloads.dirichlet_weights(nt, 2)
    out = sd.solve(x, p, y, pt, 2, eps, iters=2)
    expect = -eps * (sd.entropy(p) + sd.entropy(pt))
    assert abs(out["cost"] - expect) <= 1e-14
    K = sd.gibbs_kernel(x, y, 2, eps)
    assert np.allclose(sd.transport_plan(K, out["alpha"], out["alpha_t"]), np.outer(p, pt),
                       rtol=1e-14, atol=0)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("r", [1, 2])
def test_kernel_sum_riemann_closed_form(d, r):
    """A uniform lattice of spacing h with weights h^d integrates the kernel:
    sum_j h^d exp(-|x - y_j|^r/eps) -> int exp(-|z|^r/eps) dz, which is
    (pi eps)^(d/2) for r = 2 and eps^d d! vol(B_d) for r = 1.  The lattice rule
    is spectrally accurate for the Gaussian; for r = 1 the cusp sits on a node
    and the error is O(h^2).  Pins the cost exponent, the Euclidean norm and
    the placement of eps, in both the dense and the C direct sums."""
    eps = 0.05 if r == 2 else 0.02
    h = {1: 0.01, 2: 0.02, 3: 0.03}[d] if r == 2 else {1: 1e-3, 2: 2.5e-3, 3: 5e-3}[d]
    half = int(math.ceil((6.5 * eps ** 0.5 if r == 2 else 38 * eps) / h))
    ax = h * np.arange(-half, half + 1)
    pts = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1).reshape(-1, d)
    w = np.full(pts.shape[0], h ** d)
    tgt = np.zeros((1, d))
    if r == 2:
        exact = (math.pi * eps) ** (d / 2)
        tol = 1e-12
    else:
        vol = {1: 2.0, 2: math.pi, 3: 4.0 * math.pi / 3.0}[d]
        exact = eps ** d * math.factorial(d) * vol
        tol = 3e-3
    got_c = direct.kv(tgt, pts, w, r, eps)[0]
    assert abs(got_c - exact) <= tol * exact
    if pts.shape[0] <= 40000:
        got_dense = (sd.gibbs_kernel(tgt, pts, r, eps) @ w)[0]
        assert abs(got_dense - exact) <= tol * exact


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("rho", [1.5, 3.0])
def test_kernel_integral_real_exponent(d, rho):
    """A real exponent of the distance (Definition 2.1): the midpoint sum of
    exp(-|x|^rho/eps) over a fine grid approaches its integral over R^d,
    vol_d eps^(d/rho) Gamma(1 + d/rho) (radial substitution u = r^rho/eps).
    Pins the exponent's placement in the C direct sums and the dense kernel."""
    eps = 0.02
    h = {1: 1e-3, 2: 2.5e-3, 3: 6e-3}[d]
    half = int(math.ceil((38 * eps) ** (1.0 / rho) / h))
    ax = h * np.arange(-half, half + 1)
    pts = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1).reshape(-1, d)
    w = np.full(pts.shape[0], h ** d)
    tgt = np.zeros((1, d))
    vol = {1: 2.0, 2: math.pi, 3: 4.0 * math.pi / 3.0}[d]
    exact = vol * eps ** (d / rho) * math.gamma(1.0 + d / rho)
    got_c = direct.kv(tgt, pts, w, rho, eps)[0]
    assert abs(got_c - exact) <= 3e-3 * exact
    if pts.shape[0] <= 40000:
        got_dense = (sd.gibbs_kernel(tgt, pts, rho, eps) @ w)[0]
        assert abs(got_dense - exact) <= 3e-3 * exact


def test_real_exponent_homogeneity():
    """exp(-|l z|^rho / (l^rho eps)) = exp(-|z|^rho/eps): scaling the clouds by
    l and eps by l^rho leaves the sums unchanged only with the exponent on the
    distance itself (not on its square, nor on eps)."""
    x, y = _cloud(50, 2, 31), _cloud(70, 2, 32)
    w = np.random.default_rng(33).uniform(0, 1, 70)
    for rho in (1.5, 2.5):
        a = direct.kv(x, y, w, rho, 0.05)
        b = direct.kv(3.0 * x, 3.0 * y, w, rho, 0.05 * 3.0 ** rho)
        assert np.allclose(a, b, rtol=1e-12, atol=0)
        K = sd.gibbs_kernel(x, y, rho, 0.05)
        assert np.allclose(a, K @ w, rtol=1e-13, atol=0)


@pytest.mark.parametrize("eps", [0.02, 0.5])
def test_coincident_support_upper_value_is_zero(eps):
    """Coincident supports: c = 0, so s = -eps (H(p) + H(pt)) and the upper
    value of Section 3.2, s + (H(P) + H(Pt))/lambda, is exactly the transport
    cost 0 (the upper bound of Lemma 2.1 is attained).  An upper value that
    drops the factor eps (or 1/lambda) on the entropies is nonzero here for
    every eps != 1."""
    n, nt = 6, 9
    x = np.tile([[-0.2, 0.15]], (n, 1))
    y = np.tile([[-0.2, 0.15]], (nt, 1))
    p = workloads.dirichlet_weights(n, 21)
    pt = workloads.dirichlet_weights(nt, 22)
    out = sd.solve(x, p, y, pt, 2, eps, iters=2)
    assert abs(out["cost_upper"]) <= 1e-15
    assert abs(out["cost_primal"]) == 0.0


def test_marginal_errors_closed_form_on_unit_kernel():
    """eq. (Error) with the Euclidean norm, at a state where it is known by
    hand: coincident supports make every kernel entry 1, and at alpha = 1,
    alpha_t = 1 each row of pi sums to nt and each column to n.  With n = 3,
    p = (1/2, 1/4, 1/4) and nt = 4, pt = 1/4 the row residual vector is
    (3.5, 3.75, 3.75), of Euclidean norm sqrt(40.375) (its l1 norm is 11 and
    its squared norm 40.375), and the column residual vector is 2.75 in each
    of 4 entries, of Euclidean norm 5.5 (l1 norm 11, squared norm 30.25)."""
    x = np.zeros((3, 2))
    y = np.zeros((4, 2))
    K = sd.gibbs_kernel(x, y, 2, 0.1)
    assert np.all(K == 1.0)
    p = np.array([0.5, 0.25, 0.25])
    pt = np.full(4, 0.25)
    e_row, e_col = sd.marginal_errors(K, np.ones(3), np.ones(4), p, pt)
    assert abs(e_row - math.sqrt(40.375)) <= 1e-15
    assert abs(e_col - 5.5) <= 1e-15


# ---------------------------------------------------------------- the paper's lemmas
@pytest.mark.parametrize("r", [1, 2])
def test_dual_ascent_equals_kl(r):
    """Lemma 2.4: once the current coupling has unit mass, each half-step
    raises the dual (eq. (14)) by exactly eps*KL(target marginal | current
    marginal).  Holds from the second half-step on (the start alpha = 1 has
    no unit mass)."""
    n, nt, eps = 40, 33, 0.05
    x, y = _cloud(n, 2, 3), _cloud(nt, 2, 4)
    p, pt = workloads.dirichlet_weights(n, 5), workloads.dirichlet_weights(nt, 6)
    K = sd.gibbs_kernel(x, y, r, eps)
    out = sd.sinkhorn(K, p, pt, 6, eps=eps, record=True)
    for step in out["hist"][1:]:
        gain = step["dual_after"] - step["dual_before"]
        assert abs(gain - eps * step["kl"]) <= 1e-13 + 1e-10 * abs(gain)
        assert gain >= -1e-15


def test_lemma_2_1_chain_1d_exact_wasserstein():
    """Lemma 2.1: s <= w_2 <= <pi^s, C> <= s + eps (H(P) + H(Pt)).  In one
    dimension with equal uniform weights the exact w_2 is the mean squared
    difference of the sorted samples."""
    cfg = workloads.plain_1d(256)
    eps = cfg["eps"]
    K = sd.gibbs_kernel(cfg["x"], cfg["y"], 2, eps)
    res = sd.sinkhorn_to_tolerance(K, cfg["p"], cfg["pt"], tol=1e-13)
    a, at, tt = res["alpha"], res["alpha_t"], res["tt"]
    s = sd.cost_readout(a, at, tt, cfg["p"], cfg["pt"], eps)
    w2 = float(np.mean((np.sort(cfg["x"][:, 0]) - np.sort(cfg["y"][:, 0])) ** 2))
    primal = sd.primal_cost(K, sd.cost_matrix(cfg["x"], cfg["y"], 2), a, at)
    upper = sd.cost_upper_bound(s, cfg["p"], cfg["pt"], eps)
    assert s <= w2 <= primal <= upper
    # and the ERW identity of eq. (15): primal = s + eps*H(pi)
    pi = sd.transport_plan(K, a, at)
    H = -float(np.sum(sd.xlogy(pi, pi)))
    assert abs(primal - (s + eps * H)) <= 1e-10


def test_converged_marginals_and_positive_scalings():
    """At the fixed point both marginals of eq. (Error) vanish and the
    scalings are positive and finite (eq. (pi*) with pi > 0)."""
    cfg = workloads.subsample(workloads.gmm_2d(3000), 300)
    K = sd.gibbs_kernel(cfg["x"], cfg["y"], 2, 0.05)
    res = sd.sinkhorn_to_tolerance(K, cfg["p"], cfg["pt"], tol=1e-14)
    e_row, e_col = sd.marginal_errors(K, res["alpha"], res["alpha_t"], cfg["p"], cfg["pt"])
    assert e_row <= 1e-14 and e_col <= 1e-15
    assert np.all(res["alpha"] > 0) and np.all(np.isfinite(res["alpha"]))
    assert np.all(res["alpha_t"] > 0) and np.all(np.isfinite(res["alpha_t"]))


@pytest.mark.parametrize("r", [1, 2])
def test_symmetry_and_translation_invariance(r):
    """s(P, Pt) = s(Pt, P) at the fixed point, and s depends only on x - y."""
    n, nt, eps = 30, 25, 0.05
    x, y = _cloud(n, 2, 8), _cloud(nt, 2, 9)
    p, pt = workloads.dirichlet_weights(n, 10), workloads.dirichlet_weights(nt, 11)

    def conv_cost(xa, pa, yb, pb):
        K = sd.gibbs_kernel(xa, yb, r, eps)
        res = sd.sinkhorn_to_tolerance(K, pa, pb, tol=1e-15)
        return sd.cost_readout(res["alpha"], res["alpha_t"], res["tt"], pa, pb, eps)

    s1 = conv_cost(x, p, y, pt)
    s2 = conv_cost(y, pt, x, p)
    shift = np.array([0.37, -1.3])
    s3 = conv_cost(x + shift, p, y + shift, pt)
    assert abs(s1 - s2) <= 1e-12
    assert abs(s1 - s3) <= 1e-12


# ---------------------------------------------------------------- fast-summation sums
def test_ndft_single_source_closed_forms():
    """A unit source at y = 0 has fhat_k = 1; at y = 1/4 (d = 1) it is (-i)^k.
    A single mode fhat = delta_k0 evaluates to exp(2 pi i k0 x)."""
    N = 8
    f0 = ndft.ndft_adjoint(np.zeros((1, 2)), np.ones(1), N)
    assert np.allclose(f0, 1.0, atol=1e-15)
    f1 = ndft.ndft_adjoint(np.array([[0.25]]), np.ones(1), N)
    k = np.arange(-N // 2, N // 2)
    assert np.allclose(f1, (-1j) ** k, atol=1e-14)
    fh = np.zeros((N, N), dtype=complex)
    fh[N // 2 + 3, N // 2 - 2] = 1.0
    x = np.array([[0.1, 0.3], [-0.4, 0.2]])
    got = ndft.ndft_trafo(fh, x, N)
    assert np.allclose(got, np.exp(2j * np.pi * (3 * x[:, 0] - 2 * x[:, 1])), atol=1e-14)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_gauss_coeffs_poisson_summation(d):
    """The trigonometric polynomial with the closed-form coefficients equals
    the brute-force sum over periodic images of the Gaussian."""
    eps_t = 0.01 if d < 3 else 0.02     # truncation error exp(-pi^2 eps_t N^2/4) < 1e-20
    N = {1: 64, 2: 64, 3: 32}[d]
    b = ndft.gauss_coeffs(N, d, eps_t)
    z = np.random.default_rng(12).uniform(-0.5, 0.5, size=(20, d))
    poly = np.real(ndft.ndft_trafo(b, z, N))
    brute = ndft.periodized_gauss(z, eps_t, images=2)
    assert np.max(np.abs(poly - brute)) <= 1e-13


@pytest.mark.parametrize("d", [1, 2])
def test_ndft_fastsum_matches_dense_gibbs(d):
    """eq. (fastsum) with periodization coefficients reproduces the dense
    kernel product when the points are well inside the torus."""
    eps_t = 0.004
    N = 64
    x = np.random.default_rng(13).uniform(-0.2, 0.2, size=(50, d))
    y = np.random.default_rng(14).uniform(-0.2, 0.2, size=(60, d))
    w = np.random.default_rng(15).uniform(0.0, 1.0, size=60)
    fs = ndft.fastsum_ndft(x, y, w, ndft.gauss_coeffs(N, d, eps_t))
    dense = sd.gibbs_kernel(x, y, 2, eps_t) @ w
    assert np.max(np.abs(fs - dense)) <= 1e-13 * np.max(np.abs(dense))


def test_direct_sum_matches_dense():
    """The matrix-free C sums and the dense numpy kernel agree (two
    independent routes to the same definition)."""
    x, y = _cloud(200, 3, 16), _cloud(300, 3, 17)
    w = np.random.default_rng(18).uniform(0, 1, 300)
    for r in (1, 2):
        K = sd.gibbs_kernel(x, y, r, 0.03)
        assert np.allclose(direct.kv(x, y, w, r, 0.03), K @ w, rtol=1e-13, atol=0)
        rows = np.array([5, 0, 199])
        assert np.allclose(direct.kv(x, y, w, r, 0.03, rows=rows), (K @ w)[rows], rtol=1e-13, atol=0)
        a = np.random.default_rng(19).uniform(0.5, 1.5, 200)
        gx, _ = sd.envelope_gradient(x, y, K, a, w, r, 0.03)
        g2 = direct.grad_rows(x, y, w, r, 0.03) * a[:, None]
        assert np.allclose(gx, g2, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- gradient
def test_gradient_sum_identity_r2():
    """For r = 2: sum_i d s/d x_i = 2 (sum_i (pi 1)_i x_i - sum_j pt_j y_j),
    which at the fixed point is 2 (sum p x - sum pt y)."""
    n, nt, eps = 60, 50, 0.05
    x, y = _cloud(n, 2, 20), _cloud(nt, 2, 21)
    p, pt = workloads.dirichlet_weights(n, 22), workloads.dirichlet_weights(nt, 23)
    K = sd.gibbs_kernel(x, y, 2, eps)
    res = sd.sinkhorn_to_tolerance(K, p, pt, tol=1e-15)
    gx, gmu = sd.envelope_gradient(x, y, K, res["alpha"], res["alpha_t"], 2, eps)
    expect = 2.0 * (p @ x - pt @ y)
    assert np.allclose(gx.sum(axis=0), expect, atol=1e-13)
    assert abs(gmu.sum()) <= 1e-14


@pytest.mark.parametrize("r", [1, 2, 1.5])
def test_gradient_central_differences(r):
    """Envelope gradient vs central finite differences of the converged cost.
    Positions: h = 1e-4.  Weights: along the simplex directions e_i - e_k with
    a step relative to the smaller weight."""
    n, nt, eps = 24, 20, 0.05
    x, y = _cloud(n, 2, 24), _cloud(nt, 2, 25)
    p, pt = workloads.dirichlet_weights(n, 26), workloads.dirichlet_weights(nt, 27)

    def cost(xx, pp):
        K = sd.gibbs_kernel(xx, y, r, eps)
        res = sd.sinkhorn_to_tolerance(K, pp, pt, tol=1e-15)
        return sd.cost_readout(res["alpha"], res["alpha_t"], res["tt"], pp, pt, eps), res

    s0, res = cost(x, p)
    K = sd.gibbs_kernel(x, y, r, eps)
    gx, gmu = sd.envelope_gradient(x, y, K, res["alpha"], res["alpha_t"], r, eps)
    h = 1e-4
    for i, c in [(0, 0), (3, 1), (17, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[i, c] += h
        xm[i, c] -= h
        fd = (cost(xp, p)[0] - cost(xm, p)[0]) / (2 * h)
        assert abs(fd - gx[i, c]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8
    for i, k in [(1, 2), (5, 11)]:
        hh = 1e-3 * min(p[i], p[k])
        pp, pm = p.copy(), p.copy()
        pp[i] += hh
        pp[k] -= hh
        pm[i] -= hh
        pm[k] += hh
        fd = (cost(x, pp)[0] - cost(x, pm)[0]) / (2 * hh)
        assert abs(fd - (gmu[i] - gmu[k])) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("r", [1, 2, 1.5])
def test_target_gradient_central_differences_and_translation(r):
    """Target-side envelope gradient vs central differences of the converged
    cost (positions h = 1e-4, weights along e_j - e_k), and translation
    invariance: moving both clouds together leaves s unchanged, so the
    position gradients of both sides sum to zero."""
    n, nt, eps = 22, 24, 0.05
    x, y = _cloud(n, 2, 34), _cloud(nt, 2, 35)
    p, pt = workloads.dirichlet_weights(n, 36), workloads.dirichlet_weights(nt, 37)

    def cost(yy, qq):
        K = sd.gibbs_kernel(x, yy, r, eps)
        res = sd.sinkhorn_to_tolerance(K, p, qq, tol=1e-15)
        return sd.cost_readout(res["alpha"], res["alpha_t"], res["tt"], p, qq, eps), res

    s0, res = cost(y, pt)
    K = sd.gibbs_kernel(x, y, r, eps)
    gy, gnu = sd.envelope_gradient_targets(x, y, K, res["alpha"], res["alpha_t"], r, eps)
    gx, _ = sd.envelope_gradient(x, y, K, res["alpha"], res["alpha_t"], r, eps)
    assert np.allclose(gx.sum(axis=0) + gy.sum(axis=0), 0.0, atol=1e-14)
    assert abs(gnu.sum()) <= 1e-14
    h = 1e-4
    for j, c in [(0, 1), (9, 0), (23, 1)]:
        yp, ym = y.copy(), y.copy()
        yp[j, c] += h
        ym[j, c] -= h
        fd = (cost(yp, pt)[0] - cost(ym, pt)[0]) / (2 * h)
        assert abs(fd - gy[j, c]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8
    for j, k in [(2, 7), (13, 20)]:
        hh = 1e-3 * min(pt[j], pt[k])
        qp, qm = pt.copy(), pt.copy()
        qp[j] += hh
        qp[k] -= hh
        qm[j] -= hh
        qm[k] += hh
        fd = (cost(y, qp)[0] - cost(y, qm)[0]) / (2 * hh)
        assert abs(fd - (gnu[j] - gnu[k])) <= 1e-6 * max(1.0, abs(fd))


def test_plan_apply_marginals_and_bilinearity():
    """pi 1 is the row marginal alpha o (K alpha_t), and after an even
    half-step pi^T 1 = pt exactly (eq. (S1)); u^T (pi v) = (pi^T u)^T v."""
    n, nt, eps = 30, 26, 0.05
    x, y = _cloud(n, 2, 40), _cloud(nt, 2, 41)
    p, pt = workloads.dirichlet_weights(n, 42), workloads.dirichlet_weights(nt, 43)
    K = sd.gibbs_kernel(x, y, 2, eps)
    out = sd.sinkhorn(K, p, pt, 5)
    a, at = out["alpha"], out["alpha_t"]
    assert np.allclose(sd.plan_apply(K, a, at, np.ones(nt)), a * (K @ at), rtol=1e-14, atol=0)
    assert np.allclose(sd.plan_apply(K, a, at, np.ones(n), transpose=True), pt, rtol=1e-13, atol=0)
    rng = np.random.default_rng(44)
    u, v = rng.normal(size=n), rng.normal(size=nt)
    lhs = u @ sd.plan_apply(K, a, at, v)
    rhs = sd.plan_apply(K, a, at, u, transpose=True) @ v
    assert abs(lhs - rhs) <= 1e-14 * max(1.0, abs(lhs))


# ---------------------------------------------------------------- the pins bite
def test_planted_mistakes_are_caught():
    """Plant plausible mistakes in copies of the oracle's formulas (on the
    CPU) and check that the pins above would reject them."""
    n, nt, eps = 40, 33, 0.05
    x, y = _cloud(n, 2, 3), _cloud(nt, 2, 4)
    p, pt = workloads.dirichlet_weights(n, 5), workloads.dirichlet_weights(nt, 6)
    K = sd.gibbs_kernel(x, y, 2, eps)

    # (a) even half-step divides pt by K alpha_t (transposed kernel / wrong operand)
    def bad_sinkhorn(K, p, pt, iters):
        a, at = np.ones(K.shape[0]), np.ones(K.shape[1])
        hist = []
        for _ in range(iters):
            a = p / (K @ at)
            before = sd.dual_value(K, a, at, p, pt, eps)
            kl_term = sd.kl(pt, at * (K.T @ a))
            at = pt / (K.T @ (a * 0 + 1))          # planted: uses ones instead of alpha
            hist.append((sd.dual_value(K, a, at, p, pt, eps) - before, eps * kl_term))
        return hist
    bad = bad_sinkhorn(K, p, pt, 4)
    assert any(abs(g - e) > 1e-8 for g, e in bad[1:])

    # (b) readout that forgets the eps*(1 - sum tt*at) term, on a non-normalized state
    a, at = np.ones(n), np.ones(nt)
    tt = K.T @ a
    good = sd.cost_readout(a, at, tt, p, pt, eps)
    dropped = eps * float(np.sum(sd.xlogy(p, a))) + eps * float(np.sum(sd.xlogy(pt, at)))
    assert abs(good - dropped) > 1e-3

    # (c) Gaussian coefficients with a wrong exponent sign or a missing pi factor
    b = ndft.gauss_coeffs(64, 1, 0.01)
    z = np.linspace(-0.5, 0.5, 7)[:, None]
    brute = ndft.periodized_gauss(z, 0.01, images=2)
    assert np.max(np.abs(np.real(ndft.ndft_trafo(b, z, 64)) - brute)) < 1e-13
    wrong = b * np.pi
    assert np.max(np.abs(np.real(ndft.ndft_trafo(wrong, z, 64)) - brute)) > 1e-3
    k = np.arange(-32, 32)
    wrong_sign = (np.pi * 0.01) ** 0.5 * np.exp(-np.pi ** 2 * 0.01 * k * k) * (-1.0) ** k
    assert np.max(np.abs(np.real(ndft.ndft_trafo(wrong_sign, z, 64)) - brute)) > 1e-3

    # (d) gradient without the factor 2 breaks the sum identity
    res = sd.sinkhorn_to_tolerance(K, p, pt, tol=1e-15)
    gx, _ = sd.envelope_gradient(x, y, K, res["alpha"], res["alpha_t"], 2, eps)
    expect = 2.0 * (p @ x - pt @ y)
    assert np.allclose(gx.sum(0), expect, atol=1e-13)
    assert not np.allclose((0.5 * gx).sum(0), expect, atol=1e-6)

    # (f) upper value without the factor eps on the entropies: on coincident
    # supports it is not the closed-form 0 of test_coincident_support_upper_value_is_zero
    xc = np.zeros((n, 2))
    yc = np.zeros((nt, 2))
    sc = sd.solve(xc, p, yc, pt, 2, eps, iters=2)["cost"]
    assert abs(sd.cost_upper_bound(sc, p, pt, eps)) <= 1e-15
    assert abs(sc + sd.entropy(p) + sd.entropy(pt)) > 1e-2

    # (g) marginal residual in the l1 or squared norm instead of the Euclidean
    # one misses the closed form of test_marginal_errors_closed_form_on_unit_kernel
    K1 = np.ones((3, 4))
    p3, pt4 = np.array([0.5, 0.25, 0.25]), np.full(4, 0.25)
    row = np.ones(3) * (K1 @ np.ones(4)) - p3
    col = np.ones(4) * (K1.T @ np.ones(3)) - pt4
    assert abs(float(np.sum(np.abs(row))) - math.sqrt(40.375)) > 1.0
    assert abs(float(np.sum(row * row)) - math.sqrt(40.375)) > 1.0
    assert abs(float(np.sum(np.abs(col))) - 5.5) > 1.0
    assert abs(float(np.sum(col * col)) - 5.5) > 1.0

    # (e) Sinkhorn divergence without the factors 1/2 is not zero on identical
    # measures (the pin of property 3 rejects it)
    out = sd.sinkhorn_divergence(x, p, x, p, 2, eps, 200)
    assert abs(out["cost_xy"] - out["cost_xx"] - out["cost_yy"]) > 1e-3


# ---------------------------------------------------------------- Sinkhorn divergence
def test_sinkhorn_divergence_vanishes_on_identical_measures():
    """sd(P, P) = 0 for every eps (property 3 of the Sinkhorn divergence)."""
    x = _cloud(30, 2, 41)
    p = np.random.default_rng(42).dirichlet(np.ones(30))
    for eps in (0.01, 0.1):
        out = sd.sinkhorn_divergence(x, p, x, p, 2, eps, 200)
        assert abs(out["sd"]) <= 1e-15 * abs(out["cost_xy"])


@pytest.mark.parametrize("r", [1, 2])
def test_sinkhorn_divergence_nonnegative(r):
    """sd(P, Pt) >= 0 at convergence (property 1; the Gaussian and Laplace
    kernels are positive definite), and sd is symmetric."""
    for seed in range(4):
        x, y = _cloud(40, 2, 100 + seed), _cloud(35, 2, 200 + seed) + 0.05 * seed
        p = np.random.default_rng(300 + seed).dirichlet(np.ones(40))
        pt = np.random.default_rng(400 + seed).dirichlet(np.ones(35))
        a = sd.sinkhorn_divergence(x, p, y, pt, r, 0.05, 3000)
        b = sd.sinkhorn_divergence(y, pt, x, p, r, 0.05, 3000)
        assert a["sd"] >= -1e-12
        assert abs(a["sd"] - b["sd"]) <= 1e-12


def test_sinkhorn_divergence_tends_to_wasserstein_1d():
    """sd -> w_2 as eps -> 0 (property 2), with the exact 1-D w_2 from sorting
    (equal uniform weights): the gap shrinks with eps and is within 2% of w_2
    at the smallest eps."""
    rng = np.random.default_rng(7)
    n = 48
    x, y = rng.uniform(-0.25, 0.25, (n, 1)), rng.uniform(-0.1, 0.3, (n, 1))
    p = np.full(n, 1.0 / n)
    w2 = float(np.mean((np.sort(x[:, 0]) - np.sort(y[:, 0])) ** 2))
    gaps = [abs(sd.sinkhorn_divergence(x, p, y, p, 2, eps, 20000)["sd"] - w2) for eps in (0.02, 0.005, 0.0015)]
    assert gaps[0] > gaps[1] > gaps[2]
    assert gaps[2] <= 0.02 * w2


# ---------------------------------------------------------------- log-domain (Algorithms 2 and 4)
def test_log_domain_single_point_at_underflowing_eps():
    """n = nt = 1 with c/eps near 950: the Gibbs kernel underflows to zero in
    FP64 (Algorithm 1 divides by zero), while the log-domain result is c."""
    x = np.array([[0.1, -0.2]])
    y = np.array([[-0.05, 0.07]])
    c = float(np.sum((x - y) ** 2))
    eps = 1e-4
    assert sd.gibbs_kernel(x, y, 2, eps)[0, 0] == 0.0
    out = sd.solve_log(x, np.ones(1), y, np.ones(1), 2, eps, iters=3)
    assert abs(out["cost"] - c) <= 1e-14 * max(1.0, c)
    # the plan exp((beta + gamma - c)/eps - 1) carries the rounding of an
    # exponent of size c/eps
    assert out["marg_err"] <= 10 * 2.0 ** -52 * (c / eps)


@pytest.mark.parametrize("r", [1, 2])
def test_log_domain_equals_algorithm_1(r):
    """With alpha_t0 = exp(gamma0/eps - 1/2) Algorithm 1 produces the same
    couplings: beta = eps (log alpha + 1/2), gamma = eps (log alpha_t + 1/2),
    and the two results (Algorithm 3 read-out, Algorithm 4 result) agree."""
    n, nt, eps, iters = 40, 33, 0.05, 7
    x, y = _cloud(n, 2, 3), _cloud(nt, 2, 4)
    p, pt = workloads.dirichlet_weights(n, 5), workloads.dirichlet_weights(nt, 6)
    g0 = np.random.default_rng(9).normal(0.0, 0.02, nt)
    lg = sd.solve_log(x, p, y, pt, r, eps, iters, gamma0=g0)
    a1 = sd.solve(x, p, y, pt, r, eps, iters, alpha_t0=np.exp(g0 / eps - 0.5))
    assert np.max(np.abs(lg["beta"] - eps * (np.log(a1["alpha"]) + 0.5))) <= 1e-14
    assert np.max(np.abs(lg["gamma"] - eps * (np.log(a1["alpha_t"]) + 0.5))) <= 1e-14
    assert abs(lg["cost"] - a1["cost"]) <= 1e-14
    assert abs(lg["marg_err_row"] - a1["marg_err_row"]) <= 1e-13
    assert abs(lg["cost_upper"] - a1["cost_upper"]) <= 1e-14


def test_log_domain_dual_ascent_equals_kl():
    """Lemma 2.4 in potentials: from the second half-step on, each half-step
    raises the dual of eq. (14) by exactly eps*KL(target | current marginal)."""
    n, nt, eps = 40, 33, 0.05
    x, y = _cloud(n, 2, 3), _cloud(nt, 2, 4)
    p, pt = workloads.dirichlet_weights(n, 5), workloads.dirichlet_weights(nt, 6)
    out = sd.sinkhorn_log(sd.cost_matrix(x, y, 2), p, pt, eps, 6, record=True)
    for step in out["hist"][1:]:
        gain = step["dual_after"] - step["dual_before"]
        assert abs(gain - eps * step["kl"]) <= 1e-13 + 1e-10 * abs(gain)
        assert gain >= -1e-15


def test_log_domain_lemma_2_1_chain_where_the_kernel_underflows():
    """Lemma 2.1, s <= w_2 <= <pi, C> <= s + eps (H(P) + H(Pt)), on two 1-D
    clusters a distance 1 apart at eps = 1e-3: every entry of the Gibbs
    kernel underflows to zero in FP64 (c/eps >= 810), while the part of the
    cost that decides the coupling, -2 (x - mean x)(y - mean y)/eps, spans
    only a few units, so the iteration converges in tens of steps.  w_2 is the
    exact 1-D value from sorting."""
    rng = np.random.default_rng(17)
    n, eps = 24, 1e-3
    x, y = rng.uniform(0.0, 0.1, (n, 1)), rng.uniform(1.0, 1.1, (n, 1))
    p = np.full(n, 1.0 / n)
    C = sd.cost_matrix(x, y, 2)
    assert np.all(np.exp(-C / eps) == 0.0)
    out = sd.solve_log(x, p, y, p, 2, eps, 200)
    assert out["marg_err"] <= 10 * 2.0 ** -52 * np.max(C) / eps
    pi = np.exp((out["beta"][:, None] + out["gamma"][None, :] - C) / eps - 1.0)
    primal = float(np.sum(pi * C))
    w2 = float(np.mean((np.sort(x[:, 0]) - np.sort(y[:, 0])) ** 2))
    assert out["cost"] <= w2 <= primal <= out["cost_upper"]


def test_log_domain_planted_mistake_is_caught():
    """The printed update without the eps/2 reaches a coupling of mass
    e^(-1/2): the equivalence and Lemma 2.4 pins above reject it."""
    n, nt, eps = 40, 33, 0.05
    x, y = _cloud(n, 2, 3), _cloud(nt, 2, 4)
    p, pt = workloads.dirichlet_weights(n, 5), workloads.dirichlet_weights(nt, 6)
    C = sd.cost_matrix(x, y, 2)
    beta, gamma = np.zeros(n), np.zeros(nt)
    gains = []
    for _ in range(5):
        beta = eps * (np.log(p) - sd._logsumexp((gamma[None, :] - C) / eps - 0.5, axis=1))   # planted: no eps/2
        before = sd.log_dual_value(C, beta, gamma, p, pt, eps)
        _, cols = sd.log_plan_marginals(C, beta, gamma, eps)
        logtt = sd._logsumexp((beta[:, None] - C) / eps - 0.5, axis=0)
        gamma = eps * (np.log(pt) - logtt)
        gains.append((sd.log_dual_value(C, beta, gamma, p, pt, eps) - before, eps * sd.kl(pt, cols)))
    assert any(abs(g - e) > 1e-6 for g, e in gains)
    s_bad = float(p @ beta + pt @ gamma) - eps * float(np.sum(np.exp(logtt + gamma / eps - 0.5)))
    ref = sd.solve(x, p, y, pt, 2, eps, 5)["cost"]
    assert abs(s_bad - ref) > 0.1 * eps
