"""GPU parity of the gradient on a solver handle (nfs_solver_grad): the
envelope gradient (Proposition 2.3, eq. (14)) at the solver's scalings,
evaluated on the plan the iteration used.  Against the dense FP64 oracle
(1e-9 of the largest entry for positions, 1e-10 for weights), against the
one-shot entry points that plan again (1e-12), for single and batched
solvers, with zero weights, and through SinkhornCost's autograd path; the
3-D case also against central differences of the FP64 cost.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sinkhorn_dense as sd
from paper_2201_07524_amd import nfs, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda"


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def rel(got, ref):
    return float(np.max(np.abs(np.asarray(got) - ref)) / np.max(np.abs(ref)))


def problem(d, n, nt, seed, zeros=0):
    x = workloads.gaussian_mixture(n, d, seed)
    y = workloads.gaussian_mixture(nt, d, seed + 1)
    p = workloads.dirichlet_weights(n, seed + 2)
    pt = workloads.dirichlet_weights(nt, seed + 3)
    if zeros:
        idx = np.random.default_rng(seed + 4).choice(n, size=zeros, replace=False)
        p[idx] = 0.0
        p /= p.sum()
    return x, p, y, pt


@pytest.mark.parametrize("d,N", [(1, 128), (2, 64), (3, 32)])
def test_solver_grad_matches_oracle_and_one_shot(d, N):
    x, p, y, pt = problem(d, 700, 650, 60 + d, zeros=5)
    eps, iters = 0.05, 30
    prm = nfs.Params(d=d, eps=eps, N=N, m=8, precision="fp64")
    s = nfs.Solver(prm, T(x), T(p), T(y), T(pt))
    s.iterate(iters)
    res = s.finish()
    gx, gm, gy, gn = s.grad(True, True, True, True)
    s.close()
    a, at = res.alpha.cpu().numpy(), res.alpha_t.cpu().numpy()
    assert np.sum(a == 0.0) == 5
    K = sd.gibbs_kernel(x, y, 2, eps)
    rx, rm = sd.envelope_gradient(x, y, K, a, at, 2, eps)
    ry, rn = sd.envelope_gradient_targets(x, y, K, a, at, 2, eps)
    assert rel(gx.cpu().numpy(), rx) <= 1e-9 and rel(gy.cpu().numpy(), ry) <= 1e-9
    assert rel(gm.cpu().numpy(), rm) <= 1e-10 and rel(gn.cpu().numpy(), rn) <= 1e-10
    ox, om = nfs.sinkhorn_grad(prm, T(x), T(p), T(y), T(pt), res.alpha, res.alpha_t)
    assert rel(gx.cpu().numpy(), ox.cpu().numpy()) <= 1e-12 and rel(gm.cpu().numpy(), om.cpu().numpy()) <= 1e-12


def test_batch_solver_grad_per_problem():
    probs = [problem(2, n, nt, 70 + 3 * b) for b, (n, nt) in enumerate([(400, 500), (900, 300), (250, 260)])]
    eps = [0.05, 0.03, 0.08]
    prm = nfs.Params(d=2, eps=1.0, N=64, m=8, precision="fp64")
    s = nfs.BatchSolver(prm, [T(q[0]) for q in probs], [T(q[1]) for q in probs], [T(q[2]) for q in probs],
                        [T(q[3]) for q in probs], eps)
    s.iterate(25)
    res = s.finish()
    gx, gm, gy, gn = s.grad(True, True, True, True)
    s.close()
    for b, (q, r) in enumerate(zip(probs, res)):
        x, p, y, pt = q
        K = sd.gibbs_kernel(x, y, 2, eps[b])
        a, at = r.alpha.cpu().numpy(), r.alpha_t.cpu().numpy()
        rx, rm = sd.envelope_gradient(x, y, K, a, at, 2, eps[b])
        ry, rn = sd.envelope_gradient_targets(x, y, K, a, at, 2, eps[b])
        sx = slice(s.offs_x[b], s.offs_x[b + 1])
        sy = slice(s.offs_y[b], s.offs_y[b + 1])
        assert rel(gx[sx].cpu().numpy(), rx) <= 1e-9 and rel(gy[sy].cpu().numpy(), ry) <= 1e-9
        assert rel(gm[sx].cpu().numpy(), rm) <= 1e-10 and rel(gn[sy].cpu().numpy(), rn) <= 1e-10


def test_solver_grad_rejects_log_domain():
    x, p, y, pt = problem(2, 200, 200, 80)
    prm = nfs.Params(d=2, eps=0.05, N=64, m=8, precision="fp64", flags=nfs.FLAG_LOG_DOMAIN)
    s = nfs.Solver(prm, T(x), T(p), T(y), T(pt))
    s.iterate(2)
    with pytest.raises(nfs.NfsError) as e:
        s.grad()
    assert e.value.code == nfs.NFS_EUNSUPPORTED
    s.close()


def ball_shell(n, nt, seed):
    x = workloads.uniform_ball(n, seed)
    y = workloads.noisy_shell(nt, seed + 1)
    return x, workloads.uniform_weights(n), y, workloads.uniform_weights(nt)


@pytest.mark.parametrize("prec,eps_I,p_smooth,tol", [("fp64", 8, 10, 2e-6), ("fp32", 0, 0, 3e-4)])
def test_r1_gradient_matches_oracle(prec, eps_I, p_smooth, tol):
    """Euclidean cost (r = 1): grad_x c = (x - y)/|x - y|.  The regularized
    kernel's part goes through the spectral derivative, the correction
    K - K_R through direct sums over the pairs closer than eps_I.  3-D
    ball/shell subsample at eps = 0.02, N = 128: against the dense oracle's
    envelope gradient at the GPU's scalings, normwise.  The error is the
    truncation of the regularized kernel's Fourier series, which the
    derivative weights by |k|: with eps_I = 8/N, p = 10 (FP64) it measures
    1.2e-6; at the default near field (eps_I = 4/N, p = 8) 1.1e-4 in FP32 and
    2.2e-4 in FP64 on this shape (a sweep over eps_I N in 2..4, p in 4..10:
    1e-4 to 1e-2), so the FP32 bound is that truncation level, not
    rounding."""
    x, p, y, pt = ball_shell(1400, 1300, 95)
    eps = 0.02
    prm = nfs.Params(d=3, r=1, eps=eps, N=128, m=6 if prec == "fp32" else 8, precision=prec, eps_I=eps_I,
                     p_smooth=p_smooth)
    s = nfs.Solver(prm, T(x), T(p), T(y), T(pt))
    s.iterate(15)
    res = s.finish()
    gx, gm, gy, gn = s.grad(True, True, True, True)
    s.close()
    a, at = res.alpha.cpu().numpy(), res.alpha_t.cpu().numpy()
    K = sd.gibbs_kernel(x, y, 1, eps)
    rx, rm = sd.envelope_gradient(x, y, K, a, at, 1, eps)
    ry, rn = sd.envelope_gradient_targets(x, y, K, a, at, 1, eps)
    ex, ey = rel(gx.cpu().numpy(), rx), rel(gy.cpu().numpy(), ry)
    print(f"r=1 {prec}: grad_x {ex:.2e} grad_y {ey:.2e}")
    assert ex <= tol and ey <= tol
    assert rel(gm.cpu().numpy(), rm) <= 1e-10 and rel(gn.cpu().numpy(), rn) <= 1e-10
    ox, _ = nfs.sinkhorn_grad(prm, T(x), T(p), T(y), T(pt), res.alpha, res.alpha_t, want_mu=False)
    assert rel(gx.cpu().numpy(), ox.cpu().numpy()) <= (1e-12 if prec == "fp64" else 1e-5)


def test_autograd_through_the_solver_handle_3d_finite_differences():
    """SinkhornCost with a fixed iteration count keeps its solver for the
    backward pass.  3-D, 2048 points per cloud (the subproblem size of the
    differentiated workload), FP64: gradients in x, mu, y and nu against the
    dense oracle and against central differences of the FP64 cost (positions
    h = 1e-4; weights along e_i - e_k with h = 1e-3 min(p_i, p_k))."""
    cfg = workloads.gmm_3d(200000)
    rng = np.random.default_rng(90)
    ix = rng.choice(200000, 2048, replace=False)
    iy = rng.choice(200000, 2048, replace=False)
    x0, y0 = cfg["x"][ix], cfg["y"][iy]
    p0 = np.full(2048, 1 / 2048)
    eps, iters = 0.01, 300
    prm = nfs.Params(d=3, eps=eps, N=128, m=8, precision="fp64")
    x, p, y, pt = (T(v).requires_grad_(True) for v in (x0, p0, y0, p0))
    s = nfs.SinkhornCost.apply(x, p, y, pt, prm, iters)
    s.backward()
    res = nfs.sinkhorn(prm, T(x0), T(p0), T(y0), T(p0), iters)
    K = sd.gibbs_kernel(x0, y0, 2, eps)
    a, at = res.alpha.cpu().numpy(), res.alpha_t.cpu().numpy()
    rx, rm = sd.envelope_gradient(x0, y0, K, a, at, 2, eps)
    ry, rn = sd.envelope_gradient_targets(x0, y0, K, a, at, 2, eps)
    assert rel(x.grad.cpu().numpy(), rx) <= 1e-9 and rel(y.grad.cpu().numpy(), ry) <= 1e-9
    assert rel(p.grad.cpu().numpy(), rm) <= 1e-10 and rel(pt.grad.cpu().numpy(), rn) <= 1e-10

    def cost(xv, pv, yv, ptv):
        return nfs.sinkhorn(prm, T(xv), T(pv), T(yv), T(ptv), iters).cost

    h = 1e-4
    gx = x.grad.cpu().numpy()
    for i, c in [(0, 0), (511, 1), (2047, 2)]:
        xp, xm = x0.copy(), x0.copy()
        xp[i, c] += h
        xm[i, c] -= h
        fd = (cost(xp, p0, y0, p0) - cost(xm, p0, y0, p0)) / (2 * h)
        assert abs(fd - gx[i, c]) <= 1e-6 * max(1e-3, abs(gx[i, c])), (i, c, fd, gx[i, c])
    gp = p.grad.cpu().numpy()
    for i, k in [(3, 1000), (2000, 17)]:
        hw = 1e-3 * min(p0[i], p0[k])
        pp, pm = p0.copy(), p0.copy()
        pp[i] += hw
        pp[k] -= hw
        pm[i] -= hw
        pm[k] += hw
        fd = (cost(x0, pp, y0, p0) - cost(x0, pm, y0, p0)) / (2 * hw)
        assert abs(fd - (gp[i] - gp[k])) <= 1e-5 * max(1e-3, abs(gp[i] - gp[k])), (i, k, fd, gp[i] - gp[k])
