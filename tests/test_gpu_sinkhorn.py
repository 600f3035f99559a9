"""GPU parity of the NFFT-accelerated Sinkhorn solve and its gradient against
the FP64 oracle (dense Algorithm 1 with the read-outs of Algorithm 3).

Tolerances: FP64 with m = 8 within 1e-10 relative on the cost and the
scalings after the same number of iterations; FP32 within 1e-5 relative on
the cost.  At full size (the 2-D mixture workload with 1e6 points per
cloud) the last half-step is checked on sampled outputs with the oracle's
matrix-free FP64 sums.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import direct
from oracle import sinkhorn_dense as sd
from paper_2201_07524_amd import nfs, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda"


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def run_gpu(cfg, iters, prec, N, m, eps, flags=0, tol=0.0, alpha_t0=None, **kw):
    prm = nfs.Params(d=cfg["x"].shape[1], eps=eps, N=N, m=m, precision=prec, flags=flags, **kw)
    return nfs.sinkhorn(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), iters, tol=tol,
                        alpha_t0=None if alpha_t0 is None else T(alpha_t0))


@pytest.mark.parametrize("flags", [0, nfs.FLAG_NO_GRAPH])
def test_plain_1d_full_config_fp64(flags):
    """d = 1, n = nt = 2048, eps = 0.05, N = 256, m = 8, 200 iterations, FP64."""
    cfg = workloads.plain_1d()
    ref = sd.solve(cfg["x"], cfg["p"], cfg["y"], cfg["pt"], 2, cfg["eps"], cfg["iters"])
    res = run_gpu(cfg, cfg["iters"], "fp64", cfg["N"], cfg["m"], cfg["eps"], flags=flags | nfs.FLAG_PRIMAL_COST)
    a, at = res.alpha.cpu().numpy(), res.alpha_t.cpu().numpy()
    assert res.iters == 200
    assert np.all(a > 0) and np.all(at > 0)
    assert np.max(np.abs(a - ref["alpha"]) / ref["alpha"]) <= 1e-10
    assert np.max(np.abs(at - ref["alpha_t"]) / ref["alpha_t"]) <= 1e-10
    assert rel(res.cost, ref["cost"]) <= 1e-10
    assert rel(res.cost_upper, ref["cost_upper"]) <= 1e-10
    assert rel(res.cost_primal, ref["cost_primal"]) <= 1e-10
    assert abs(res.marg_err_row - ref["marg_err_row"]) <= 1e-10 * max(ref["marg_err_row"], 1e-6)
    assert res.marg_err_col <= 1e-12


def test_2d_mixture_fp32_small_vs_oracle():
    """A 3000-point subsample of the 2-D mixture workload (Dirichlet weights),
    eps = 0.01, N = 128, m = 8, FP32 grids, 100 iterations."""
    cfg = workloads.subsample(workloads.gmm_2d(20000), 3000, seed=3)
    eps, iters = 0.01, 100
    ref = sd.solve(cfg["x"], cfg["p"], cfg["y"], cfg["pt"], 2, eps, iters)
    res = run_gpu(cfg, iters, "fp32", 128, 8, eps, flags=nfs.FLAG_PRIMAL_COST)
    assert rel(res.cost, ref["cost"]) <= 1e-5
    assert rel(res.cost_primal, ref["cost_primal"]) <= 1e-5
    a = res.alpha.cpu().numpy()
    assert np.all(a > 0) and np.all(np.isfinite(a))
    # marginal error of the GPU scalings (evaluated with the exact kernel) within
    # 10x the oracle's after the same number of iterations, plus the FP32 floor:
    # FP32 grid sums carry absolute errors of order u * max_i t_i (u = 2^-24), so
    # a target with kernel sum t_i sees a relative error up to u max(t) / t_i and
    # its marginal entry an error up to p_i times that
    K = sd.gibbs_kernel(cfg["x"], cfg["y"], 2, eps)
    e_row, e_col = sd.marginal_errors(K, a, res.alpha_t.cpu().numpy(), cfg["p"], cfg["pt"])
    u = 2.0 ** -24
    t, tt = K @ ref["alpha_t"], K.T @ ref["alpha"]
    floor = (np.linalg.norm(cfg["p"] * np.minimum(1.0, u * t.max() / t))
             + np.linalg.norm(cfg["pt"] * np.minimum(1.0, u * tt.max() / tt)))
    assert e_row + e_col <= 10 * ref["marg_err"] + floor
    # and the row marginals of the two states agree to FP32 accuracy amplified by the iteration
    row_gpu = a * (K @ res.alpha_t.cpu().numpy())
    row_ref = ref["alpha"] * (K @ ref["alpha_t"])
    assert np.max(np.abs(row_gpu - row_ref)) <= 1e-4 * np.max(row_ref)


def test_2d_fp64_small_vs_oracle():
    cfg = workloads.subsample(workloads.gmm_2d(20000), 2000, seed=4)
    eps, iters = 0.02, 60
    ref = sd.solve(cfg["x"], cfg["p"], cfg["y"], cfg["pt"], 2, eps, iters)
    res = run_gpu(cfg, iters, "fp64", 128, 8, eps)
    assert rel(res.cost, ref["cost"]) <= 1e-10
    assert np.max(np.abs(res.alpha.cpu().numpy() / ref["alpha"] - 1)) <= 1e-9
    assert np.max(np.abs(res.alpha_t.cpu().numpy() / ref["alpha_t"] - 1)) <= 1e-9


def test_3d_fp64_small_vs_oracle():
    cfg = workloads.subsample(workloads.gmm_3d(20000), 1500, seed=5)
    eps, iters = 0.05, 30
    ref = sd.solve(cfg["x"], cfg["p"], cfg["y"], cfg["pt"], 2, eps, iters)
    res = run_gpu(cfg, iters, "fp64", 32, 8, eps)
    assert rel(res.cost, ref["cost"]) <= 1e-10
    assert np.max(np.abs(res.alpha.cpu().numpy() / ref["alpha"] - 1)) <= 1e-9


def test_warm_start_resume_equals_continuous_run():
    cfg = workloads.plain_1d(1024)
    full = run_gpu(cfg, 50, "fp64", 256, 8, 0.05)
    first = run_gpu(cfg, 20, "fp64", 256, 8, 0.05)
    second = run_gpu(cfg, 30, "fp64", 256, 8, 0.05, alpha_t0=first.alpha_t.cpu().numpy())
    assert np.max(np.abs(second.alpha.cpu().numpy() / full.alpha.cpu().numpy() - 1)) <= 1e-12
    assert rel(second.cost, full.cost) <= 1e-12


def oracle_errors(K, p, pt, iters):
    """||E|| of eq. (Error) after each of `iters` oracle iterations (the
    column term is zero after an alpha_t update)."""
    out = []
    a_t = np.ones(K.shape[1])
    for _ in range(iters):
        a = p / (K @ a_t)
        a_t = pt / (K.T @ a)
        out.append(float(np.linalg.norm(a * (K @ a_t) - p)))
    return np.array(out)


def test_tolerance_stops_early():
    """Each alpha update evaluates ||E|| of the state the previous iteration
    left; the solve finishes that iteration and stops.  So the state after
    iters - 1 iterations is the first one within the tolerance, and the
    result is the oracle's after `iters` iterations."""
    cfg = workloads.plain_1d(512)
    tol, eps = 1e-9, 0.05
    res = run_gpu(cfg, 5000, "fp64", 256, 8, eps, tol=tol)
    K = sd.gibbs_kernel(cfg["x"], cfg["y"], 2, eps)
    errs = oracle_errors(K, cfg["p"], cfg["pt"], res.iters)
    k = res.iters
    assert k < 5000
    assert errs[k - 2] <= tol * (1 + 1e-4) and errs[k - 3] > tol * (1 - 1e-4)
    assert res.marg_err <= tol
    ref = sd.solve(cfg["x"], cfg["p"], cfg["y"], cfg["pt"], 2, eps, k)
    assert abs(res.cost - ref["cost"]) <= 1e-10 * abs(ref["cost"])
    assert np.max(np.abs(res.alpha.cpu().numpy() / ref["alpha"] - 1)) <= 1e-9


def test_dynamic_range_statistic_matches_oracle_iterates():
    """nfs_result.dyn_range is the largest ||w||_1 / min_i t_i over the
    solve's half-steps, w the source weights of the sums t (the quantity the
    fast sums' normwise error is measured against); the same on the oracle's
    dense iterates."""
    cfg = workloads.subsample(workloads.gmm_2d(10000), 800, seed=6)
    eps, iters = 0.02, 12
    res = run_gpu(cfg, iters, "fp64", 128, 8, eps)
    K = sd.gibbs_kernel(cfg["x"], cfg["y"], 2, eps)
    p, pt = cfg["p"], cfg["pt"]
    a_t = np.ones(len(pt))
    worst = 0.0
    for _ in range(iters):
        t = K @ a_t
        worst = max(worst, a_t.sum() / t[p > 0].min())
        a = p / t
        tt = K.T @ a
        worst = max(worst, a.sum() / tt[pt > 0].min())
        a_t = pt / tt
    assert worst > 10.0
    assert res.dyn_range == pytest.approx(worst, rel=1e-6)


def test_kl_identity_on_device_iterates():
    """Lemma 2.4 on the GPU iterates: the dual rises by eps*KL(p | pi 1) over
    one extra row half-step, with the dual evaluated by the oracle."""
    cfg = workloads.subsample(workloads.gmm_2d(10000), 800, seed=6)
    eps = 0.05
    K = sd.gibbs_kernel(cfg["x"], cfg["y"], 2, eps)
    r5 = run_gpu(cfg, 5, "fp64", 64, 8, eps)
    a, at = r5.alpha.cpu().numpy(), r5.alpha_t.cpu().numpy()
    before = sd.dual_value(K, a, at, cfg["p"], cfg["pt"], eps)
    a_next = cfg["p"] / (K @ at)
    after = sd.dual_value(K, a_next, at, cfg["p"], cfg["pt"], eps)
    assert abs((after - before) - eps * sd.kl(cfg["p"], a * (K @ at))) <= 1e-12


def test_gradient_fp64_vs_oracle():
    cfg = workloads.subsample(workloads.gmm_2d(10000), 1000, seed=8)
    eps = 0.03
    prm = nfs.Params(d=2, eps=eps, N=128, m=8, precision="fp64")
    res = nfs.sinkhorn(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), 80)
    gx, gm = nfs.sinkhorn_grad(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), res.alpha, res.alpha_t)
    K = sd.gibbs_kernel(cfg["x"], cfg["y"], 2, eps)
    rx, rm = sd.envelope_gradient(cfg["x"], cfg["y"], K, res.alpha.cpu().numpy(), res.alpha_t.cpu().numpy(), 2, eps)
    assert np.max(np.abs(gx.cpu().numpy() - rx)) <= 1e-9 * np.max(np.abs(rx))
    assert np.max(np.abs(gm.cpu().numpy() - rm)) <= 1e-10 * np.max(np.abs(rm))


def test_sinkhorn_cost_autograd_matches_finite_differences():
    cfg = workloads.subsample(workloads.gmm_2d(5000), 300, seed=9)
    eps = 0.05
    prm = nfs.Params(d=2, eps=eps, N=64, m=8, precision="fp64")
    x = T(cfg["x"]).requires_grad_(True)
    s = nfs.SinkhornCost.apply(x, T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), prm, 400)
    s.backward()
    g = x.grad.cpu().numpy()
    h = 1e-4
    for i, c in [(0, 0), (7, 1), (100, 0)]:
        xp, xm = cfg["x"].copy(), cfg["x"].copy()
        xp[i, c] += h
        xm[i, c] -= h
        sp = nfs.sinkhorn(prm, T(xp), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), 400).cost
        sm = nfs.sinkhorn(prm, T(xm), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), 400).cost
        assert abs((sp - sm) / (2 * h) - g[i, c]) <= 1e-6 * max(1.0, abs(g[i, c]))


def test_2d_mixture_full_size_sampled_parity():
    """The 2-D mixture workload at its full size (1e6 points per cloud, N = 512,
    m = 8, eps = 0.01, FP32), 20 iterations in the benchmarked launch
    configuration.  The last half-step alpha_t = nu / (K^T alpha) is checked
    on 256 sampled targets with the oracle's FP64 matrix-free sums."""
    cfg = workloads.gmm_2d()
    res = run_gpu(cfg, 20, "fp32", cfg["N"], cfg["m"], cfg["eps"])
    a = res.alpha.cpu().numpy()
    at = res.alpha_t.cpu().numpy()
    assert np.all(a > 0) and np.all(np.isfinite(a)) and np.all(at > 0)
    rows = np.random.default_rng(11).choice(cfg["y"].shape[0], size=256, replace=False)
    tt = direct.kv(cfg["y"], cfg["x"], a, 2, cfg["eps"], rows=rows)
    tt_gpu = cfg["pt"][rows] / at[rows]          # the K^T alpha the GPU divided by
    assert np.max(np.abs(tt_gpu - tt)) <= 1e-5 * np.max(tt)
    assert np.isfinite(res.cost) and res.marg_err_col <= 1e-3 * np.linalg.norm(cfg["pt"])


def test_sinkhorn_r1_3d_vs_oracle():
    """Euclidean cost (r = 1) on a ball/shell subsample: the solve with the
    near-field corrected fast summation tracks the dense oracle."""
    x = workloads.uniform_ball(1200, 1300)
    y = workloads.noisy_shell(1000, 1301)
    p, pt = workloads.uniform_weights(1200), workloads.uniform_weights(1000)
    eps, iters = 0.02, 40
    ref = sd.solve(x, p, y, pt, 1, eps, iters)
    prm = nfs.Params(d=3, r=1, eps=eps, N=128, m=8, precision="fp64", eps_I=8, p_smooth=10)
    res = nfs.sinkhorn(prm, T(x), T(p), T(y), T(pt), iters)
    assert rel(res.cost, ref["cost"]) <= 1e-6
    a = res.alpha.cpu().numpy()
    assert np.all(a > 0)
    K = sd.gibbs_kernel(x, y, 1, eps)
    e_row, e_col = sd.marginal_errors(K, a, res.alpha_t.cpu().numpy(), p, pt)
    assert e_row + e_col <= 10 * ref["marg_err"] + 1e-5 * np.linalg.norm(p)



@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_repeated_solves_are_bit_identical(prec):
    """The plan puts the points of each cell in the order of their input
    index, the spread grid holds exact integer sums of the LDS tiles'
    fixed-point words, and every reduction runs in a fixed order, so a solve
    does not depend on the order in which workgroups or atomics run: two runs
    agree bit for bit (single problem and batch)."""
    cfg = workloads.subsample(workloads.gmm_2d(20000), 5000, seed=21)
    prm = nfs.Params(d=2, eps=0.01, N=256, m=8, precision=prec)
    runs = [nfs.sinkhorn(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), 30) for _ in range(2)]
    assert runs[0].cost == runs[1].cost and runs[0].marg_err == runs[1].marg_err
    assert torch.equal(runs[0].alpha, runs[1].alpha) and torch.equal(runs[0].alpha_t, runs[1].alpha_t)
    probs = [workloads.subsample(workloads.gmm_2d(8000), n, seed=30 + n) for n in (900, 2500, 400)]
    bprm = nfs.Params(d=2, eps=1.0, N=128, m=8, precision=prec)
    b = [nfs.batch_sinkhorn(bprm, [T(q["x"]) for q in probs], [T(q["p"]) for q in probs],
                            [T(q["y"]) for q in probs], [T(q["pt"]) for q in probs], [0.02, 0.03, 0.05], 25)
         for _ in range(2)]
    for r0, r1 in zip(*b):
        assert r0.cost == r1.cost and torch.equal(r0.alpha, r1.alpha) and torch.equal(r0.alpha_t, r1.alpha_t)
