"""GPU parity of the batched form (many problems, one launch per stage):
each problem of a batch against its own single-problem solve and against the
FP64 oracle (dense Algorithm 1)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sinkhorn_dense as sd
from paper_2201_07524_amd import nfs, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda"


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def make_batch(d, sizes, eps_list, seed=900):
    probs = []
    for b, (n, e) in enumerate(zip(sizes, eps_list)):
        x = workloads.gaussian_mixture(n, d, seed + 2 * b)
        y = workloads.gaussian_mixture(n + 7 * b, d, seed + 2 * b + 1)
        probs.append(dict(x=x, p=workloads.uniform_weights(n), y=y,
                          pt=workloads.dirichlet_weights(n + 7 * b, seed + 1000 + b), eps=e))
    return probs


@pytest.mark.parametrize("d,N", [(1, 128), (2, 64), (3, 32)])
def test_batched_fp64_matches_oracle_and_single(d, N):
    sizes = [150, 900, 37, 1500, 400]
    eps_list = [0.05, 0.03, 0.08, 0.04, 0.06]
    probs = make_batch(d, sizes, eps_list)
    prm = nfs.Params(d=d, eps=1.0, N=N, m=8, precision="fp64", chunk=128)
    iters = 25
    res = nfs.batch_sinkhorn(prm, [T(p["x"]) for p in probs], [T(p["p"]) for p in probs],
                             [T(p["y"]) for p in probs], [T(p["pt"]) for p in probs], eps_list, iters)
    assert len(res) == len(probs)
    for p, r in zip(probs, res):
        ref = sd.solve(p["x"], p["p"], p["y"], p["pt"], 2, p["eps"], iters)
        assert abs(r.cost - ref["cost"]) <= 1e-10 * abs(ref["cost"])
        assert np.max(np.abs(r.alpha.cpu().numpy() / ref["alpha"] - 1)) <= 1e-9
        assert np.max(np.abs(r.alpha_t.cpu().numpy() / ref["alpha_t"] - 1)) <= 1e-9
        single = nfs.sinkhorn(nfs.Params(d=d, eps=p["eps"], N=N, m=8, precision="fp64", chunk=128),
                              T(p["x"]), T(p["p"]), T(p["y"]), T(p["pt"]), iters)
        assert abs(r.cost - single.cost) <= 1e-12 * abs(single.cost)


def test_batched_fp32_matches_oracle():
    sizes = [3000, 200, 1200, 5000, 800, 2500]
    eps_list = [0.02, 0.05, 0.03, 0.015, 0.04, 0.025]
    probs = make_batch(2, sizes, eps_list, seed=950)
    prm = nfs.Params(d=2, eps=1.0, N=256, m=6, precision="fp32")
    iters = 60
    res = nfs.batch_sinkhorn(prm, [T(p["x"]) for p in probs], [T(p["p"]) for p in probs],
                             [T(p["y"]) for p in probs], [T(p["pt"]) for p in probs], eps_list, iters)
    for p, r in zip(probs, res):
        ref = sd.solve(p["x"], p["p"], p["y"], p["pt"], 2, p["eps"], iters)
        assert abs(r.cost - ref["cost"]) <= 1e-5 * abs(ref["cost"])
        assert r.n_nonpos == 0


def test_batched_warm_and_residual_api():
    probs = make_batch(2, [500, 800, 300], [0.05, 0.04, 0.06], seed=970)
    prm = nfs.Params(d=2, eps=1.0, N=64, m=8, precision="fp64")
    s = nfs.BatchSolver(prm, [T(p["x"]) for p in probs], [T(p["p"]) for p in probs],
                        [T(p["y"]) for p in probs], [T(p["pt"]) for p in probs], [0.05, 0.04, 0.06])
    s.iterate(5)
    e5 = s.residual()
    s.iterate(45)
    e50 = s.residual()
    res = s.finish()
    s.close()
    assert e50 < e5
    assert max(r.marg_err_row for r in res) == pytest.approx(e50, rel=1e-6)
    assert all(r.iters == 50 for r in res)


def test_batched_problems_stop_on_their_own_tolerance():
    """With a tolerance, each problem of a batch stops on its own: the
    iteration after its first state with ||E|| <= tol (eq. (Error)); the
    others keep iterating.  Every problem matches the oracle after its own
    iteration count."""
    sizes = [400, 900, 250, 600]
    eps_list = [0.08, 0.03, 0.05, 0.02]
    probs = make_batch(2, sizes, eps_list, seed=990)
    prm = nfs.Params(d=2, eps=1.0, N=64, m=8, precision="fp64")
    tol = 1e-7
    res = nfs.batch_sinkhorn(prm, [T(p["x"]) for p in probs], [T(p["p"]) for p in probs],
                             [T(p["y"]) for p in probs], [T(p["pt"]) for p in probs], eps_list, 3000, tol=tol)
    iters = [r.iters for r in res]
    assert len(set(iters)) > 1 and max(iters) < 3000
    for p, r in zip(probs, res):
        K = sd.gibbs_kernel(p["x"], p["y"], 2, p["eps"])
        a_t = np.ones(len(p["pt"]))
        errs = []
        for _ in range(r.iters):
            a = p["p"] / (K @ a_t)
            a_t = p["pt"] / (K.T @ a)
            errs.append(float(np.linalg.norm(a * (K @ a_t) - p["p"])))
        assert errs[-2] <= tol * (1 + 1e-4) and (r.iters < 3 or errs[-3] > tol * (1 - 1e-4))
        assert r.marg_err <= tol
        ref = sd.solve(p["x"], p["p"], p["y"], p["pt"], 2, p["eps"], r.iters)
        assert abs(r.cost - ref["cost"]) <= 1e-10 * abs(ref["cost"])
        assert np.max(np.abs(r.alpha.cpu().numpy() / ref["alpha"] - 1)) <= 1e-9
