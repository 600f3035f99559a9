"""GPU parity of the Sinkhorn divergence s(P, Pt) - s(P, P)/2 - s(Pt, Pt)/2
(the three problems solved as one batch) against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sinkhorn_dense as sd
from paper_2201_07524_amd import nfs, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda"


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def run(prec, x, p, y, pt, eps, iters, N=64, d=2):
    prm = nfs.Params(d=d, eps=eps, N=N, m=8, precision=prec)
    return nfs.sinkhorn_divergence(prm, T(x), T(p), T(y), T(pt), iters)


def test_divergence_fp64_matches_oracle():
    cfg = workloads.subsample(workloads.gmm_2d(20000), 400, seed=8)
    y, pt = cfg["y"][:350], workloads.dirichlet_weights(350, 77)
    eps, iters = 0.03, 40
    ref = sd.sinkhorn_divergence(cfg["x"], cfg["p"], y, pt, 2, eps, iters)
    got, costs, nonpos = run("fp64", cfg["x"], cfg["p"], y, pt, eps, iters)
    scale = max(abs(ref["cost_xy"]), abs(ref["cost_xx"]), abs(ref["cost_yy"]))
    for g, r in zip(costs, (ref["cost_xy"], ref["cost_xx"], ref["cost_yy"])):
        assert abs(g - r) <= 1e-10 * abs(r)
    assert abs(got - ref["sd"]) <= 1e-10 * scale
    assert nonpos == [0, 0, 0]


def test_divergence_vanishes_on_identical_measures():
    x = np.random.default_rng(5).uniform(-0.2, 0.2, (700, 2))
    p = workloads.dirichlet_weights(700, 6)
    got, costs, _ = run("fp64", x, p, x, p, 0.02, 30)
    assert abs(got) <= 1e-12 * abs(costs[0])


@pytest.mark.parametrize("d,N", [(1, 256), (3, 32)])
def test_divergence_fp32_matches_oracle(d, N):
    rng = np.random.default_rng(30 + d)
    x, y = rng.uniform(-0.2, 0.2, (600, d)), rng.uniform(-0.15, 0.25, (500, d))
    p, pt = workloads.dirichlet_weights(600, 31), workloads.dirichlet_weights(500, 32)
    eps, iters = 0.05, 30
    ref = sd.sinkhorn_divergence(x, p, y, pt, 2, eps, iters)
    got, costs, _ = run("fp32", x, p, y, pt, eps, iters, N=N, d=d)
    scale = max(abs(ref["cost_xy"]), abs(ref["cost_xx"]), abs(ref["cost_yy"]))
    for g, r in zip(costs, (ref["cost_xy"], ref["cost_xx"], ref["cost_yy"])):
        assert abs(g - r) <= 1e-5 * abs(r)
    assert abs(got - ref["sd"]) <= 1e-5 * scale
