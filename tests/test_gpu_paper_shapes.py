"""GPU parity on the paper-shaped standing workloads: two images on one k x k
pixel grid (the shape of the benchmark-image experiments, with smoothed
random-field intensities, about one pixel in six of zero weight) and uniform
samples on [0,1]^2 (the two-dimensional synthetic experiment), eps = 0.05
(lambda = 20), r = 2, FP64 grids with N = 64, m = 8.

Small sizes against the dense oracle within 1e-10; the 256^2 grid against the
oracle's matrix-free sums on sampled targets (FP64 1e-10, FP32 1e-5, both
relative to the largest output).
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
    return abs(a - b) / abs(b)


@pytest.mark.parametrize("name", ["grid32", "uniform2000"])
def test_small_vs_dense_oracle(name):
    cfg = workloads.pixel_grid_pair(32) if name == "grid32" else workloads.uniform_square(2000)
    iters = 100
    prm = nfs.Params(d=2, eps=cfg["eps"], N=64, m=8, precision="fp64")
    res = nfs.sinkhorn(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), iters)
    ref = sd.solve(cfg["x"], cfg["p"], cfg["y"], cfg["pt"], 2, cfg["eps"], iters)
    a, at = res.alpha.cpu().numpy(), res.alpha_t.cpu().numpy()
    assert res.kernel_err <= 1e-15
    assert np.array_equal(a == 0, ref["alpha"] == 0) and np.array_equal(at == 0, ref["alpha_t"] == 0)
    nz, nzt = ref["alpha"] > 0, ref["alpha_t"] > 0
    assert np.max(np.abs(a[nz] / ref["alpha"][nz] - 1)) <= 1e-10
    assert np.max(np.abs(at[nzt] / ref["alpha_t"][nzt] - 1)) <= 1e-10
    assert rel(res.cost, ref["cost"]) <= 1e-10
    assert rel(res.cost_upper, ref["cost_upper"]) <= 1e-10


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_grid256_sampled(prec, tol):
    """65536 pixels per image, 20 iterations: the last half-step on 256 sampled
    targets of positive weight (plus the largest sum)."""
    cfg = workloads.pixel_grid_pair(256)
    prm = nfs.Params(d=2, eps=cfg["eps"], N=64, m=8, precision=prec)
    res = nfs.sinkhorn(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), 20)
    a, at = res.alpha.cpu().numpy(), res.alpha_t.cpu().numpy()
    assert res.n_nonpos == 0
    pos = np.flatnonzero(cfg["pt"] > 0)
    tt_gpu = np.zeros_like(at)
    tt_gpu[pos] = cfg["pt"][pos] / at[pos]
    rows = np.union1d(np.random.default_rng(31).choice(pos, size=256, replace=False), [np.argmax(tt_gpu)])
    tt = direct.kv(cfg["y"], cfg["x"], a, 2, cfg["eps"], rows=rows)
    assert np.max(np.abs(tt_gpu[rows] - tt)) <= tol * np.max(tt)
