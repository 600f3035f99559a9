"""NFS_FLAG_AUTOTUNE: the solver plans and times a few iterations at each
candidate tile size (half, one and two times the default) and then at each
candidate chunk size, keeps the fastest, and restores the starting values.
The fixed-point grids make the spread sums exact, so tiles and chunks only
change the order of the FP64 reductions: the tuned and the plain solves agree
to rounding, the iteration count and the t <= 0 counters are unaffected, and
at the default tile the tuned chunk is never smaller than the default (fewer
or as many chunks)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2201_07524_amd import nfs, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda"


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def solve(cfg, flags, iters, prec="fp64", N=128, eps=0.02, alpha_t0=None):
    prm = nfs.Params(d=cfg["x"].shape[1], eps=eps, N=N, m=8, precision=prec, flags=flags)
    s = nfs.Solver(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]),
                   alpha_t0=None if alpha_t0 is None else T(alpha_t0))
    s.iterate(iters)
    _, info = s.profile(1)
    res = s.finish()
    s.close()
    return res, info


@pytest.mark.parametrize("warm", [False, True])
def test_autotuned_solve_matches_plain(warm):
    cfg = workloads.subsample(workloads.gmm_2d(200000), 50000, seed=4)
    start = np.random.default_rng(6).uniform(0.5, 2.0, 50000) if warm else None
    plain, ip = solve(cfg, 0, 15, alpha_t0=start)
    tuned, it = solve(cfg, nfs.FLAG_AUTOTUNE, 15, alpha_t0=start)
    assert tuned.iters == plain.iters == 16 and tuned.n_nonpos == 0
    assert ip["tile"] == 32 and it["tile"] in (16, 32, 64)
    if it["tile"] == ip["tile"]:
        assert it["chunks_x"] <= ip["chunks_x"]
    a, b = tuned.alpha.cpu().numpy(), plain.alpha.cpu().numpy()
    assert np.max(np.abs(a / b - 1)) <= 1e-12
    assert abs(tuned.cost - plain.cost) <= 1e-13 * abs(plain.cost)


def test_autotune_dense_cloud_and_batch():
    """1e6 uniform points on a 128^2 grid (dense) in FP32, and a batch in FP64."""
    cfg = workloads.uniform_square(10**6)
    plain, ip = solve(cfg, 0, 4, prec="fp32", N=64, eps=0.05)
    tuned, it = solve(cfg, nfs.FLAG_AUTOTUNE, 4, prec="fp32", N=64, eps=0.05)
    assert ip["tile"] == 32 and it["tile"] in (16, 32, 64)
    if it["tile"] == ip["tile"]:
        assert it["chunks_x"] <= ip["chunks_x"]
    assert abs(tuned.cost - plain.cost) <= 1e-6 * abs(plain.cost)
    probs = [workloads.subsample(workloads.gmm_2d(20000), n, seed=10 + n) for n in (3000, 800, 5000)]
    eps = [0.03, 0.05, 0.02]
    out = []
    for flags in (0, nfs.FLAG_AUTOTUNE):
        prm = nfs.Params(d=2, eps=1.0, N=128, m=8, precision="fp64", flags=flags)
        out.append(nfs.batch_sinkhorn(prm, [T(q["x"]) for q in probs], [T(q["p"]) for q in probs],
                                      [T(q["y"]) for q in probs], [T(q["pt"]) for q in probs], eps, 20))
    for r0, r1 in zip(*out):
        assert abs(r1.cost - r0.cost) <= 1e-13 * abs(r0.cost)
        assert np.max(np.abs(r1.alpha.cpu().numpy() / r0.alpha.cpu().numpy() - 1)) <= 1e-12
