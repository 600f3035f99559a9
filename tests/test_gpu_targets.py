"""GPU parity of the target-side envelope gradient and of the coupling-vector
product pi v against the FP64 oracle.

Tolerances as for the source-side gradient and the fast summation: FP64 with
m = 8 within 1e-9 (gradient positions) and 1e-10 (weights, products, normwise
relative to the largest output); FP32 within 1e-5; r = 1 within the measured
truncation bound of its regularized kernel (eps_I = 8/N, p = 10).
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


def relerr(got, ref):
    return np.max(np.abs(got - ref)) / np.max(np.abs(ref))


def solved(n, eps, N, iters, seed, prec="fp64", r=2, **kw):
    cfg = workloads.subsample(workloads.gmm_2d(10000), n, seed=seed)
    prm = nfs.Params(d=2, r=r, eps=eps, N=N, m=8, precision=prec, **kw)
    res = nfs.sinkhorn(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]), iters)
    return cfg, prm, res


def test_target_gradient_fp64_vs_oracle():
    cfg, prm, res = solved(1000, 0.03, 128, 80, 18)
    gy, gn = nfs.sinkhorn_grad_targets(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]),
                                       res.alpha, res.alpha_t)
    K = sd.gibbs_kernel(cfg["x"], cfg["y"], 2, 0.03)
    ry, rn = sd.envelope_gradient_targets(cfg["x"], cfg["y"], K, res.alpha.cpu().numpy(),
                                          res.alpha_t.cpu().numpy(), 2, 0.03)
    assert relerr(gy.cpu().numpy(), ry) <= 1e-9
    assert relerr(gn.cpu().numpy(), rn) <= 1e-10
    # one output only (the grid flush adds with atomics, so two calls agree to rounding)
    gy2, none = nfs.sinkhorn_grad_targets(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]),
                                          res.alpha, res.alpha_t, want_nu=False)
    assert none is None and relerr(gy2.cpu().numpy(), gy.cpu().numpy()) <= 1e-12


def test_autograd_in_target_positions_and_weights():
    """SinkhornCost backward in y and nu against central differences of the
    solved cost (positions h = 1e-4; weights along nu_j - nu_k)."""
    cfg = workloads.subsample(workloads.gmm_2d(5000), 300, seed=19)
    eps = 0.05
    prm = nfs.Params(d=2, eps=eps, N=64, m=8, precision="fp64")
    y = T(cfg["y"]).requires_grad_(True)
    nu = T(cfg["pt"]).requires_grad_(True)
    s = nfs.SinkhornCost.apply(T(cfg["x"]), T(cfg["p"]), y, nu, prm, 400)
    s.backward()
    gy, gn = y.grad.cpu().numpy(), nu.grad.cpu().numpy()
    assert abs(gn.sum()) <= 1e-12

    def cost(yy, qq):
        return nfs.sinkhorn(prm, T(cfg["x"]), T(cfg["p"]), T(yy), T(qq), 400).cost

    h = 1e-4
    for j, c in [(0, 1), (50, 0), (299, 1)]:
        yp, ym = cfg["y"].copy(), cfg["y"].copy()
        yp[j, c] += h
        ym[j, c] -= h
        fd = (cost(yp, cfg["pt"]) - cost(ym, cfg["pt"])) / (2 * h)
        assert abs(fd - gy[j, c]) <= 1e-6 * max(1.0, abs(fd))
    pt = cfg["pt"]
    for j, k in [(3, 8), (120, 250)]:
        hh = 1e-3 * min(pt[j], pt[k])
        qp, qm = pt.copy(), pt.copy()
        qp[j] += hh
        qp[k] -= hh
        qm[j] -= hh
        qm[k] += hh
        fd = (cost(cfg["y"], qp) - cost(cfg["y"], qm)) / (2 * hh)
        assert abs(fd - (gn[j] - gn[k])) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("transpose", [False, True])
def test_plan_apply_fp64_vs_oracle(transpose):
    cfg, prm, res = solved(1200, 0.03, 128, 40, 20)
    a, at = res.alpha.cpu().numpy(), res.alpha_t.cpu().numpy()
    n, nt = cfg["x"].shape[0], cfg["y"].shape[0]
    v = np.random.default_rng(21).normal(size=n if transpose else nt)
    got = nfs.plan_apply(prm, T(cfg["x"]), T(cfg["y"]), res.alpha, res.alpha_t, T(v), transpose=transpose)
    K = sd.gibbs_kernel(cfg["x"], cfg["y"], 2, 0.03)
    ref = sd.plan_apply(K, a, at, v, transpose=transpose)
    assert relerr(got.cpu().numpy(), ref) <= 1e-10
    # the column marginal after a full iteration is nu exactly (up to rounding)
    if transpose:
        ones = nfs.plan_apply(prm, T(cfg["x"]), T(cfg["y"]), res.alpha, res.alpha_t, T(np.ones(n)), transpose=True)
        assert relerr(ones.cpu().numpy(), cfg["pt"]) <= 1e-10


def test_plan_apply_fp32_and_r1():
    cfg, prm, res = solved(1500, 0.02, 128, 30, 22, prec="fp32")
    a, at = res.alpha.cpu().numpy(), res.alpha_t.cpu().numpy()
    v = np.random.default_rng(23).uniform(0.0, 1.0, cfg["y"].shape[0])
    got = nfs.plan_apply(prm, T(cfg["x"]), T(cfg["y"]), res.alpha, res.alpha_t, T(v)).cpu().numpy()
    ref = sd.plan_apply(sd.gibbs_kernel(cfg["x"], cfg["y"], 2, 0.02), a, at, v)
    assert relerr(got, ref) <= 1e-5
    cfg1, prm1, res1 = solved(1200, 0.05, 64, 20, 24, r=1, eps_I=8, p_smooth=10)
    a1, at1 = res1.alpha.cpu().numpy(), res1.alpha_t.cpu().numpy()
    v1 = np.random.default_rng(25).uniform(0.0, 1.0, cfg1["y"].shape[0])
    got1 = nfs.plan_apply(prm1, T(cfg1["x"]), T(cfg1["y"]), res1.alpha, res1.alpha_t, T(v1)).cpu().numpy()
    ref1 = sd.plan_apply(sd.gibbs_kernel(cfg1["x"], cfg1["y"], 1, 0.05), a1, at1, v1)
    # r = 1: the truncation floor of the regularized kernel (1e-8 to 5e-7 over
    # the fast-summation tests); the weights alpha_t o v span a wider range
    assert relerr(got1, ref1) <= 5e-7


def test_plan_apply_rejects_bad_transpose():
    cfg, prm, res = solved(200, 0.05, 32, 5, 26)
    lib = nfs.load_library()
    import ctypes
    ws, nb = nfs._workspace(prm, 200, 200, torch.device(DEV))
    out = torch.empty(200, dtype=torch.float64, device=DEV)
    v = torch.ones(200, dtype=torch.float64, device=DEV)
    rc = lib.nfs_plan_apply(ctypes.byref(prm.to_c()), T(cfg["x"]).data_ptr(), 200, T(cfg["y"]).data_ptr(), 200,
                            res.alpha.data_ptr(), res.alpha_t.data_ptr(), v.data_ptr(), 2, out.data_ptr(),
                            ws.data_ptr(), nb, nfs._stream())
    assert rc == nfs.NFS_EINVAL
