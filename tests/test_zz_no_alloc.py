"""GPU check of the allocation-free fast summation (nfs_fastsum_apply_noalloc).

It is the workspace entry point nfs_fastsum_apply with its scratch in the
library's static device array.  Two calls in a row, the second on a smaller
problem (the array keeps the first call's contents), each compared with
nfs_fastsum_apply on the same inputs and with the dense FP64 oracle.
Tolerances as for fast summation: FP64 with m = 8 within 1e-10 of the largest
output against the oracle, FP32 within 1e-5; the two entry points run the
same kernels, so they agree to the spread flush's summation order (1e-12
FP64, 1e-6 FP32).
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
    return float(np.max(np.abs(np.asarray(got) - np.asarray(ref))) / np.max(np.abs(ref)))


def _case(d, ns, nt, seed):
    tgt = workloads.gaussian_mixture(nt, d, seed)
    src = workloads.gaussian_mixture(ns, d, seed + 1)
    w = np.random.default_rng(seed + 2).uniform(0.0, 1.0, size=ns)
    return src, w, tgt


@pytest.mark.parametrize("prec,tol_same,tol_oracle", [("fp64", 1e-12, 1e-10), ("fp32", 1e-6, 1e-5)])
@pytest.mark.parametrize("d,N,eps", [(1, 256, 0.05), (2, 128, 0.01), (3, 32, 0.05)])
def test_noalloc_matches_workspace_entry_point(d, N, eps, prec, tol_same, tol_oracle):
    prm = nfs.Params(d=d, eps=eps, N=N, m=8, precision=prec, chunk=257)
    # the second call is smaller: it runs on whatever the first one left in the scratch
    for ns, nt, seed in ((3000, 2500, 40 + d), (700, 333, 50 + d)):
        src, w, tgt = _case(d, ns, nt, seed)
        print(f"noalloc d={d} N={N} {prec} ns={ns} nt={nt}", flush=True)
        got = nfs.fastsum_noalloc(prm, T(src), T(w), T(tgt)).cpu().numpy()
        ref_ws = nfs.fastsum(prm, T(src), T(w), T(tgt)).cpu().numpy()
        ref = sd.gibbs_kernel(tgt, src, 2, eps) @ w
        assert relerr(got, ref_ws) <= tol_same
        assert relerr(got, ref) <= tol_oracle


def test_noalloc_caller_output_buffer_and_limit():
    prm = nfs.Params(d=2, eps=0.01, N=64, m=6, precision="fp32")
    src, w, tgt = _case(2, 500, 400, 61)
    out = torch.full((400,), float("nan"), dtype=torch.float64, device=DEV)
    got = nfs.fastsum_noalloc(prm, T(src), T(w), T(tgt), out=out)
    assert got.data_ptr() == out.data_ptr()
    ref = sd.gibbs_kernel(tgt, src, 2, 0.01) @ w
    assert relerr(out.cpu().numpy(), ref) <= 1e-5
    # above the static scratch: rejected on the host before any device work
    big = nfs.Params(d=3, eps=0.01, N=128, m=8, precision="fp64")
    assert nfs.workspace_size(big, 10, 10) > nfs.NOALLOC_SCRATCH_BYTES
    one = T(np.zeros((10, 3)))
    with pytest.raises(nfs.NfsError) as ei:
        nfs.fastsum_noalloc(big, one, T(np.ones(10)), one)
    assert ei.value.code == nfs.NFS_EWORKSPACE
