"""The batch workload's small problems at the full iteration count against
the FP64 dense oracle (values in tests/golden/batched_t300.json, written by
tests/golden/make_batched_t300.py from the oracle alone): every problem with
eps < 0.01 and at most 5000 points per cloud, plus 16 more at random, solved
as one batch with NFS_AUTO for 300 iterations.

Problems that stay on FP32 grids meet the FP32 tolerance 1e-5 on the cost
after the fixed iteration count.  A scaling alpha_i = p_i / t_i carries the
relative error of its sum t_i, and the fast sum's error is normwise in the
l1 norm of the source weights: about 1e-7 of it with FP32 grids (measured
on this batch, 2.7e-6 of the largest sum at most), so at point i up to about
1e-7 ||w||_1 / t_i <= 1e-7 dyn_range.  The sampled scalings of FP32 problems
are held to 1e-6 dyn_range (dyn_range <= 1e5 on FP32 grids under NFS_AUTO).
Problems promoted to FP64 grids (or to the centred form, whose iterates are
the same) meet 1e-10 on the cost, and on the scalings 1e-9 plus the same
model with FP64 rounding, 1e-15 dyn_range.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2201_07524_amd import nfs, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda"
HERE = os.path.dirname(os.path.abspath(__file__))


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def test_small_batch_problems_full_iterations_match_oracle():
    gold = json.load(open(os.path.join(HERE, "golden", "batched_t300.json")))
    cfg = workloads.batched_2d()
    sel = [g["b"] for g in gold["problems"]]
    probs = [cfg["problems"][b] for b in sel]
    prm = nfs.Params(d=2, eps=1.0, N=cfg["N"], m=cfg["m"], precision="auto")
    res = nfs.batch_sinkhorn(prm, [T(q["x"]) for q in probs], [T(q["p"]) for q in probs],
                             [T(q["y"]) for q in probs], [T(q["pt"]) for q in probs],
                             [q["eps"] for q in probs], gold["iters"])
    report = []
    for g, q, r in zip(gold["problems"], probs, res):
        assert r.n_nonpos == 0 and r.iters == gold["iters"]
        fp64 = r.precision_used == "fp64"
        ea = np.max(np.abs(r.alpha.cpu().numpy()[g["idx_alpha"]] / np.array(g["alpha"]) - 1))
        et = np.max(np.abs(r.alpha_t.cpu().numpy()[g["idx_alpha_t"]] / np.array(g["alpha_t"]) - 1))
        ec = abs(r.cost - g["cost"]) / abs(g["cost"])
        report.append((g["b"], r.precision_used, r.centred, r.dyn_range, ec, ea, et))
        assert ec <= (1e-10 if fp64 else 1e-5), report[-1]
        assert abs(r.cost_upper - g["cost_upper"]) <= (1e-10 if fp64 else 1e-5) * abs(g["cost_upper"]), report[-1]
        assert max(ea, et) <= (1e-9 + 1e-15 * r.dyn_range if fp64 else 1e-6 * r.dyn_range), report[-1]
    print("worst cost errors:", sorted(report, key=lambda t: -t[4])[:4])
    print("promoted:", [t[:4] for t in report if t[1] == "fp64"])
