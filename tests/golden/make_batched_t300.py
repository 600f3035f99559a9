"""Writes batched_t300.json: the FP64 dense oracle (Algorithm 1, 300
iterations from the default start, with the Algorithm 3 read-outs) on
problems of the 512-problem batch workload (workloads.batched_2d): every
problem with eps < 0.01 and at most 5000 points per cloud, plus 16 more drawn
at random among those with at most 5000 points.  For each: the cost, the
upper value, ||E||, and the scalings at 16 sampled points of each cloud.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_batched_t300.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import sinkhorn_dense as sd  # noqa: E402
from paper_2201_07524_amd import workloads  # noqa: E402

ITERS = 300
NMAX = 5000


def main():
    sizes, eps = workloads.batched_sizes()
    small = [b for b in range(len(sizes)) if sizes[b] <= NMAX]
    sel = [b for b in small if eps[b] < 0.01]
    rest = [b for b in small if b not in sel]
    extra = np.random.default_rng(16).choice(rest, size=16, replace=False)
    sel = sorted(sel + [int(b) for b in extra])
    cfg = workloads.batched_2d()
    out = {"iters": ITERS, "problems": []}
    for b in sel:
        q = cfg["problems"][b]
        r = sd.solve(q["x"], q["p"], q["y"], q["pt"], 2, q["eps"], ITERS)
        rng = np.random.default_rng(1000 + b)
        ia = np.sort(rng.choice(len(q["p"]), size=16, replace=False))
        it = np.sort(rng.choice(len(q["pt"]), size=16, replace=False))
        out["problems"].append({
            "b": b, "n": int(len(q["p"])), "eps": q["eps"], "cost": r["cost"], "cost_upper": r["cost_upper"],
            "marg_err": r["marg_err"], "idx_alpha": ia.tolist(), "alpha": r["alpha"][ia].tolist(),
            "idx_alpha_t": it.tolist(), "alpha_t": r["alpha_t"][it].tolist()})
        print(f"b={b} n={len(q['p'])} eps={q['eps']:.4f} cost={r['cost']:.12e} marg={r['marg_err']:.2e}", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched_t300.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
