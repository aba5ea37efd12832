"""Writes gl_batched_instances.json: the 64 accepted instances (N, mu0, mu2) of the batched GL workload.

Candidates come in seeded draw order from ``workloads.batched_draws``; a candidate is kept when the largest
real part of the spectrum of its discretised operator (built by the CPU oracle) is below the stability margin
(-0.01), since the time-stepped method needs a stable system (Sec. 2.1: homogeneous solutions must decay).
Calls only ``oracle/`` and ``workloads``.  Run from the repository root:  python tests/golden/make_gl_batched_instances.py
"""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
import workloads  # noqa: E402
from oracle.operators import gl_operator  # noqa: E402


def main():
    cfg = workloads.GL_BATCHED
    accepted, rejected = [], []
    for (n, mu0, mu2) in workloads.batched_draws(cfg, 400):
        L, _ = gl_operator(n, mu0, mu2)
        lam = np.linalg.eigvals(L.toarray()).real.max()
        (accepted if lam < cfg["stability_margin"] else rejected).append([n, mu0, mu2, float(lam)])
        print(n, mu0, mu2, lam, flush=True)
        if len(accepted) == cfg["ninst"]:
            break
    out = dict(workload=cfg["name"], seed=cfg["seed"], stability_margin=cfg["stability_margin"],
               instances=[a[:3] for a in accepted], max_real_eig=[a[3] for a in accepted],
               rejected=rejected)
    with open(workloads.BATCHED_INSTANCES_JSON, "w") as f:
        json.dump(out, f, indent=1)
    print("accepted", len(accepted), "rejected", len(rejected), "total N", sum(a[0] for a in accepted))


if __name__ == "__main__":
    main()
