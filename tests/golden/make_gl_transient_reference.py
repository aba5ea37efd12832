"""Writes gl_transient_reference.json: the CPU oracle's block power iteration on the transient-response workload
(1-D Ginzburg-Landau, N = 200, mu0 = 0.30, h = 0.01, 64 frequencies in [-2, 2] snapped to P = 9,896 steps, one
forcing window of P steps and a 20,000-step tail, k = 1, 20 iterations, seeded N(0,1) complex start).

The method is the transient-response method of Sec. 2.2 with the frequency-domain power iteration of App. A
(eqs. iteration, powerMethod and the Rayleigh-Ritz estimate after arDec): every iteration is one explicit RK4
direct run and one adjoint run of the oracle (``oracle.stepping``), 29,896 steps each.  Stored: the gain history
of both estimators for every frequency and iteration, the final gains, and the final force and response modes at
eight sampled frequencies (both band edges included).  The run takes about three minutes on one CPU core.

Calls only ``oracle/`` and ``workloads``.  Run from the repository root:
    python tests/golden/make_gl_transient_reference.py
"""
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
import workloads  # noqa: E402
from oracle.iteration import block_power_iteration, stepped_applies  # noqa: E402
from oracle.operators import gl_operator  # noqa: E402
from oracle.stepping import snap_grid  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gl_transient_reference.json")
SAMPLED = [0, 9, 18, 27, 36, 45, 54, 63]


def main():
    cfg = workloads.GL_TRANSIENT
    L, _ = gl_operator(cfg["N"], cfg["mu0"], cfg["mu2"])
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"])
    F0 = workloads.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], cfg["N"])
    a, ad = stepped_applies(L, cfg["h"], w0, dw, "transient", tail=cfg["tail"])
    t = time.perf_counter()
    gains, V, U, hist = block_power_iteration(a, ad, F0, cfg["iters"])
    dt = time.perf_counter() - t
    out = dict(workload=cfg["name"], N=cfg["N"], mu0=cfg["mu0"], mu2=cfg["mu2"], h=cfg["h"], omega0=w0, domega=dw,
               P=P, tail=cfg["tail"], n_omega=cfg["n_omega"], k=cfg["k"], iters=cfg["iters"], seed=cfg["seed"],
               oracle_seconds=dt,
               gains=gains.tolist(),
               hist_rayleigh_ritz=hist[..., 0].tolist(), hist_norm_ratio=hist[..., 1].tolist(),
               sampled=SAMPLED,
               V_re=V[SAMPLED].real.tolist(), V_im=V[SAMPLED].imag.tolist(),
               U_re=U[SAMPLED].real.tolist(), U_im=U[SAMPLED].imag.tolist())
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, "oracle %.1f s" % dt, "gains at the band edges and centre:",
          gains[0, 0], gains[32, 0], gains[-1, 0])


if __name__ == "__main__":
    main()
