"""The transient-response method's power iteration at its workload's own configuration, against the CPU oracle.

Workload: 1-D Ginzburg-Landau, N = 200, mu0 = 0.30, h = 0.01, 64 frequencies in [-2, 2] (P = 9,896), one forcing
window of P steps followed by a 20,000-step tail, k = 1, 20 iterations (Sec. 2.2 with the power iteration of
App. A, eqs. iteration and powerMethod, normalised per frequency).  The truncated tail couples the frequencies
(leakage, Sec. 2.2), so the oracle must march all 64 of them: its 20 iterations (40 explicit RK4 runs of 29,896
steps) take about three minutes on one core and are stored in tests/golden/gl_transient_reference.json by the
script beside it, which calls only the oracle.  The GPU runs the same iteration from the same seeded start:

* FP64: every gain of every iteration within 1e-8 relative, the force and response modes at the stored frequencies
  within 1e-8 (phase-aligned 2-norm difference of unit vectors);
* mixed precision: every final gain within 1e-4 relative; mode errors are printed.
"""
import json
import os

import numpy as np
import pytest

from _helpers import gpu_tensor, mode_errors, say

REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gl_transient_reference.json")


def reference():
    with open(REF) as f:
        r = json.load(f)
    r["gains"] = np.array(r["gains"])
    r["hist"] = np.array(r["hist_rayleigh_ritz"])
    r["V"] = np.array(r["V_re"]) + 1j * np.array(r["V_im"])
    r["U"] = np.array(r["U_re"]) + 1j * np.array(r["U_im"])
    return r


def run_gpu(precision, iters=None):
    import torch
    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import gl_coefficients, snap_grid
    cfg = W.GL_TRANSIENT
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"])
    F = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], cfg["N"])
    lo, d, up = gl_coefficients(cfg["N"], cfg["mu0"], cfg["mu2"])
    op = ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision=precision, probe=True)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    g, V, U, hist = op.modes(gpu_tensor(F, dt), op.grid(w0, dw, cfg["n_omega"]),
                             op.run("transient", tail=cfg["tail"]), iters or cfg["iters"])
    torch.cuda.synchronize()
    op.check()
    return (w0, dw, P), g[0], V.cpu().numpy().astype(complex), U.cpu().numpy().astype(complex), hist[:, 0]


def test_reference_matches_workload():
    import workloads as W
    from paper_2008_10904_amd.operators import snap_grid
    r = reference()
    cfg = W.GL_TRANSIENT
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"])
    assert (r["N"], r["n_omega"], r["k"], r["iters"], r["tail"], r["P"], r["seed"]) == \
        (cfg["N"], cfg["n_omega"], cfg["k"], cfg["iters"], cfg["tail"], P, cfg["seed"])
    assert abs(r["domega"] - dw) < 1e-15 and r["omega0"] == w0


@pytest.mark.gpu
def test_transient_modes_fp64_match_oracle():
    say("case: transient power iteration, GL N=200, 64 frequencies, P=9896 + 20000 tail, k=1, 20 iterations, FP64")
    r = reference()
    (w0, dw, P), g, V, U, hist = run_gpu("fp64")
    eg = float(np.abs(g / r["gains"] - 1).max())
    eh = float(np.abs(hist[..., 0] / r["hist"] - 1).max())
    js = r["sampled"]
    ev = max(mode_errors(V[j], r["V"][i], r["gains"][j]).max() for i, j in enumerate(js))
    eu = max(mode_errors(U[j], r["U"][i], r["gains"][j]).max() for i, j in enumerate(js))
    say("  gains: band edges %.6f %.6f, peak %.6f" % (g[0, 0], g[-1, 0], g.max()))
    say("  final gain err %.2e, history err %.2e, force-mode err %.2e, response-mode err %.2e" % (eg, eh, ev, eu))
    assert eg < 1e-8 and eh < 1e-8
    assert ev < 1e-8 and eu < 1e-8


@pytest.mark.gpu
def test_transient_modes_mixed_match_oracle():
    say("case: transient power iteration at the same configuration, mixed precision")
    r = reference()
    _, g, V, U, _ = run_gpu("mixed")
    eg = float(np.abs(g / r["gains"] - 1).max())
    js = r["sampled"]
    ev = max(mode_errors(V[j], r["V"][i], r["gains"][j]).max() for i, j in enumerate(js))
    eu = max(mode_errors(U[j], r["U"][i], r["gains"][j]).max() for i, j in enumerate(js))
    say("  final gain err %.2e, force-mode err %.2e, response-mode err %.2e" % (eg, ev, eu))
    assert eg < 1e-4
    assert ev < 1e-2 and eu < 1e-2


def test_reference_first_iteration_is_the_oracles():
    # The stored history is the oracle's: its first iteration (one direct and one adjoint run, about 10 s) is
    # recomputed here and must agree to rounding.
    import workloads as W
    from oracle.iteration import block_power_iteration, stepped_applies
    from oracle.operators import gl_operator
    from oracle.stepping import snap_grid
    r = reference()
    cfg = W.GL_TRANSIENT
    L, _ = gl_operator(cfg["N"], cfg["mu0"], cfg["mu2"])
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"])
    F0 = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], cfg["N"])
    a, ad = stepped_applies(L, cfg["h"], w0, dw, "transient", tail=cfg["tail"])
    g, _, _, _ = block_power_iteration(a, ad, F0, 1)
    assert np.abs(g / r["hist"][0] - 1).max() < 1e-12
