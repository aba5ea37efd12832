"""Parity at the benchmark's full sizes, in the launch configuration bench.py times (default stepper plan for the
N = 2000 workload, tuned plan for the batched one, whole-period forcing tables), on sampled outputs that the
oracle computes one by one.  After its settle periods the periodic method has reached the RK4 steady state (the
transient is below e^-40 for these operators), so u_hat_j = R_d(w_j) F_j and z_hat_j = R_d(w_j)^H G_j for every
sampled frequency j, with R_d from the oracle's dense solve.  Tolerances as for the small parity tests: 1e-10 per
response vector in FP64, 1e-3 in mixed precision."""
import gc

import numpy as np
import pytest

from _helpers import gpu_tensor, say
from oracle import dense as O_dense
from oracle import operators as O_ops

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def release():
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gl_periodic_n2000_full_size(precision, monkeypatch):
    import torch
    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import gl_coefficients, snap_grid
    monkeypatch.delenv("RESOLVENT_STEP1D", raising=False)
    cfg = W.GL_PERIODIC
    say("case: full-size GL N=2000 periodic apply/adjoint,", precision)
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"], cfg["stride"])
    F = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], cfg["N"])
    G = W.random_forcing(cfg["seed"] + 100, cfg["n_omega"], cfg["k"], cfg["N"])
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    lo, d, up = gl_coefficients(cfg["N"], cfg["mu0"], cfg["mu2"])
    op = ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision=precision)
    grid = op.grid(w0, dw, cfg["n_omega"])
    run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
    u = op.apply(gpu_tensor(F, dt), grid, run).cpu().numpy()
    z = op.adjoint_apply(gpu_tensor(G, dt), grid, run).cpu().numpy()
    op.check()
    del op
    release()
    L, _ = O_ops.gl_operator(cfg["N"], cfg["mu0"], cfg["mu2"])
    tol = 1e-10 if precision == "fp64" else 1e-3
    for j in (0, 101, 255):
        Rd = O_dense.resolvent_rk4(L, w0 + j * dw, cfg["h"])
        eu = max(rel(u[j, c], Rd @ F[j, c]) for c in range(cfg["k"]))
        ez = max(rel(z[j, c], Rd.conj().T @ G[j, c]) for c in range(cfg["k"]))
        say("  j=%d  apply %.2e  adjoint %.2e" % (j, eu, ez))
        assert eu < tol and ez < tol


def test_gl_batched_64_full_size(tmp_path, monkeypatch):
    import torch
    import workloads as W
    from paper_2008_10904_amd import ResolventOp, autotune
    from paper_2008_10904_amd.operators import gl_batched_coefficients, snap_grid
    monkeypatch.delenv("RESOLVENT_STEP1D", raising=False)
    cfg = W.GL_BATCHED
    say("case: full-size batched GL (64 instances) periodic apply, mixed, tuned plan")
    inst = W.batched_instances()
    lo, d, up, off = gl_batched_coefficients(inst)
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"], cfg["stride"])
    F = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], int(off[-1]))
    release()
    op = ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision="mixed", offsets=off)
    plan, _ = autotune.tuned(op, cfg["k"], path=str(tmp_path / "plans.json"))
    u = op.apply(gpu_tensor(F, torch.complex64), op.grid(w0, dw, cfg["n_omega"]),
                 op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])).cpu().numpy()
    op.check()
    del op
    release()
    say("  plan", plan)
    sizes = [n for n, _, _ in inst]
    picks = [int(np.argmin(sizes)), len(inst) // 2, int(np.argmax(sizes))]
    for m, j in zip(picks, (0, 64, 127)):
        n, mu0, mu2 = inst[m]
        L, _ = O_ops.gl_operator(n, mu0, mu2)
        sl = slice(int(off[m]), int(off[m + 1]))
        Rd = O_dense.resolvent_rk4(L, w0 + j * dw, cfg["h"])
        e = max(rel(u[j, c, sl], Rd @ F[j, c, sl]) for c in range(cfg["k"]))
        say("  instance %d (N=%d) j=%d  apply %.2e" % (m, n, j, e))
        assert e < 1e-3
