"""Parity at the benchmark's full sizes, in the launch configuration bench.py times (default stepper plan for the
N = 2000 workload, tuned plan for the batched one, whole-period forcing tables, the 2-D step kernel on the full
1024 x 512 grid), on sampled outputs that the oracle computes one by one, or, where R_d cannot be formed, through
the steady-state equation e^{i w h} u - P(Z) u = h Q_w(Z) f evaluated by the oracle's matrix-vector products.  After its settle periods the periodic method has reached the RK4 steady state (the
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
    """The headline configuration at full size (N = 2000, k = 4, 256 frequencies, 10 periods of 267,008 steps):
    apply and adjoint at three frequencies against the oracle's dense R_d(w) and R_d(w)^H, and at every frequency
    and column through the normwise backward error of the RK4 steady-state equation (1e-10 FP64, 8e-6 mixed)."""
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
    # Every frequency and column through the RK4 steady-state equation (e^{iwh} - P(Z)) u = h Q_w(Z) f (sparse
    # products of the oracle's operator), the adjoint through R_d(w)^H = R_d(-w; L^H).  The measure is the normwise
    # backward error |r| / (|u| + |P(Z) u| + |h Q_w(Z) f|): the operator is stiff (|h L| ~ 1.6), so the residual
    # relative to |h Q f| alone would multiply the state's rounding by |L| times the gain.  A response at a wrong
    # frequency or column gives an error of order one.
    LH = L.conj().T
    Fc = F.astype(np.complex64).astype(np.complex128) if precision == "mixed" else F
    Gc = G.astype(np.complex64).astype(np.complex128) if precision == "mixed" else G
    hh, zero = cfg["h"], np.zeros(cfg["N"], np.complex128)

    def backward_error(Lop, w, x, rhs):
        r = O_dense.rk4_steady_residual(Lop, w, hh, x, rhs)
        r0 = O_dense.rk4_steady_residual(Lop, w, hh, x, zero)     # e^{iwh} x - P(Z) x
        q = O_dense.rk4_steady_residual(Lop, w, hh, zero, rhs)    # -h Q_w(Z) f
        px = np.exp(1j * w * hh) * x - r0
        return np.linalg.norm(r) / (np.linalg.norm(x) + np.linalg.norm(px) + np.linalg.norm(q))

    worst_u = worst_z = 0.0
    for j in range(cfg["n_omega"]):
        w = w0 + j * dw
        for c in range(cfg["k"]):
            worst_u = max(worst_u, backward_error(L, w, u[j, c].astype(np.complex128), Fc[j, c]))
            worst_z = max(worst_z, backward_error(LH, -w, z[j, c].astype(np.complex128), Gc[j, c]))
    say("  all %d frequencies x %d columns: steady-state backward error apply %.2e  adjoint %.2e" % (
        cfg["n_omega"], cfg["k"], worst_u, worst_z))
    # A response one frequency bin off gives about h dw / 2 = 1.2e-5 here (|e^{iw'h} - e^{iwh}| |u| over about
    # 2 |u|), so the mixed bound sits below that: measured 3.7e-6 (apply 2.1e-6), the FP32 state and forcing rows
    # rounded at 6e-8 and multiplied by the stiff operator's terms; FP64 measured 5e-14.
    be_tol = 1e-10 if precision == "fp64" else 8e-6
    assert worst_u < be_tol and worst_z < be_tol


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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adr2d_1024x512_full_size_steady_state(precision):
    """The 2-D operator on its full grid, periodic method (P = 500, 150 periods: the numerical abscissa of L is at
    most max(mu - sponge) = -0.02, so the transient is below e^-30 when the last period is projected).  Every
    frequency and column of the response must satisfy the RK4 steady-state equation; the residual is relative to
    the forcing term h Q_w(Z) f."""
    import torch
    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr2d_coefficients
    cfg = W.ADR2D
    nx, ny, h, k = cfg["nx"], cfg["ny"], cfg["h"], cfg["k"]
    P, periods, nw, w0 = 500, 150, 4, 0.2
    dw = 2 * np.pi / (P * h)
    say("case: full-size 2-D %d x %d periodic apply (P=%d, %d periods), %s" % (nx, ny, P, periods, precision))
    c = adr2d_coefficients(nx, ny, Re=cfg["Re"], mu_base=cfg["mu_base"], mu_amp=cfg["mu_amp"], mu_xc=cfg["mu_xc"],
                           mu_w2=cfg["mu_w2"], nu_s=cfg["nu_s"])
    op = ResolventOp.grid_operator("adr2d", nx, ny, 1, c, h, precision=precision)
    F = W.random_forcing(cfg["seed"], nw, k, nx * ny)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    u = op.apply(gpu_tensor(F, dt), op.grid(w0, dw, nw), op.run("periodic", periods=periods, stride=1))
    u = u.cpu().numpy().astype(np.complex128)
    op.check()
    del op
    release()
    f = O_ops.adr2d_fields(nx, ny, nu_s=cfg["nu_s"])
    mu = O_ops.adr2d_mu_default(f["X"], f["Y"], base=cfg["mu_base"], amp=cfg["mu_amp"], xc=cfg["mu_xc"],
                                width2=cfg["mu_w2"])
    L, _ = O_ops.adr2d_operator(nx, ny, Re=cfg["Re"], mu=mu, nu_s=cfg["nu_s"])
    Fc = F.astype(np.complex64).astype(np.complex128) if precision == "mixed" else F
    tol = 1e-10 if precision == "fp64" else 1e-4  # measured: 3e-15 and 1.5e-6
    worst = 0.0
    for j in range(nw):
        w = w0 + j * dw
        for col in range(k):
            r = O_dense.rk4_steady_residual(L, w, h, u[j, col], Fc[j, col])
            q = O_dense.rk4_steady_residual(L, w, h, np.zeros_like(u[j, col]), Fc[j, col])  # -h Q_w(Z) f
            e = float(np.linalg.norm(r) / np.linalg.norm(q))
            worst = max(worst, e)
            say("  j=%d col=%d  residual %.2e" % (j, col, e))
    assert worst < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adr3d3c_256x128x128_full_size_steady_state(precision):
    """The 3-D three-component operator on its full grid with the workload's k = 3, periodic method (P = 100,
    100 periods).  Its eigenvalues are those of the three diagonal blocks (the shear coupling only feeds u from v
    and w), whose abscissa is at most mu = -0.05, so the transient is below e^-49 times a polynomial factor when the
    last period is projected.  Two frequencies, every column, against the RK4 steady-state equation."""
    import torch
    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr3d3c_coefficients
    cfg = W.ADR3D
    nx, ny, nz, h, k = cfg["nx"], cfg["ny"], cfg["nz"], cfg["h"], cfg["k"]
    P, periods, nw, w0 = 100, 100, 2, 0.3
    dw = 2 * np.pi / (P * h)
    say("case: full-size 3-D %d x %d x %d periodic apply (P=%d, %d periods), %s" % (nx, ny, nz, P, periods,
                                                                                  precision))
    wake = W.wake_parameters(cfg["seed"])
    mu = np.full((nz, ny, nx), cfg["mu_const"])
    c = adr3d3c_coefficients(nx, ny, nz, wake, Re=cfg["Re"], mu=mu, nu_s=cfg["nu_s"])
    op = ResolventOp.grid_operator("adr3d3c", nx, ny, nz, c, h, precision=precision)
    N = 3 * nx * ny * nz
    F = W.random_forcing(cfg["seed"], nw, k, N, dtype=np.complex64)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    u = op.apply(gpu_tensor(F, dt), op.grid(w0, dw, nw), op.run("periodic", periods=periods, stride=1))
    u = u.cpu().numpy()
    op.check()
    del op
    release()
    L, _ = O_ops.adr3d3c_operator(nx, ny, nz, wake, Re=cfg["Re"], mu=mu, nu_s=cfg["nu_s"])
    tol = 1e-10 if precision == "fp64" else 1e-4
    worst = 0.0
    for j in range(nw):
        w = w0 + j * dw
        for col in range(k):
            f = F[j, col].astype(np.complex128)
            r = O_dense.rk4_steady_residual(L, w, h, u[j, col].astype(np.complex128), f)
            q = O_dense.rk4_steady_residual(L, w, h, np.zeros(N, np.complex128), f)  # -h Q_w(Z) f
            e = float(np.linalg.norm(r) / np.linalg.norm(q))
            worst = max(worst, e)
            say("  j=%d col=%d  residual %.2e" % (j, col, e))
    assert worst < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adr3d3c_256x128x128_full_size_modes(precision):
    """Gains and modes of the block power iteration on the 3-D workload's full grid (k = 3, two frequencies,
    periodic method with P = 100 and 60 periods: the transient is below e^-30 when the last period is projected;
    one iteration in FP64, two in mixed precision so that the amplitude weighting runs).  R_d cannot be formed
    here, so each returned triple is checked through what holds at any size: sigma u = R_d v, i.e. the RK4
    steady-state equation e^{iwh}(sigma u) - P(Z)(sigma u) = h Q_w(Z) v evaluated by the oracle's sparse products
    (relative to h Q_w(Z) v: 1e-10 FP64, 1e-4 mixed); V and U orthonormal per frequency (1e-12, 1e-5); gains
    descending."""
    import torch
    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr3d3c_coefficients
    cfg = W.ADR3D
    nx, ny, nz, h, k = cfg["nx"], cfg["ny"], cfg["nz"], cfg["h"], cfg["k"]
    P, periods, nw, w0 = 100, 60, 2, 0.3
    iters = 1 if precision == "fp64" else 2
    dw = 2 * np.pi / (P * h)
    say("case: full-size 3-D %d x %d x %d modes (P=%d, %d periods, %d iterations), %s" % (nx, ny, nz, P, periods,
                                                                                        iters, precision))
    wake = W.wake_parameters(cfg["seed"])
    mu = np.full((nz, ny, nx), cfg["mu_const"])
    c = adr3d3c_coefficients(nx, ny, nz, wake, Re=cfg["Re"], mu=mu, nu_s=cfg["nu_s"])
    op = ResolventOp.grid_operator("adr3d3c", nx, ny, nz, c, h, precision=precision)
    N = 3 * nx * ny * nz
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    f0 = W.random_forcing_device(cfg["seed"] + 7, nw, k, N, dt, "cuda")
    gains, V, U, _ = op.modes(f0, op.grid(w0, dw, nw), op.run("periodic", periods=periods, stride=1), iters,
                              want_hist=False)
    V = V.cpu().numpy().astype(np.complex128)
    U = U.cpu().numpy().astype(np.complex128)
    op.check()
    del op, f0
    release()
    L, _ = O_ops.adr3d3c_operator(nx, ny, nz, wake, Re=cfg["Re"], mu=mu, nu_s=cfg["nu_s"])
    tol_res, tol_orth = (1e-10, 1e-12) if precision == "fp64" else (1e-4, 1e-5)
    worst_res = worst_orth = 0.0
    for j in range(nw):
        w = w0 + j * dw
        g = gains[0, j]
        say("  j=%d gains %s" % (j, np.array2string(g, precision=6)))
        assert np.all(np.diff(g) <= 0) and np.all(g > 0)
        for M in (V[j], U[j]):
            G = M.conj() @ M.T
            worst_orth = max(worst_orth, float(np.abs(G - np.eye(k)).max()))
        for col in range(k):
            r = O_dense.rk4_steady_residual(L, w, h, g[col] * U[j, col], V[j, col])
            q = O_dense.rk4_steady_residual(L, w, h, np.zeros(N, np.complex128), V[j, col])  # -h Q_w(Z) v
            e = float(np.linalg.norm(r) / np.linalg.norm(q))
            worst_res = max(worst_res, e)
            say("  j=%d col=%d  residual of sigma u = R_d v: %.2e" % (j, col, e))
    say("  worst residual %.2e, worst orthonormality %.2e" % (worst_res, worst_orth))
    assert worst_res < tol_res and worst_orth < tol_orth


def test_adr2d_1024x512_full_size_reverse_mode():
    """The reverse mode at the 2-D workload's full size, in the run the bench times (transient method, 19,949
    forced steps and a tail of 15,000, 128 frequencies, k = 2, default checkpoints), on the FP64 operator.  The
    forcing gradient A^H g must satisfy the duality <A^H g, d> = <g, A d> with the library's own forward apply, and
    at four sampled elements equal conj(<g, A e>) for the unit forcing e (1e-9 of the frequency's rms; measured
    2e-15); the mu gradient must match central differences of J(mu) = Re <g, A(mu) f> from two forward applies with
    the diagonal moved by -+ eps d, along a random direction and along three 32 x 32-node patches (1e-5; measured
    1.9e-7 at most)."""
    import torch
    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr2d_coefficients, snap_grid
    cfg = W.ADR2D
    nx, ny, h, k, nw = cfg["nx"], cfg["ny"], cfg["h"], cfg["k"], cfg["n_omega"]
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], nw, h, cfg["stride"])
    say("case: full-size 2-D %d x %d reverse mode, FP64, transient P=%d tail=%d, %d frequencies" % (
        nx, ny, P, cfg["tail"], nw))
    c = adr2d_coefficients(nx, ny, Re=cfg["Re"], mu_base=cfg["mu_base"], mu_amp=cfg["mu_amp"], mu_xc=cfg["mu_xc"],
                           mu_w2=cfg["mu_w2"], nu_s=cfg["nu_s"])
    op = ResolventOp.grid_operator("adr2d", nx, ny, 1, c, h, precision="fp64")
    N = nx * ny
    grid, run = op.grid(w0, dw, nw), op.run("transient", tail=cfg["tail"])
    f = gpu_tensor(W.random_forcing(cfg["seed"], nw, k, N), torch.complex128)
    g = gpu_tensor(W.random_forcing(cfg["seed"] + 100, nw, k, N), torch.complex128)
    d = gpu_tensor(W.random_forcing(cfg["seed"] + 200, nw, k, N), torch.complex128)
    fg, mg = op.apply_backward(f, g, grid, run)
    ad = op.apply(d, grid, run)
    lhs = complex(torch.vdot(fg.flatten(), d.flatten()).item())
    rhs = complex(torch.vdot(g.flatten(), ad.flatten()).item())
    say("  duality: <A^H g, d> %s  <g, A d> %s  rel %.2e" % (lhs, rhs, abs(lhs - rhs) / abs(rhs)))
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)
    del ad, d
    # Element by element: the forcing gradient at a (frequency, column, node) equals conj(<g, A e>) for the unit
    # forcing e there (A is complex-linear, so J(e) = Re <g, A e> and J(i e) = -Im <g, A e>): one forward apply per
    # sampled element, through the forward march, synthesis and projection instead of the reverse mode.
    node = lambda ix, iy: iy * nx + ix  # noqa: E731
    picks = [(0, 0, node(10, 200)), (64, 1, node(300, 256)), (127, 0, node(1000, 30)), (100, 1, node(512, 500))]
    worst = 0.0
    for j, col, n in picks:
        e = torch.zeros_like(f)
        e[j, col, n] = 1.0
        ref = complex(torch.vdot(g.flatten(), op.apply(e, grid, run).flatten()).item()).conjugate()
        got = complex(fg[j, col, n].item())
        rms = float(torch.linalg.vector_norm(fg[j]).item()) / np.sqrt(fg[j].numel())
        err = abs(got - ref) / rms
        worst = max(worst, err)
        say("  forcing gradient [%d, %d, %d]: %s against %s, error %.2e of the frequency's rms" % (j, col, n, got,
                                                                                              ref, err))
    assert worst < 1e-9
    del fg, e
    mg = mg.cpu().numpy()
    dfield = np.asarray(c["dfield"], np.float64).ravel()
    delta = np.random.default_rng(cfg["seed"] + 300).standard_normal(N)
    eps = 1e-4

    def J(diag):
        op.set_diagonal(diag)
        u = op.apply(f, grid, run)
        return float(torch.vdot(g.flatten(), u.flatten()).real.item())

    fd = (J(dfield + eps * delta) - J(dfield - eps * delta)) / (2 * eps)
    gd = float(mg @ delta)
    say("  mu directional: reverse mode %.12e  central differences %.12e  rel %.2e" % (gd, fd, abs(gd - fd) / abs(fd)))
    assert abs(gd - fd) < 1e-6 * abs(fd)  # measured 5.7e-9: the O(eps^2) truncation of the central difference
    # Local structure of the mu gradient: 32 x 32-node patches (0.2 % of the domain) in the mu bump, in the sponge
    # and near the inflow corner, each against central differences along the patch's indicator.
    for cx, cy in ((256, 256), (960, 256), (40, 40)):
        patch = np.zeros((ny, nx))
        patch[cy - 16:cy + 16, cx - 16:cx + 16] = 1.0
        patch = patch.ravel()
        fdp = (J(dfield + eps * patch) - J(dfield - eps * patch)) / (2 * eps)
        gdp = float(mg @ patch)
        say("  mu on the patch at (%d, %d): reverse mode %.12e  central differences %.12e  rel %.2e" % (
            cx, cy, gdp, fdp, abs(gdp - fdp) / abs(fdp)))
        assert abs(gdp - fdp) < 1e-5 * abs(fdp)
    op.set_diagonal(dfield)
    op.check()
    del op
    release()


def test_adr3d3c_256x128x128_full_grid_reverse_mode_checkpoint_64():
    """The reverse mode on the 3-D workload's full grid (256 x 128 x 128, three components, k = 3) with the
    mixed-precision operator's FP32 rows and a checkpoint every 64 steps, on a short periodic run (4 frequencies,
    P = 64, three periods projected every 8th step of the last: three 64-step segments) so that the FP64 references
    stay cheap.  The forcing gradient must satisfy the duality <A^H g, d> = <g, A d> with A d from the FP64
    operator's apply, and at three sampled elements equal conj(<g, A e>) for the unit forcing e (relative to the
    frequency's rms); the mu gradient must match central differences of J(mu) = Re <g, A(mu) f> from two FP64
    applies with the diagonal moved by -+ eps d, along a random direction and along three 16 x 16 x 16-node
    patches.  Bound: 1e-4 relative, the mixed-precision bound (the FP32 rows round every stored value to 2^-24;
    measured 2e-7 at most)."""
    import torch
    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr3d3c_coefficients
    cfg = W.ADR3D
    nx, ny, nz, h, k = cfg["nx"], cfg["ny"], cfg["nz"], cfg["h"], cfg["k"]
    nw, P, w0 = 4, 64, 0.2
    dw = 2 * np.pi / (P * h)
    say("case: full-grid 3-D %d x %d x %d reverse mode, mixed (FP32 rows), periodic P=%d x 3, checkpoint 64" % (
        nx, ny, nz, P))
    wake = W.wake_parameters(cfg["seed"])
    mu = np.full((nz, ny, nx), cfg["mu_const"])
    c = adr3d3c_coefficients(nx, ny, nz, wake, Re=cfg["Re"], mu=mu, nu_s=cfg["nu_s"])
    N = 3 * nx * ny * nz
    f = W.random_forcing_device(cfg["seed"], nw, k, N, torch.complex64, "cuda")
    g = W.random_forcing_device(cfg["seed"] + 100, nw, k, N, torch.complex64, "cuda")
    opm = ResolventOp.grid_operator("adr3d3c", nx, ny, nz, c, h, precision="mixed")
    grid, run = opm.grid(w0, dw, nw), opm.run("periodic", periods=3, stride=8)
    fg, mg = opm.apply_backward(f, g, grid, run, checkpoint_every=64)
    torch.cuda.synchronize()
    opm.check()
    del opm
    release()
    say("  backward done")
    nodes = nx * ny * nz
    node = lambda comp, ix, iy, iz: comp * nodes + (iz * ny + iy) * nx + ix  # noqa: E731
    picks = [(0, 0, node(0, 40, 64, 64)), (2, 1, node(1, 128, 20, 100)), (3, 2, node(2, 250, 100, 10))]
    fg_picks = [complex(fg[j, col, n].item()) for j, col, n in picks]
    fg_rms = [float(torch.linalg.vector_norm(fg[j].to(torch.complex128)).item()) / np.sqrt(fg[j].numel())
              for j, _, _ in picks]
    d = W.random_forcing_device(cfg["seed"] + 200, nw, k, N, torch.complex64, "cuda")
    lhs = complex(torch.vdot(fg.flatten().to(torch.complex128), d.flatten().to(torch.complex128)).item())
    del fg
    op = ResolventOp.grid_operator("adr3d3c", nx, ny, nz, c, h, precision="fp64")
    f64, g64 = f.to(torch.complex128), g.flatten().to(torch.complex128)
    del f, g
    ad = op.apply(d.to(torch.complex128), grid, run)
    del d
    rhs = complex(torch.vdot(g64, ad.flatten()).item())
    del ad
    say("  duality: <A^H g, d> %s  <g, A d> %s  rel %.2e" % (lhs, rhs, abs(lhs - rhs) / abs(rhs)))
    assert abs(lhs - rhs) < 1e-4 * abs(rhs)
    # Element by element: conj(<g, A e>) for the unit forcing e at sampled (frequency, column, component and node),
    # from the FP64 operator's forward apply.
    for (j, col, n), got, rms in zip(picks, fg_picks, fg_rms):
        e = torch.zeros_like(f64)
        e[j, col, n] = 1.0
        ref = complex(torch.vdot(g64, op.apply(e, grid, run).flatten()).item()).conjugate()
        err = abs(got - ref) / rms
        say("  forcing gradient [%d, %d, %d]: %s against %s, error %.2e of the frequency's rms" % (j, col, n, got,
                                                                                              ref, err))
        assert err < 1e-4
        del e
    mg = mg.cpu().numpy()
    dfield = np.asarray(c["dfield"], np.float64).ravel()
    delta = np.random.default_rng(cfg["seed"] + 300).standard_normal(nx * ny * nz)
    eps = 1e-4

    def J(diag):
        op.set_diagonal(diag)
        u = op.apply(f64, grid, run)
        return float(torch.vdot(g64, u.flatten()).real.item())

    fd = (J(dfield + eps * delta) - J(dfield - eps * delta)) / (2 * eps)
    gd = float(mg @ delta)
    say("  mu directional: reverse mode %.12e  central differences %.12e  rel %.2e" % (gd, fd, abs(gd - fd) / abs(fd)))
    assert abs(gd - fd) < 1e-4 * abs(fd)
    # Local structure: 16 x 16 x 16-node patches (0.1 % of the grid) in the wake, in the sponge and in a corner.
    for cx, cy, cz in ((64, 64, 64), (240, 64, 64), (20, 20, 20)):
        patch = np.zeros((nz, ny, nx))
        patch[cz - 8:cz + 8, cy - 8:cy + 8, cx - 8:cx + 8] = 1.0
        patch = patch.ravel()
        fdp = (J(dfield + eps * patch) - J(dfield - eps * patch)) / (2 * eps)
        gdp = float(mg @ patch)
        say("  mu on the patch at (%d, %d, %d): reverse mode %.12e  central differences %.12e  rel %.2e" % (
            cx, cy, cz, gdp, fdp, abs(gdp - fdp) / abs(fdp)))
        assert abs(gdp - fdp) < 1e-4 * abs(fdp)
    op.set_diagonal(dfield)
    op.check()
    del op, f64, g64
    release()


def test_gl_periodic_n2000_full_size_block_arnoldi(monkeypatch):
    """The Arnoldi line's configuration (N = 2000, k = 4, 256 frequencies, 10 periods per run, 10 blocks of 4
    forcings, FP64, default stepper plan): the four leading gains at sampled frequencies against the singular values
    of the oracle's dense R_d(w_j), to the FP64 gain bound 1e-8 (measured: 6e-11 at most)."""
    import torch
    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import gl_coefficients, snap_grid
    monkeypatch.delenv("RESOLVENT_STEP1D", raising=False)
    cfg = W.GL_PERIODIC
    say("case: full-size GL N=2000 block Arnoldi, 10 blocks of k=4, FP64")
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"], cfg["stride"])
    F = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], cfg["N"])
    lo, d, up = gl_coefficients(cfg["N"], cfg["mu0"], cfg["mu2"])
    op = ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision="fp64")
    grid = op.grid(w0, dw, cfg["n_omega"])
    run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
    gains, _, _, _ = op.krylov(gpu_tensor(F, torch.complex128), grid, run, 10, want_modes=False, want_hist=False)
    op.check()
    del op
    release()
    L, _ = O_ops.gl_operator(cfg["N"], cfg["mu0"], cfg["mu2"])
    worst = 0.0
    for j in (0, 101, 255):
        s = np.linalg.svd(O_dense.resolvent_rk4(L, w0 + j * dw, cfg["h"]), compute_uv=False)[:cfg["k"]]
        e = float(np.abs(gains[0, j] / s - 1).max())
        worst = max(worst, e)
        say("  j=%d  gains %s  rel err %.2e" % (j, np.array2string(gains[0, j], precision=6), e))
    assert worst < 1e-8
