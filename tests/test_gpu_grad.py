"""GPU parity of the reverse mode (resolvent_apply_backward, the torch.autograd function) against the CPU oracle.

The oracle's references are the conjugate transpose of the time-stepped run's transfer matrix (assembled from
runs on unit forcings) for the forcing gradient, and central differences of the stepped objective
J(mu) = Re sum conj(G) run(L0 + diag(mu), F) for the reaction-field gradient.  Tolerances: the forcing gradient is
linear algebra in FP64 on both sides (different order only): 1e-10 of its largest entry; the mu gradient is
compared with second-order central differences (step 1e-5): 1e-6 of its largest entry.  A mixed-precision
operator's backward computes in FP64 on FP32-rounded inputs; with FP64 rows (resolvent_op_set_backward_rows) its
bounds are 1e-5 and 1e-6, with the default FP32 rows every stored state, stage value and adjoint state is rounded
to FP32 (2^-24 relative), and over the few hundred steps of these runs those roundings add up to at most a few
1e-6 of the largest entry (measured values are printed): 1e-4 for both gradients, the mixed-precision bound.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from _helpers import gpu_tensor, say
from oracle import dense as O_dense
from oracle import gradient as O_grad
from oracle import operators as O_ops
from oracle import stepping as O_st

pytestmark = pytest.mark.gpu

XL_T, XR_T = -15.0, 15.0
WAKE = dict(amp=0.5, delta=2.0, y0=0.2, z0=-0.3)


def forcing(seed, nw, k, n):
    g = np.random.default_rng(seed)
    return g.standard_normal((nw, k, n)) + 1j * g.standard_normal((nw, k, n))


def to_np(t):
    return t.cpu().numpy().astype(np.complex128)


def maxrel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def gpu_gl(n, mu0, h, precision="fp64", xl=XL_T, xr=XR_T):
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import gl_coefficients
    lo, d, up = gl_coefficients(n, mu0, -0.01, xl=xl, xr=xr)
    return ResolventOp.tridiagonal(lo, d, up, h, precision=precision)


def backward(op, F, G, grid, run, ckpt, dtype=None):
    import torch
    fg, mg = op.apply_backward(gpu_tensor(F, dtype), gpu_tensor(G, dtype), grid, run, checkpoint_every=ckpt)
    torch.cuda.synchronize()
    op.check()
    return to_np(fg), mg.cpu().numpy()


RUNS = {"transient": dict(tail=90), "periodic": dict(periods=3, stride=6)}


@pytest.mark.parametrize("method,ckpt", [("transient", 1), ("transient", 7), ("transient", 0), ("transient", 1000),
                                         ("periodic", 7), ("periodic", 0)])
def test_gl_backward_matches_oracle(method, ckpt):
    say("case: GL N=40 backward", method, "checkpoint_every", ckpt)
    n, h, P, nw, k, w0 = 40, 0.1, 60, 3, 2, -0.4
    dw = 2 * np.pi / (P * h)
    op = gpu_gl(n, 0.2, h)
    F, G = forcing(41, nw, k, n), forcing(42, nw, k, n)
    fg, mg = backward(op, F, G, op.grid(w0, dw, nw), op.run(method, **RUNS[method]), ckpt)
    L0 = O_ops.gl_operator(n, 0.2, -0.01, xl=XL_T, xr=XR_T)[0]
    ref_f = O_grad.stepped_vjp(L0, h, w0, dw, G, method, **RUNS[method])
    ref_mu = O_grad.stepped_mu_gradient(L0, np.zeros(n), h, w0, dw, F, G, method, **RUNS[method])
    e = (maxrel(fg, ref_f), maxrel(mg, ref_mu))
    say("  f_grad err %.3e  mu_grad err %.3e" % e)
    assert e[0] < 1e-10 and e[1] < 1e-6


@pytest.mark.parametrize("ckpt", [64, 3])
def test_gl_backward_several_projection_groups(ckpt):
    """300 steps: the forcing gradient projects the lambda rows of up to 256 steps at a time, so checkpoints every
    64 steps make groups of four segments and one ragged group (64 64 64 64 | 44), every 3 steps groups of 85
    segments (255 | 45 rows)."""
    say("case: GL N=40 backward, periodic 5 periods (300 steps), checkpoint_every", ckpt)
    n, h, P, nw, k, w0 = 40, 0.1, 60, 3, 2, -0.4
    dw = 2 * np.pi / (P * h)
    run = dict(periods=5, stride=6)
    op = gpu_gl(n, 0.2, h)
    F, G = forcing(57, nw, k, n), forcing(58, nw, k, n)
    fg, mg = backward(op, F, G, op.grid(w0, dw, nw), op.run("periodic", **run), ckpt)
    L0 = O_ops.gl_operator(n, 0.2, -0.01, xl=XL_T, xr=XR_T)[0]
    ref_f = O_grad.stepped_vjp(L0, h, w0, dw, G, "periodic", **run)
    ref_mu = O_grad.stepped_mu_gradient(L0, np.zeros(n), h, w0, dw, F, G, "periodic", **run)
    e = (maxrel(fg, ref_f), maxrel(mg, ref_mu))
    say("  f_grad err %.3e  mu_grad err %.3e" % e)
    assert e[0] < 1e-10 and e[1] < 1e-6


def test_gl_backward_spans_several_workgroups():
    # N = 300: two 256-wide blocks of the stage kernels with a ragged tail; mu checked along random directions.
    say("case: GL N=300 on [-50, 50] backward, periodic, checkpoint_every 16")
    n, h, P, nw, k, w0 = 300, 0.02, 80, 3, 2, -0.3
    dw = 2 * np.pi / (P * h)
    run = dict(periods=2, stride=8)
    op = gpu_gl(n, 0.2, h, xl=-50.0, xr=50.0)
    F, G = forcing(43, nw, k, n), forcing(44, nw, k, n)
    fg, mg = backward(op, F, G, op.grid(w0, dw, nw), op.run("periodic", **run), 16)
    L0 = O_ops.gl_operator(n, 0.2, -0.01, xl=-50.0, xr=50.0)[0]
    ref_f = O_grad.stepped_vjp(L0, h, w0, dw, G, "periodic", **run)
    say("  f_grad err %.3e" % maxrel(fg, ref_f))
    assert maxrel(fg, ref_f) < 1e-10
    rng = np.random.default_rng(45)
    for _ in range(2):
        d = rng.standard_normal(n)
        fd = O_grad.stepped_mu_directional(L0, np.zeros(n), d, h, w0, dw, F, G, "periodic", **run)
        say("  directional: gpu %.12e fd %.12e" % (float(mg @ d), fd))
        assert abs(mg @ d - fd) < 1e-6 * np.abs(mg).sum() * np.abs(d).max()


@pytest.mark.parametrize("rows", ["fp32", "fp64"])
def test_gl_backward_mixed_precision_operator(rows):
    import torch
    say("case: GL N=40 backward, mixed-precision operator,", rows, "rows")
    n, h, P, nw, k, w0 = 40, 0.1, 60, 3, 1, 0.2
    dw = 2 * np.pi / (P * h)
    op = gpu_gl(n, 0.2, h, "mixed")
    if rows == "fp64":
        op.set_backward_rows(True)
    F = forcing(46, nw, k, n).astype(np.complex64).astype(np.complex128)
    G = forcing(47, nw, k, n).astype(np.complex64).astype(np.complex128)
    fg, mg = backward(op, F, G, op.grid(w0, dw, nw), op.run("transient", tail=90), 0, torch.complex64)
    L0 = O_ops.gl_operator(n, 0.2, -0.01, xl=XL_T, xr=XR_T)[0]
    ref_f = O_grad.stepped_vjp(L0, h, w0, dw, G, "transient", tail=90)
    ref_mu = O_grad.stepped_mu_gradient(L0, np.zeros(n), h, w0, dw, F, G, "transient", tail=90)
    e = (maxrel(fg, ref_f), maxrel(mg, ref_mu))
    say("  f_grad err %.3e  mu_grad err %.3e" % e)
    if rows == "fp64":
        assert e[0] < 1e-5 and e[1] < 1e-6
    else:
        assert e[0] < 1e-4 and e[1] < 1e-4


def grid_case(case, h, precision="fp64"):
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr2d_coefficients, adr3d3c_coefficients
    if case == "2d":
        nx, ny = 10, 8
        f = O_ops.adr2d_fields(nx, ny)
        mu = O_ops.adr2d_mu_default(f["X"], f["Y"], base=-0.3, amp=0.08)
        op = ResolventOp.grid_operator("adr2d", nx, ny, 1, adr2d_coefficients(nx, ny, mu=mu), h, precision=precision)
        return op, O_ops.adr2d_operator(nx, ny, mu=mu)[0], 1, nx * ny
    nx, ny, nz = 6, 4, 4
    mu = np.full((nz, ny, nx), -0.2)
    op = ResolventOp.grid_operator("adr3d3c", nx, ny, nz, adr3d3c_coefficients(nx, ny, nz, WAKE, mu=mu), h,
                                   precision=precision)
    return op, O_ops.adr3d3c_operator(nx, ny, nz, WAKE, mu=mu)[0], 3, nx * ny * nz


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_grid_backward_matches_oracle(case):
    say("case: grid", case, "backward, transient, checkpoint_every 9")
    h, P, nw, k, w0 = 0.1, 50, 3, 2, 0.1
    dw = 2 * np.pi / (P * h)
    run = dict(tail=60)
    op, L0, ncomp, nodes = grid_case(case, h)
    F, G = forcing(48, nw, k, op.n), forcing(49, nw, k, op.n)
    fg, mg = backward(op, F, G, op.grid(w0, dw, nw), op.run("transient", **run), 9)
    ref_f = O_grad.stepped_vjp(L0, h, w0, dw, G, "transient", **run)
    say("  f_grad err %.3e" % maxrel(fg, ref_f))
    assert maxrel(fg, ref_f) < 1e-10
    if case == "2d":
        ref_mu = O_grad.stepped_mu_gradient(L0, np.zeros(nodes), h, w0, dw, F, G, "transient", **run)
        say("  mu_grad err %.3e" % maxrel(mg, ref_mu))
        assert maxrel(mg, ref_mu) < 1e-6
    else:
        rng = np.random.default_rng(50)
        for _ in range(2):
            d = rng.standard_normal(nodes)
            fd = O_grad.stepped_mu_directional(L0, np.zeros(nodes), d, h, w0, dw, F, G, "transient", ncomp=ncomp,
                                               **run)
            say("  directional: gpu %.12e fd %.12e" % (float(mg @ d), fd))
            assert abs(mg @ d - fd) < 1e-6 * np.abs(mg).sum() * np.abs(d).max()


def test_grid3d_periodic_backward_checkpoint_64():
    """The 3-D gradient pattern of the periodic method: three periods of 50 steps with a checkpoint every 64 steps
    (three segments, the last one ragged).  Forcing gradient against the oracle's stepped VJP, mu gradient along
    random directions against central differences of the oracle's objective."""
    say("case: grid 3d backward, periodic (3 periods, stride 5), checkpoint_every 64")
    h, P, nw, k, w0 = 0.1, 50, 3, 2, 0.1
    dw = 2 * np.pi / (P * h)
    run = dict(periods=3, stride=5)
    op, L0, ncomp, nodes = grid_case("3d", h)
    F, G = forcing(54, nw, k, op.n), forcing(55, nw, k, op.n)
    fg, mg = backward(op, F, G, op.grid(w0, dw, nw), op.run("periodic", **run), 64)
    ref_f = O_grad.stepped_vjp(L0, h, w0, dw, G, "periodic", **run)
    say("  f_grad err %.3e" % maxrel(fg, ref_f))
    assert maxrel(fg, ref_f) < 1e-10
    rng = np.random.default_rng(56)
    for _ in range(2):
        d = rng.standard_normal(nodes)
        fd = O_grad.stepped_mu_directional(L0, np.zeros(nodes), d, h, w0, dw, F, G, "periodic", ncomp=ncomp, **run)
        say("  directional: gpu %.12e fd %.12e" % (float(mg @ d), fd))
        assert abs(mg @ d - fd) < 1e-6 * np.abs(mg).sum() * np.abs(d).max()


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_grid_mixed_backward_fp32_rows_checkpoint_64(case):
    """Mixed-precision grid operators with the default FP32 rows (the form that lets the full 3-D grid fit): the
    periodic pattern of three periods of 50 steps with a checkpoint every 64 steps.  Forcing gradient against the
    oracle's stepped VJP and mu gradient along random directions against central differences of the oracle's FP64
    objective, both to the mixed-precision bound 1e-4."""
    import torch
    say("case: grid", case, "mixed backward, FP32 rows, periodic (3 periods, stride 5), checkpoint_every 64")
    h, P, nw, k, w0 = 0.1, 50, 3, 2, 0.1
    dw = 2 * np.pi / (P * h)
    run = dict(periods=3, stride=5)
    op, L0, ncomp, nodes = grid_case(case, h, "mixed")
    F = forcing(61, nw, k, op.n).astype(np.complex64).astype(np.complex128)
    G = forcing(62, nw, k, op.n).astype(np.complex64).astype(np.complex128)
    fg, mg = backward(op, F, G, op.grid(w0, dw, nw), op.run("periodic", **run), 64, torch.complex64)
    ref_f = O_grad.stepped_vjp(L0, h, w0, dw, G, "periodic", **run)
    say("  f_grad err %.3e" % maxrel(fg, ref_f))
    assert maxrel(fg, ref_f) < 1e-4
    rng = np.random.default_rng(63)
    for _ in range(2):
        d = rng.standard_normal(nodes)
        fd = O_grad.stepped_mu_directional(L0, np.zeros(nodes), d, h, w0, dw, F, G, "periodic", ncomp=ncomp, **run)
        say("  directional: gpu %.12e fd %.12e" % (float(mg @ d), fd))
        assert abs(mg @ d - fd) < 1e-4 * np.abs(mg).sum() * np.abs(d).max()


@pytest.mark.parametrize("case,precision", [("gl", "fp64"), ("3d", "fp64"), ("3d", "mixed")])
def test_backward_in_column_chunks_matches_all_columns(case, precision, monkeypatch):
    """When the rows of all k columns do not fit, the reverse mode runs the columns in chunks (they evolve
    independently, and the mu gradient sums over them).  Chunks of one column and of two (the last one ragged),
    forced through RESOLVENT_BACKWARD_COLUMNS, against all three columns at once: the same arithmetic up to the
    projection's and the column sum's order (1e-12 in FP64, 1e-6 with FP32 rows), and the forcing gradient against
    the oracle."""
    import torch
    say("case: backward in column chunks,", case, precision)
    h, P, nw, k, w0 = 0.1, 50, 3, 3, 0.1
    dw = 2 * np.pi / (P * h)
    run = dict(periods=2, stride=5)
    if case == "gl":
        op = gpu_gl(40, 0.2, h, precision)
        L0 = O_ops.gl_operator(40, 0.2, -0.01, xl=XL_T, xr=XR_T)[0]
    else:
        op, L0, _, _ = grid_case(case, h, precision)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    F = forcing(64, nw, k, op.n).astype(np.complex64).astype(np.complex128)
    G = forcing(65, nw, k, op.n).astype(np.complex64).astype(np.complex128)
    grid, rn = op.grid(w0, dw, nw), op.run("periodic", **run)
    monkeypatch.delenv("RESOLVENT_BACKWARD_COLUMNS", raising=False)
    whole = backward(op, F, G, grid, rn, 16, dt)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for kc in ("1", "2"):
        monkeypatch.setenv("RESOLVENT_BACKWARD_COLUMNS", kc)
        part = backward(op, F, G, grid, rn, 16, dt)
        e = (maxrel(part[0], whole[0]), maxrel(part[1], whole[1]))
        say("  chunks of %s: f_grad %.3e  mu_grad %.3e" % (kc, e[0], e[1]))
        assert e[0] < tol and e[1] < tol
    ref = O_grad.stepped_vjp(L0, h, w0, dw, G, "periodic", **run)
    say("  f_grad err %.3e" % maxrel(whole[0], ref))
    assert maxrel(whole[0], ref) < (1e-10 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("case", ["gl", "2d", "3d", "3d-mixed"])
def test_forcing_gradient_alone_skips_the_forward_trajectory(case):
    """Without the mu gradient the reverse mode runs the adjoint recursion alone (no forward march, checkpoints or
    recomputation: lambda does not depend on the trajectory).  Its forcing gradient must equal the one computed
    beside the mu gradient (to rounding), and match the oracle's stepped VJP.  The mixed 3-D operator runs that
    recursion as lambda_s = P(Z^H) lambda_{s+1} + seed_s with the forward march's fused FP32 step, against the
    FP64-arithmetic stage kernels beside the mu gradient: 1e-5 between the two, 1e-4 against the oracle."""
    import torch
    say("case: forcing gradient without mu,", case)
    h, P, nw, k, w0 = 0.1, 50, 3, 2, 0.1
    dw = 2 * np.pi / (P * h)
    run = dict(periods=2, stride=5)
    mixed = case.endswith("mixed")
    if case == "gl":
        op = gpu_gl(40, 0.2, h)
        L0 = O_ops.gl_operator(40, 0.2, -0.01, xl=XL_T, xr=XR_T)[0]
    else:
        op, L0, _, _ = grid_case(case.split("-")[0], h, "mixed" if mixed else "fp64")
    F, G = forcing(59, nw, k, op.n), forcing(60, nw, k, op.n)
    dt = None
    if mixed:
        F = F.astype(np.complex64).astype(np.complex128)
        G = G.astype(np.complex64).astype(np.complex128)
        dt = torch.complex64
    grid, rn = op.grid(w0, dw, nw), op.run("periodic", **run)
    f, g = gpu_tensor(F, dt), gpu_tensor(G, dt)
    fg_both, _ = op.apply_backward(f, g, grid, rn, checkpoint_every=16)
    fg_alone, mg = op.apply_backward(f, g, grid, rn, checkpoint_every=16, want_mu=False)
    torch.cuda.synchronize()
    op.check()
    assert mg is None
    say("  alone vs with mu: %.3e" % maxrel(to_np(fg_alone), to_np(fg_both)))
    # same recursion; only the projection grouping (and, mixed, the arithmetic precision) may differ
    assert maxrel(to_np(fg_alone), to_np(fg_both)) < (1e-5 if mixed else 1e-13)
    ref = O_grad.stepped_vjp(L0, h, w0, dw, G, "periodic", **run)
    say("  f_grad err %.3e" % maxrel(to_np(fg_alone), ref))
    assert maxrel(to_np(fg_alone), ref) < (1e-4 if mixed else 1e-10)


def test_grid_backward_spans_several_tiles():
    """The fused 2-D forward step of the reverse mode works on 64 x 16 tiles with halos taken from neighbouring
    tiles: a 150 x 40 grid (three ragged tiles in each direction).  The forcing gradient is checked by the exact
    duality <A^H G, d> = <G, A d> of the discrete run against the oracle's forward run, the mu gradient along random
    directions against central differences of the oracle's objective."""
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr2d_coefficients
    say("case: grid 2d backward on 150 x 40 (several fused-step tiles), transient, checkpoint_every 7")
    nx, ny, h, P, nw, k, w0 = 150, 40, 0.1, 40, 3, 2, 0.1
    dw = 2 * np.pi / (P * h)
    run = dict(tail=30)
    f = O_ops.adr2d_fields(nx, ny)
    mu = O_ops.adr2d_mu_default(f["X"], f["Y"], base=-0.3, amp=0.08)
    op = ResolventOp.grid_operator("adr2d", nx, ny, 1, adr2d_coefficients(nx, ny, mu=mu), h)
    L0 = O_ops.adr2d_operator(nx, ny, mu=mu)[0]
    F, G = forcing(51, nw, k, op.n), forcing(52, nw, k, op.n)
    fg, mg = backward(op, F, G, op.grid(w0, dw, nw), op.run("transient", **run), 7)
    rng = np.random.default_rng(53)
    D = rng.standard_normal((nw, k, op.n)) + 1j * rng.standard_normal((nw, k, op.n))
    AD = O_st.run(L0, h, w0, dw, D, "transient", **run)
    lhs, rhs = np.vdot(fg, D), np.vdot(G, AD)
    say("  duality: <A^H G, d> %s  <G, A d> %s" % (lhs, rhs))
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)
    for _ in range(2):
        d = rng.standard_normal(nx * ny)
        fd = O_grad.stepped_mu_directional(L0, np.zeros(nx * ny), d, h, w0, dw, F, G, "transient", **run)
        say("  directional: gpu %.12e fd %.12e" % (float(mg @ d), fd))
        assert abs(mg @ d - fd) < 1e-6 * np.abs(mg).sum() * np.abs(d).max()


def test_autograd_gain_objective_matches_oracle():
    # J = sum_j c_j ||u_j||, u = R(mu) V through the torch.autograd function; gradients against the oracle's
    # (forcing: A^H applied to dJ/du; mu: directional central differences of the same J).
    import torch
    from paper_2008_10904_amd import resolvent_apply
    from paper_2008_10904_amd.operators import gl_coefficients
    say("case: autograd J = sum c_j ||u_j||, GL N=40, periodic")
    n, h, P, nw, w0 = 40, 0.1, 60, 3, -0.4
    dw = 2 * np.pi / (P * h)
    run = dict(periods=3, stride=6)
    c = np.array([1.0, 0.5, 2.0])
    op = gpu_gl(n, 0.2, h)
    base = gl_coefficients(n, 0.2, -0.01, xl=XL_T, xr=XR_T)[1]
    V = forcing(51, nw, 1, n)
    f = gpu_tensor(V).requires_grad_(True)
    mu = torch.zeros(n, dtype=torch.float64, requires_grad=True)
    u = resolvent_apply(f, mu, op, op.grid(w0, dw, nw), op.run("periodic", **run), base)
    J = (torch.from_numpy(c).cuda() * torch.linalg.vector_norm(u[:, 0, :], dim=-1)).sum()
    J.backward()
    torch.cuda.synchronize()
    L0 = O_ops.gl_operator(n, 0.2, -0.01, xl=XL_T, xr=XR_T)[0]
    U = O_st.run(L0, h, w0, dw, V, "periodic", **run)
    Jref = float(np.sum(c * np.linalg.norm(U[:, 0, :], axis=-1)))
    say("  J gpu %.14e oracle %.14e" % (J.item(), Jref))
    assert abs(J.item() - Jref) < 1e-10 * Jref
    Gu = c[:, None, None] * U / np.linalg.norm(U, axis=-1, keepdims=True)  # dJ/du (dJ/dRe + i dJ/dIm)
    ref_f = O_grad.stepped_vjp(L0, h, w0, dw, Gu, "periodic", **run)
    say("  f.grad err %.3e" % maxrel(to_np(f.grad), ref_f))
    assert maxrel(to_np(f.grad), ref_f) < 1e-10

    def Jmu(m):
        L = (L0 + sp.diags(m)).tocsr()
        Um = O_st.run(L, h, w0, dw, V, "periodic", **run)
        return float(np.sum(c * np.linalg.norm(Um[:, 0, :], axis=-1)))

    rng = np.random.default_rng(52)
    g = mu.grad.numpy()
    for _ in range(2):
        d = rng.standard_normal(n)
        fd = O_grad.central_difference_directional(Jmu, np.zeros(n), d, 1e-5)
        say("  directional: gpu %.12e fd %.12e" % (float(g @ d), fd))
        assert abs(g @ d - fd) < 1e-6 * np.abs(g).sum() * np.abs(d).max()


def test_leading_gain_gradient_tends_to_continuous_sensitivity():
    # V = leading force mode of the RK4 steady-state resolvent, J = ||R_d V|| = sigma_1: in a long periodic run the
    # autograd mu gradient approaches sigma_1^2 Re(conj(v_1) u_1) of the continuous resolvent (RK4 error h^4).
    import torch
    from paper_2008_10904_amd import resolvent_apply
    from paper_2008_10904_amd.operators import gl_coefficients
    say("case: leading-gain sensitivity, GL N=32, h=0.05, 14 periods")
    n, h, P, w = 32, 0.05, 400, -0.2
    dw = 2 * np.pi / (P * h)
    L0 = O_ops.gl_operator(n, 0.2, -0.01, xl=XL_T, xr=XR_T)[0]
    v1 = O_dense.gains_and_modes(O_dense.resolvent_rk4(L0, w, h), 1)[2][:, 0]
    op = gpu_gl(n, 0.2, h)
    base = gl_coefficients(n, 0.2, -0.01, xl=XL_T, xr=XR_T)[1]
    mu = torch.zeros(n, dtype=torch.float64, requires_grad=True)
    u = resolvent_apply(gpu_tensor(v1[None, None, :]), mu, op, op.grid(w, dw, 1), op.run("periodic", periods=14), base)
    J = torch.linalg.vector_norm(u)
    J.backward()
    cf = O_grad.leading_gain_sensitivity(L0, w)
    err = np.linalg.norm(mu.grad.numpy() - cf) / np.linalg.norm(cf)
    say("  rel err vs closed form %.3e" % err)
    assert err < 1e-4


def test_backward_argument_errors():
    from paper_2008_10904_amd import ResolventError
    say("case: backward argument errors")
    op = gpu_gl(16, 0.2, 0.1)
    F = gpu_tensor(forcing(53, 2, 1, 16))
    grid = op.grid(0.0, 2 * np.pi / 6.0, 2)
    with pytest.raises(ResolventError):
        op.apply_backward(F, F, grid, op.run("transient", tail=10), checkpoint_every=-1)
    with pytest.raises(ResolventError):
        op.apply_backward(F, F, op.grid(0.0, 0.123456, 2), op.run("transient", tail=10))
