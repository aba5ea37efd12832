"""GPU parity of the 2-D (five-point) and 3-D three-component (seven-point, shear-coupled) paths against the
CPU oracle on small grids, element by element on seeded inputs.  Tolerances as for the 1-D path: FP64 runs
within 1e-10 per frequency vector (only the order of the arithmetic differs), gains within 1e-8; mixed runs
within 1e-3 per vector and 1e-4 per gain."""
import numpy as np
import pytest

from _helpers import gpu_tensor, mode_alignment, per_freq_relerr, say
from oracle import iteration as O_it
from oracle import operators as O_ops
from oracle import stepping as O_st

pytestmark = pytest.mark.gpu

WAKE = dict(amp=0.5, delta=2.0, y0=0.2, z0=-0.3)


def forcing(seed, nw, k, n):
    g = np.random.default_rng(seed)
    return g.standard_normal((nw, k, n)) + 1j * g.standard_normal((nw, k, n))


def to_np(t):
    return t.cpu().numpy().astype(np.complex128)


def mu2d(nx, ny, seed=0):
    f = O_ops.adr2d_fields(nx, ny)
    return O_ops.adr2d_mu_default(f["X"], f["Y"], base=-0.3, amp=0.08)


def make2d(nx, ny, h, precision="fp64", mu=None):
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr2d_coefficients
    mu = mu2d(nx, ny) if mu is None else mu
    c = adr2d_coefficients(nx, ny, mu=mu)
    op = ResolventOp.grid_operator("adr2d", nx, ny, 1, c, h, precision=precision)
    L, _ = O_ops.adr2d_operator(nx, ny, mu=mu)
    return op, L


def make3d(nx, ny, nz, h, precision="fp64", mu=None):
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr3d3c_coefficients
    mu = np.full((nz, ny, nx), -0.2) if mu is None else mu
    c = adr3d3c_coefficients(nx, ny, nz, WAKE, mu=mu)
    op = ResolventOp.grid_operator("adr3d3c", nx, ny, nz, c, h, precision=precision)
    L, _ = O_ops.adr3d3c_operator(nx, ny, nz, WAKE, mu=mu)
    return op, L


CASES = {"2d": lambda p="fp64", mu=None: make2d(24, 16, 0.1, p, mu),
         "3d": lambda p="fp64", mu=None: make3d(12, 8, 8, 0.1, p, mu)}


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_apply_adjoint_and_transient_match_oracle(case):
    import torch
    say("case: grid", case, "apply / adjoint / transient")
    op, L = CASES[case]()
    h, P, nw, k = 0.1, 200, 3, 2
    dw = 2 * np.pi / (P * h)
    F = forcing(21, nw, k, op.n)
    grid = op.grid(0.1, dw, nw)
    up = to_np(op.apply(gpu_tensor(F), grid, op.run("periodic", periods=8, stride=50)))
    za = to_np(op.adjoint_apply(gpu_tensor(F), grid, op.run("periodic", periods=8, stride=50)))
    ut = to_np(op.apply(gpu_tensor(F), grid, op.run("transient", tail=800)))
    torch.cuda.synchronize()
    rp = O_st.run(L, h, 0.1, dw, F, "periodic", periods=8, stride=50)
    ra = O_st.run(L, h, 0.1, dw, F, "periodic", periods=8, stride=50, adjoint=True)
    rt = O_st.run(L, h, 0.1, dw, F, "transient", tail=800)
    e = (per_freq_relerr(up, rp), per_freq_relerr(za, ra), per_freq_relerr(ut, rt))
    say("  errors", e)
    assert max(e) < 1e-10
    # adjoint identity on the GPU results
    lhs = np.sum(np.conj(F) * up, axis=-1)
    rhs = np.sum(np.conj(za) * F, axis=-1)
    assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(lhs).max()


@pytest.mark.parametrize("prec,shape", [("fp64", (66, 10, 36)), ("mixed", (66, 14, 36))])
def test_3d_tiles_and_z_chunks_match_oracle(prec, shape):
    """3-D grids that span two x tiles, several y tiles and two z chunks of the two-stage pass kernel, each with a
    ragged tail, against the oracle's four-stage march (FP64 1e-10, mixed 1e-3)."""
    import torch
    nx, ny, nz = shape
    say("case: 3-D tiles and z chunks", prec, shape)
    op, L = make3d(nx, ny, nz, 0.1, prec)
    h, P, nw, k = 0.1, 100, 2, 1
    dw = 2 * np.pi / (P * h)
    F = forcing(24, nw, k, op.n)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    out = to_np(op.apply(gpu_tensor(F, dt), op.grid(0.1, dw, nw), op.run("periodic", periods=3, stride=25)))
    torch.cuda.synchronize()
    ref = O_st.run(L, h, 0.1, dw, F, "periodic", periods=3, stride=25)
    e = per_freq_relerr(out, ref)
    say("  error", e)
    assert e < (1e-10 if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("shape", [(130, 21, 5), (60, 9, 40)])
def test_3d_fused_step_matches_oracle(shape):
    """The one-launch 3-D step of FP32 states (four stages pipelined along z): grids with ragged x and y tiles (56 x 8
    output nodes), fewer planes than the pipeline depth or many, two columns; direct (shear coupling of the first
    component), adjoint (its transpose) and transient runs against the oracle's four-stage march.  Bar 1e-4 per
    response vector (FP32 rounding, measured about 1e-6)."""
    import torch
    nx, ny, nz = shape
    say("case: 3-D fused FP32 step", shape)
    op, L = make3d(nx, ny, nz, 0.1, "mixed")
    h, P, nw, k = 0.1, 100, 2, 2
    dw = 2 * np.pi / (P * h)
    F = forcing(25, nw, k, op.n)
    f = gpu_tensor(F, torch.complex64)
    grid = op.grid(0.1, dw, nw)
    up = to_np(op.apply(f, grid, op.run("periodic", periods=3, stride=25)))
    za = to_np(op.adjoint_apply(f, grid, op.run("periodic", periods=3, stride=25)))
    ut = to_np(op.apply(f, grid, op.run("transient", tail=60)))
    torch.cuda.synchronize()
    Fr = F.astype(np.complex64).astype(np.complex128)
    rp = O_st.run(L, h, 0.1, dw, Fr, "periodic", periods=3, stride=25)
    ra = O_st.run(L, h, 0.1, dw, Fr, "periodic", periods=3, stride=25, adjoint=True)
    rt = O_st.run(L, h, 0.1, dw, Fr, "transient", tail=60)
    e = (per_freq_relerr(up, rp), per_freq_relerr(za, ra), per_freq_relerr(ut, rt))
    say("  errors", e)
    assert max(e) < 1e-4


@pytest.mark.parametrize("shape,chunks", [((60, 9, 40), 3), ((70, 12, 64), 4), ((130, 21, 5), 2)])
def test_3d_fused_step_in_z_chunks(shape, chunks, monkeypatch):
    """The one-launch 3-D step with the planes split among workgroups (each chunk after the first starts its
    march two planes early and discards the outputs below its first plane): the same bits as one chunk per tile,
    for chunks of 14, 16 and 3 planes (the last one shorter than the pipeline depth), and the oracle's run."""
    import torch
    nx, ny, nz = shape
    say("case: 3-D fused step in z chunks", shape, chunks)
    op, L = make3d(nx, ny, nz, 0.1, "mixed")
    h, P, nw, k = 0.1, 100, 2, 1
    dw = 2 * np.pi / (P * h)
    F = forcing(26, nw, k, op.n)
    grid, run = op.grid(0.1, dw, nw), op.run("periodic", periods=2, stride=25)
    outs = []
    for nzc in ("1", str(chunks)):
        monkeypatch.setenv("RESOLVENT_STEP3D_ZCHUNKS", nzc)
        outs.append(to_np(op.apply(gpu_tensor(F, torch.complex64), grid, run)))
        outs.append(to_np(op.adjoint_apply(gpu_tensor(F, torch.complex64), grid, run)))
        torch.cuda.synchronize()
    op.check()
    Fr = F.astype(np.complex64).astype(np.complex128)
    ref = O_st.run(L, h, 0.1, dw, Fr, "periodic", periods=2, stride=25)
    e = per_freq_relerr(outs[2], ref)
    say("  chunked equals one chunk: %s %s, vs oracle %.2e" % (np.array_equal(outs[2], outs[0]),
                                                             np.array_equal(outs[3], outs[1]), e))
    assert np.array_equal(outs[2], outs[0]) and np.array_equal(outs[3], outs[1])
    assert e < 1e-4


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_modes_match_oracle(case):
    import torch
    say("case: grid", case, "modes")
    op, L = CASES[case]()
    h, P, nw, k, iters = 0.1, 200, 2, 2, 3
    dw = 2 * np.pi / (P * h)
    F0 = forcing(22, nw, k, op.n)
    g, V, U, H = op.modes(gpu_tensor(F0), op.grid(0.0, dw, nw), op.run("periodic", periods=8, stride=50), iters)
    torch.cuda.synchronize()
    a, ad = O_it.stepped_applies(L, h, 0.0, dw, "periodic", periods=8, stride=50)
    g_ref, V_ref, U_ref, _ = O_it.block_power_iteration(a, ad, F0, iters)
    say("  gains err", np.abs(g[0] / g_ref - 1).max())
    assert np.abs(g[0] / g_ref - 1).max() < 1e-8
    assert mode_alignment(to_np(V)[:, :1], V_ref[:, :1]) > 1 - 1e-8


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_mixed_precision_error(case):
    import torch
    say("case: grid", case, "mixed")
    op, L = CASES[case]("mixed")
    h, P, nw, k = 0.1, 200, 3, 1
    dw = 2 * np.pi / (P * h)
    F = forcing(23, nw, k, op.n)
    out = to_np(op.apply(gpu_tensor(F, torch.complex64), op.grid(0.2, dw, nw), op.run("periodic", periods=8, stride=50)))
    torch.cuda.synchronize()
    ref = O_st.run(L, h, 0.2, dw, F, "periodic", periods=8, stride=50)
    say("  mixed err", per_freq_relerr(out, ref))
    assert per_freq_relerr(out, ref) < 1e-3


def test_set_diagonal_grid():
    import torch
    say("case: grid 2d set_diagonal")
    nx, ny, h, P, nw = 24, 16, 0.1, 200, 2
    dw = 2 * np.pi / (P * h)
    op, _ = make2d(nx, ny, h)
    from paper_2008_10904_amd.operators import adr2d_coefficients
    mu_new = mu2d(nx, ny) - 0.05 * np.random.default_rng(3).random((ny, nx))
    op.set_diagonal(adr2d_coefficients(nx, ny, mu=mu_new)["dfield"])
    F = forcing(24, nw, 1, op.n)
    out = to_np(op.apply(gpu_tensor(F), op.grid(0.0, dw, nw), op.run("periodic", periods=8, stride=50)))
    torch.cuda.synchronize()
    L, _ = O_ops.adr2d_operator(nx, ny, mu=mu_new)
    ref = O_st.run(L, h, 0.0, dw, F, "periodic", periods=8, stride=50)
    assert per_freq_relerr(out, ref) < 1e-10


def test_grid_operator_has_no_stepper_plan():
    from paper_2008_10904_amd import ResolventError
    say("case: grid operator plan calls")
    op, _ = make2d(8, 6, 0.1)
    with pytest.raises(ResolventError):
        op.get_plan()
    with pytest.raises(ResolventError):
        op.tune(1)
    with pytest.raises(ResolventError):
        op.set_step_power(2)


@pytest.mark.parametrize("shape", [(130, 70), (50, 21)])
def test_2d_step_pairs_match_single_steps(shape, monkeypatch):
    """FP32 2-D steps two per launch (windows of 64 and of 48 rows, halo 8) against one step per launch: the same
    bits for a periodic run (snapshots every third step, so sampled steps fall on both halves of a pair) and a
    transient run of an odd number of steps (the last one alone), direct and adjoint, with several tiles per
    direction and ragged edges; and the oracle's periodic run."""
    import torch
    nx, ny = shape
    say("case: 2-D step pairs against single steps", shape)
    op, L = make2d(nx, ny, 0.1, "mixed")
    h, P, nw, k = 0.1, 60, 3, 2
    dw = 2 * np.pi / (P * h)
    F = forcing(31, nw, k, op.n)
    grid = op.grid(-0.2, dw, nw)
    runs = [op.run("periodic", periods=3, stride=3), op.run("transient", tail=37)]
    outs = {}
    for wy in ("0", "64", "48"):
        monkeypatch.setenv("RESOLVENT_STEP2D_PAIR", wy)
        res = []
        for run in runs:
            res.append(to_np(op.apply(gpu_tensor(F, torch.complex64), grid, run)))
            res.append(to_np(op.adjoint_apply(gpu_tensor(F, torch.complex64), grid, run)))
        torch.cuda.synchronize()
        outs[wy] = res
    op.check()
    Fr = F.astype(np.complex64).astype(np.complex128)
    ref = O_st.run(L, h, -0.2, dw, Fr, "periodic", periods=3, stride=3)
    e = per_freq_relerr(outs["64"][0], ref)
    same = {wy: all(np.array_equal(a, b) for a, b in zip(outs[wy], outs["0"])) for wy in ("64", "48")}
    say("  pairs equal single steps: %s, periodic direct vs oracle %.2e" % (same, e))
    assert same["64"] and same["48"]
    assert e < 1e-4
