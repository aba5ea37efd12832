"""resolvent_apply_noalloc (the apply for callers that cannot allocate) against resolvent_apply on the same handle
and inputs, through the C ABI: two calls in a row, the second with a smaller input, for the 1-D operator (FP64 and
mixed precision, periodic and transient runs, the relaunched and the persistent stepper) and the 2-D operator, and
the rejection of a run whose workspace exceeds the fixed scratch.  Bars: 1e-10 per response vector in FP64 and
1e-5 in mixed precision (the two entry points differ only in rounding: tiles or a table for the forcing, and the
order of the projection's partial sums)."""
import numpy as np
import pytest

from _helpers import gpu_tensor, per_freq_relerr, say

pytestmark = pytest.mark.gpu
H = 0.02


def gl_op(n, precision):
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import gl_coefficients
    lo, d, up = gl_coefficients(n, 0.2, -0.01)  # x in [-50, 50]: dx = 0.33, |h lambda| <= 1 at h = 0.02
    return ResolventOp.tridiagonal(lo, d, up, H, precision=precision)


def forcing(seed, nw, k, n):
    g = np.random.default_rng(seed)
    return g.standard_normal((nw, k, n)) + 1j * g.standard_normal((nw, k, n))


def two_calls(op, F, grid_args, run, small, dtype, tol):
    """noalloc on F (before any apply: no exchange area yet), apply on F, noalloc on the smaller F[small]."""
    import torch
    nw = F.shape[0]
    f = gpu_tensor(F, dtype)
    g1 = op.grid(grid_args[0], grid_args[1], nw)
    out1 = torch.full_like(f, float("nan"))
    op.apply_noalloc(f, g1, run, out1)
    ref1 = op.apply(f, g1, run)
    Fs = np.ascontiguousarray(F[small[0], small[1]])
    fs = gpu_tensor(Fs, dtype)
    g2 = op.grid(grid_args[0], grid_args[1], Fs.shape[0])
    out2 = torch.full_like(fs, float("nan"))
    op.apply_noalloc(fs, g2, run, out2)
    ref2 = op.apply(fs, g2, run)
    torch.cuda.synchronize()
    op.check()
    e1 = per_freq_relerr(out1.cpu().numpy(), ref1.cpu().numpy())
    e2 = per_freq_relerr(out2.cpu().numpy(), ref2.cpu().numpy())
    say("  first call %.2e, second (smaller) call %.2e" % (e1, e2))
    assert e1 < tol and e2 < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_periodic_gl_matches_apply(precision):
    import torch
    say("case: no-allocation apply, GL N=300 h=0.02 periodic (P=400, 14 periods, stride 4), 8 frequencies, k=2,",
        precision)
    op = gl_op(300, precision)
    dw = 2 * np.pi / (400 * H)
    F = forcing(101, 8, 2, 300)
    dtype = torch.complex128 if precision == "fp64" else torch.complex64
    two_calls(op, F, (-0.3, dw), op.run("periodic", periods=14, stride=4), (slice(0, 3), slice(0, 1)), dtype,
              1e-10 if precision == "fp64" else 1e-5)


def test_noalloc_transient_gl_matches_apply():
    import torch
    say("case: no-allocation apply, GL N=300 h=0.02 transient (P=400, tail 600), 5 frequencies, k=3, FP64")
    op = gl_op(300, "fp64")
    dw = 2 * np.pi / (400 * H)
    F = forcing(102, 5, 3, 300)
    two_calls(op, F, (0.1, dw), op.run("transient", tail=600), (slice(1, 3), slice(1, 3)), torch.complex128, 1e-10)


def test_noalloc_grid2d_matches_apply():
    import torch
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr2d_coefficients
    say("case: no-allocation apply, 2-D 90 x 40 periodic (P=200, 6 periods), 4 frequencies, k=2, FP64")
    nx, ny, h = 90, 40, 0.05
    op = ResolventOp.grid_operator("adr2d", nx, ny, 1, adr2d_coefficients(nx, ny, Re=50.0, Lx=9.0, ylo=-2.0, yhi=2.0),
                                   h, precision="fp64")
    dw = 2 * np.pi / (200 * h)
    F = forcing(103, 4, 2, nx * ny)
    two_calls(op, F, (0.2, dw), op.run("periodic", periods=6, stride=2), (slice(0, 2), slice(0, 1)),
              torch.complex128, 1e-10)


def test_noalloc_rejects_a_run_beyond_the_scratch():
    import torch
    from paper_2008_10904_amd import ResolventError
    from paper_2008_10904_amd import _lib as L
    say("case: no-allocation apply of a run whose workspace exceeds the scratch (N=20000, k=4, 256 frequencies)")
    op = gl_op(20000, "fp64")
    dw = 2 * np.pi / (400 * H)
    f = torch.zeros((256, 4, 20000), dtype=torch.complex128, device="cuda")
    out = torch.empty_like(f)
    with pytest.raises(ResolventError) as e:
        op.apply_noalloc(f, op.grid(-1.0, dw, 256), op.run("periodic", periods=2), out)
    assert e.value.code == L.RES_EINVAL and "no-allocation scratch" in str(e.value)
