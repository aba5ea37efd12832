"""Pins of the CPU oracle against facts fixed by the paper and by mathematics (no GPU).

Each test names what it pins.  None of them re-types an oracle formula: they compare the oracle with
textbook results (dense inverses, closed-form spectra, convergence orders, exact Fourier identities) or
compare two independent computations (explicit time marching vs the algebraic transfer matrix).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dense, gradient, iteration, krylov, operators, stepping, trm, weights

# A small, stable GL problem on [-15, 15] (32 nodes) shared by several pins.
N_T, XL_T, XR_T = 32, -15.0, 15.0
MU0_T, MU2_T = 0.20, -0.01
H_T, P_T = 0.05, 400


def tiny_gl(mu0=MU0_T, mu2=MU2_T, n=N_T):
    L, x = operators.gl_operator(n, mu0, mu2, xl=XL_T, xr=XR_T)
    return L, x


def forcing(seed, nw, k, n):
    g = np.random.default_rng(seed)
    return g.standard_normal((nw, k, n)) + 1j * g.standard_normal((nw, k, n))


def test_tiny_gl_is_stable():
    L, _ = tiny_gl()
    assert np.linalg.eigvals(L.toarray()).real.max() < -0.05


# ---------------------------------------------------------------------------------------------
# Operators: each PDE term against its analytic action on a smooth function (pins signs and indices).
# ---------------------------------------------------------------------------------------------
def test_gl_operator_matches_pde_on_smooth_function():
    # g vanishes at both ends; L g must approach -nu g' + gamma g'' + mu g at second order in dx.
    errs = []
    for n in (200, 400):
        L, x = operators.gl_operator(n, 0.3, -0.01)
        a = np.pi / 100.0
        g = np.sin(a * (x + 50.0)) ** 2
        gp = 2 * a * np.sin(a * (x + 50.0)) * np.cos(a * (x + 50.0))
        gpp = 2 * a * a * np.cos(2 * a * (x + 50.0))
        mu = (0.3 - 0.04) - 0.005 * x * x
        exact = -(2 + 0.4j) * gp + (1 - 1j) * gpp + mu * g
        errs.append(np.abs(L @ g - exact).max())
    assert errs[0] < 1e-3 and 3.5 < errs[0] / errs[1] < 4.5  # second-order


def test_gl_constant_mu_spectrum_is_tridiagonal_toeplitz():
    # Dirichlet tridiagonal Toeplitz (sub a, diag b, super c): lambda_m = b + 2 sqrt(a c) cos(m pi/(n+1)).
    n = 60
    L, x = operators.gl_operator(n, 0.1, 0.0)
    dx = x[1] - x[0]
    nu, gam = 2 + 0.4j, 1 - 1j
    a = nu / (2 * dx) + gam / dx ** 2
    c = -nu / (2 * dx) + gam / dx ** 2
    b = -2 * gam / dx ** 2 + (0.1 - 0.04)
    m = np.arange(1, n + 1)
    ref = b + 2 * np.sqrt(a * c) * np.cos(m * np.pi / (n + 1))
    got = np.linalg.eigvals(L.toarray())
    assert np.abs(np.sort_complex(got) - np.sort_complex(ref)).max() < 1e-9 * np.abs(ref).max()


def test_adr2d_operator_matches_pde_on_smooth_function():
    errs = []
    for (nx, ny) in ((64, 32), (128, 64)):
        mu = None
        L, f = operators.adr2d_operator(nx, ny, Re=200.0, mu=mu)
        X, Y = f["X"], f["Y"]
        ax, ay = np.pi / 40.0, np.pi / 20.0
        g = np.sin(ax * X) ** 2 * np.sin(ay * (Y + 10)) ** 2
        gx = 2 * ax * np.sin(ax * X) * np.cos(ax * X) * np.sin(ay * (Y + 10)) ** 2
        gxx = 2 * ax * ax * np.cos(2 * ax * X) * np.sin(ay * (Y + 10)) ** 2
        gyy = 2 * ay * ay * np.cos(2 * ay * (Y + 10)) * np.sin(ax * X) ** 2
        exact = -np.tanh(Y) * gx + (gxx + gyy) / 200.0 + (f["mu"] - f["sponge"]) * g
        errs.append(np.abs((L @ g.ravel()).reshape(ny, nx) - exact).max())
    assert 3.3 < errs[0] / errs[1] < 4.7


def test_adr3d3c_operator_matches_pde_on_smooth_function():
    wake = dict(amp=0.5, delta=2.0, y0=0.2, z0=-0.3)
    errs = []
    for n in ((24, 16, 16), (48, 32, 32)):
        nx, ny, nz = n
        L, f = operators.adr3d3c_operator(nx, ny, nz, wake, Re=200.0)
        X, Y, Z = f["X"], f["Y"], f["Z"]
        a, b = np.pi / 40.0, np.pi / 20.0
        sx, sy, sz = np.sin(a * X) ** 2, np.sin(b * (Y + 10)) ** 2, np.sin(b * (Z + 10)) ** 2
        g = sx * sy * sz
        gx = 2 * a * np.sin(a * X) * np.cos(a * X) * sy * sz
        lap = (2 * a * a * np.cos(2 * a * X) * sy * sz + 2 * b * b * np.cos(2 * b * (Y + 10)) * sx * sz
               + 2 * b * b * np.cos(2 * b * (Z + 10)) * sx * sy)
        Ug = 1 - 0.5 * np.exp(-((Y - 0.2) ** 2 + (Z + 0.3) ** 2) / 4.0)
        Uy = 0.5 * np.exp(-((Y - 0.2) ** 2 + (Z + 0.3) ** 2) / 4.0) * 2 * (Y - 0.2) / 4.0
        Uz = 0.5 * np.exp(-((Y - 0.2) ** 2 + (Z + 0.3) ** 2) / 4.0) * 2 * (Z + 0.3) / 4.0
        scal = -Ug * gx + lap / 200.0 + (-0.05 - f["sponge"]) * g
        # components (u, v, w) = (g, 2g, 3g)
        q = np.concatenate([g.ravel(), 2 * g.ravel(), 3 * g.ravel()])
        out = (L @ q).reshape(3, nz, ny, nx)
        ex = np.stack([scal - 2 * g * Uy - 3 * g * Uz, 2 * scal, 3 * scal])
        errs.append(np.abs(out - ex).max())
    assert 3.3 < errs[0] / errs[1] < 4.7


def test_input_fields_take_their_defining_values():
    # The sponge ramp is 0 at least w = frac (hi - lo) inside both ends, 1 at an end and linear in between; the
    # 2-D sponge is nu_s max(r_x, r_y)^2; the reaction bump peaks at base + amp at (xc, 0) and falls to base; the
    # wake deficit is amp at (y0, z0) and vanishes far away.  Interior grids exclude the end points.
    s = np.array([0.0, 0.5, 1.0, 2.0, 5.0, 9.5, 10.0])
    assert np.allclose(operators.sponge_ramp(s, 0.0, 10.0, 0.1), [1.0, 0.5, 0.0, 0.0, 0.0, 0.5, 1.0], atol=1e-15)
    x, d = operators.uniform_interior_grid(9, 0.0, 40.0)
    assert d == 4.0 and x[0] == 4.0 and x[-1] == 36.0
    f = operators.adr2d_fields(79, 39, nu_s=2.0)  # dx = 0.5, dy = 0.5: node (x, y) = (0.5 (i+1), -10 + 0.5 (j+1))
    assert f["sponge"][19, 39] == 0.0  # (20, 0): interior
    # ramp widths 4 in x (0.1 of 40) and 2 in y (0.1 of 20)
    assert abs(f["sponge"][0, 0] - 2.0 * 0.875 ** 2) < 1e-14  # (0.5, -9.5): r_x = 3.5/4, r_y = 1.5/2
    assert abs(f["sponge"][1, 2] - 2.0 * 0.625 ** 2) < 1e-14  # (1.5, -9): r_x = 2.5/4, r_y = 1/2
    assert abs(operators.adr2d_mu_default(10.0, 0.0, base=-0.1, amp=0.08) - (-0.02)) < 1e-15
    assert abs(operators.adr2d_mu_default(30.0, 9.0, base=-0.1, amp=0.08) + 0.1) < 1e-15
    U, _, _ = operators.wake_profile(np.array([0.2, 9.0]), np.array([-0.3, 9.0]), amp=0.5, delta=2.0, y0=0.2, z0=-0.3)
    assert abs(U[0] - 0.5) < 1e-15 and abs(U[1] - 1.0) < 1e-15
    assert abs(operators.gl_mu(np.array(10.0), 0.3, -0.01) - (0.3 - 0.04 - 0.5)) < 1e-15


def test_wake_shear_is_the_derivative_of_the_wake():
    # U_y and U_z of the wake profile against central differences of its own U: second order in the step, so
    # halving the step cuts the error by 4.  A wrong sign, a dropped factor, delta instead of delta^2 or y0 and z0
    # swapped all break it.
    wake = dict(amp=0.5, delta=2.0, y0=0.2, z0=-0.3)
    y = np.linspace(-10.0, 10.0, 41)
    Y, Z = np.meshgrid(y, y + 0.05, indexing="ij")
    _, Uy, Uz = operators.wake_profile(Y, Z, **wake)
    errs = []
    for d in (2e-2, 1e-2):
        cy = (operators.wake_profile(Y + d, Z, **wake)[0] - operators.wake_profile(Y - d, Z, **wake)[0]) / (2 * d)
        cz = (operators.wake_profile(Y, Z + d, **wake)[0] - operators.wake_profile(Y, Z - d, **wake)[0]) / (2 * d)
        errs.append(max(np.abs(cy - Uy).max(), np.abs(cz - Uz).max()))
    assert errs[1] < 1e-4 * np.abs(Uy).max()
    assert 3.8 < errs[0] / errs[1] < 4.2


def _tiny_adr3d(mu=None):
    wake = dict(amp=0.5, delta=2.0, y0=0.2, z0=-0.3)
    return operators.adr3d3c_operator(5, 4, 3, wake, Re=50.0, mu=mu, Lx=8.0, lo=-4.0, hi=4.0)


def test_node_field_expansion_is_the_operators_reaction_term():
    # A node field mu enters the three-component operator (built block by block with Kronecker products) on the
    # diagonal of every component block: L(mu) - L(0) = diag(expand(mu)).  A node-major expansion (repeat instead
    # of tile) or a field on one component only breaks it.
    g = np.random.default_rng(41)
    mu = g.standard_normal((3, 4, 5))
    d = (_tiny_adr3d(mu)[0] - _tiny_adr3d(np.zeros((3, 4, 5)))[0]).toarray()
    assert np.abs(d - np.diag(gradient.expand_node_field(mu, 3))).max() < 1e-14


def test_shared_node_field_gradient_sums_the_per_component_gradients():
    # The gradient with respect to a node field shared by three components is the per-unknown gradient of the
    # diagonal (central differences, one unknown of the 3 x 60 at a time) summed over the components of each node
    # (chain rule through the expansion).  Pins the ncomp = 3 path of the oracle's mu gradient.
    L0, _ = _tiny_adr3d(np.zeros((3, 4, 5)))
    nodes = 60
    h, P = 0.1, 20
    dw = 2 * np.pi / (P * h)
    F, G = forcing(42, 2, 2, 3 * nodes), forcing(43, 2, 2, 3 * nodes)
    mu = np.random.default_rng(44).uniform(-0.1, 0.1, nodes)
    kw = dict(tail=15)
    node = gradient.stepped_mu_gradient(L0, mu, h, 0.3, dw, F, G, "transient", eps=1e-5, ncomp=3, **kw)
    dof = gradient.stepped_mu_gradient(L0, np.tile(mu, 3), h, 0.3, dw, F, G, "transient", eps=1e-5, ncomp=1, **kw)
    summed = dof.reshape(3, nodes).sum(axis=0)
    assert np.abs(node - summed).max() < 1e-7 * np.abs(summed).max()
    assert np.abs(dof.reshape(3, nodes)[1:]).max() > 1e-3 * np.abs(summed).max()  # every component contributes


# ---------------------------------------------------------------------------------------------
# Dense ground truth against closed forms.
# ---------------------------------------------------------------------------------------------
def test_diagonal_operator_gains_closed_form():
    mu = np.array([-0.3, -1.0, -0.05 + 0.2j, -2.0])
    w = 0.7
    s, U, V = dense.gains_and_modes(dense.resolvent(np.diag(mu), w))
    assert np.allclose(s, np.sort(1 / np.abs(1j * w - mu))[::-1], rtol=1e-13)


def test_circulant_operator_gains_closed_form_and_iteration():
    # Periodic constant-coefficient stencil: normal operator, Fourier eigenvectors,
    # lambda_m = b + a e^{-i theta_m} + c e^{+i theta_m}; gains = 1/|i w - lambda_m|.
    n = 40
    a, b, c = 0.9 + 0.3j, -2.5 + 0.1j, 1.1 - 0.3j
    L = (np.diag(np.full(n, b)) + np.diag(np.full(n - 1, a), -1) + np.diag(np.full(n - 1, c), 1)).astype(complex)
    L[0, -1] = a
    L[-1, 0] = c
    th = 2 * np.pi * np.arange(n) / n
    lam = b + a * np.exp(-1j * th) + c * np.exp(1j * th)
    w = 0.4
    ref = np.sort(1 / np.abs(1j * w - lam))[::-1]
    s, _, _ = dense.gains_and_modes(dense.resolvent(L, w))
    assert np.allclose(s, ref, rtol=1e-12)
    # the block power iteration on the continuous resolvent recovers the top 3
    R = dense.resolvent(L, w)
    ap = lambda F: np.stack([(R @ F[0].T).T])
    ad = lambda G: np.stack([(R.conj().T @ G[0].T).T])
    g, V, U, _ = iteration.block_power_iteration(ap, ad, forcing(3, 1, 3, n), 200)
    assert np.allclose(g[0], ref[:3], rtol=1e-10)


def test_rk4_transfer_converges_at_fourth_order():
    # R_d(w) -> (i w I - L)^{-1} as h^4: the gain error drops by ~16 per halving of h.
    L, _ = tiny_gl()
    w = -0.3
    s0 = dense.gains_and_modes(dense.resolvent(L, w), 1)[0][0]
    errs = [abs(dense.gains_and_modes(dense.resolvent_rk4(L, w, h), 1)[0][0] / s0 - 1)
            for h in (0.1, 0.05, 0.025)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 14.5 < r1 < 17.5 and 14.5 < r2 < 17.5


def test_rk4_steady_residual_vanishes_on_discrete_resolvent_and_converges_at_fifth_order():
    # The matrix-free residual e^{iwh}u - P(Z)u - hQ_w(Z)f of the steady RK4 response: zero (to rounding) for
    # u = R_d(w) f; for the continuous response u = (iwI - L)^{-1} f it is (e^{iwh} - P(Z))(R - R_d) f, an O(h)
    # factor times an O(h^4) difference, so it drops by ~32 per halving of h.
    L, _ = tiny_gl()
    w = 0.4
    rng = np.random.default_rng(7)
    f = rng.standard_normal(L.shape[0]) + 1j * rng.standard_normal(L.shape[0])
    for h in (0.1, 0.05):
        Qf = dense.rk4_forcing_matrix(h * L.toarray(), w, h) @ f
        r = dense.rk4_steady_residual(L, w, h, dense.resolvent_rk4(L, w, h) @ f, f)
        assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(Qf)
    u = dense.resolvent(L, w) @ f
    res = [np.linalg.norm(dense.rk4_steady_residual(L, w, h, u, f)) for h in (0.1, 0.05, 0.025)]
    r1, r2 = res[0] / res[1], res[1] / res[2]
    assert 28 < r1 < 36 and 28 < r2 < 36


def test_rk4_amplification_is_taylor_of_exponential():
    # P(z) agrees with e^z to fourth order: |P(z) - e^z| ~ |z|^5/120.
    for z in (0.01 + 0.02j, -0.02 + 0.01j):
        p = dense.rk4_amplification(np.array([[z]]))[0, 0]
        assert abs(p - np.exp(z)) < 2 * abs(z) ** 5 / 120


# ---------------------------------------------------------------------------------------------
# Time stepping: explicit runs against the algebraic transfer matrix and the continuous resolvent.
# ---------------------------------------------------------------------------------------------
def _grid3():
    dw = 2 * np.pi / (P_T * H_T)
    return -0.3, dw, stepping.frequencies(-0.3, dw, 3)


def test_periodic_run_equals_rk4_transfer_matrix():
    L, _ = tiny_gl()
    w0, dw, om = _grid3()
    F = forcing(1, 3, 2, N_T)
    Ustep = stepping.run(L, H_T, w0, dw, F, "periodic", periods=14)
    for j, w in enumerate(om):
        ref = (dense.resolvent_rk4(L, w, H_T) @ F[j].T).T
        assert np.linalg.norm(Ustep[j] - ref) / np.linalg.norm(ref) < 1e-12


def test_transient_run_equals_rk4_transfer_matrix():
    L, _ = tiny_gl()
    w0, dw, om = _grid3()
    F = forcing(2, 3, 1, N_T)
    U, uend = stepping.transient_run(L, H_T, om, F, P_T, 13 * P_T)
    assert np.linalg.norm(uend) < 1e-13 * np.linalg.norm(F)
    for j, w in enumerate(om):
        ref = (dense.resolvent_rk4(L, w, H_T) @ F[j].T).T
        assert np.linalg.norm(U[j] - ref) / np.linalg.norm(ref) < 1e-12


def test_stepped_response_converges_to_continuous_resolvent_at_fourth_order():
    # Independent of the algebraic transfer matrix: marched response vs (i w I - L)^{-1} F.
    L, _ = tiny_gl()
    F = forcing(4, 1, 1, N_T)
    errs = []
    for h, P in ((0.1, 100), (0.05, 200)):
        dw = 2 * np.pi / (P * h)
        U = stepping.run(L, h, -0.4, dw, F, "periodic", periods=20)
        ref = np.linalg.solve(1j * (-0.4) * np.eye(N_T) - L.toarray(), F[0, 0])
        errs.append(np.linalg.norm(U[0, 0] - ref) / np.linalg.norm(ref))
    assert errs[0] < 1e-5 and 13 < errs[0] / errs[1] < 19


def test_adjoint_run_is_hermitian_transpose():
    # Sec. 2.1 adjoint relations: the adjoint run realises R_d^H and <R f, g> = <f, R^H g>.
    L, _ = tiny_gl()
    w0, dw, om = _grid3()
    F = forcing(5, 3, 1, N_T)
    G = forcing(6, 3, 1, N_T)
    RF = stepping.run(L, H_T, w0, dw, F, "periodic", periods=14)
    RHG = stepping.run(L, H_T, w0, dw, G, "periodic", periods=14, adjoint=True)
    for j, w in enumerate(om):
        Rd = dense.resolvent_rk4(L, w, H_T)
        assert np.linalg.norm(RHG[j, 0] - Rd.conj().T @ G[j, 0]) / np.linalg.norm(RHG[j, 0]) < 1e-12
        lhs = np.vdot(G[j, 0], RF[j, 0])
        rhs = np.vdot(RHG[j, 0], F[j, 0])
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_subsampled_projection_is_exact_for_steady_state():
    L, _ = tiny_gl()
    w0, dw, om = _grid3()
    F = forcing(7, 3, 1, N_T)
    full = stepping.run(L, H_T, w0, dw, F, "periodic", periods=14, stride=1)
    sub = stepping.run(L, H_T, w0, dw, F, "periodic", periods=14, stride=100)  # 4 samples >= 3 freqs
    assert np.linalg.norm(full - sub) / np.linalg.norm(full) < 1e-12


def test_grid_snapping_and_commensurability():
    w0, dw, P = stepping.snap_grid(-3.0, 3.0, 256, 0.001, stride=256)
    assert P % 256 == 0 and abs(dw * P * 0.001 - 2 * np.pi) < 1e-12
    assert abs(w0 + 255 * dw - 3.0) < 2e-3
    with pytest.raises(ValueError):
        stepping.period_steps(0.0123456, 0.001)


def test_real_operator_gains_symmetric_in_frequency():
    # Real L: R(-w) = conj(R(w)), so the gains at +-w coincide; the stepped runs respect it.
    L = operators.gl_operator(N_T, 0.2, -0.01, nu=1.5, gamma=1.0, xl=XL_T, xr=XR_T)[0]
    h, P = 0.05, 400
    dw = 2 * np.pi / (P * h)
    w = 3 * dw  # +w and -w both on the grid starting at -w
    apply, adj = iteration.stepped_applies(L, h, -w, dw, "periodic", periods=8, stride=50)
    F = forcing(8, 7, 2, N_T)
    g, _, _, _ = iteration.block_power_iteration(apply, adj, F, 16)
    assert abs(g[0, 0] / g[6, 0] - 1) < 1e-11


# ---------------------------------------------------------------------------------------------
# Block power iteration (Appendix A) against the SVD.
# ---------------------------------------------------------------------------------------------
def test_block_iteration_converges_to_svd_of_transfer_matrix():
    L, _ = tiny_gl()
    om = np.array([-0.3, 0.0, 0.5])
    apply, adj = iteration.dense_rk4_applies(L, H_T, om)
    F0 = forcing(9, 3, 3, N_T)
    g, V, U, hist = iteration.block_power_iteration(apply, adj, F0, 60)
    for j, w in enumerate(om):
        Rd = dense.resolvent_rk4(L, w, H_T)
        s, Us, Vs = dense.gains_and_modes(Rd, 3)
        assert np.allclose(g[j], s, rtol=1e-10)
        for i in range(2):  # modes up to phase
            assert abs(abs(np.vdot(Vs[:, i], V[j, i])) - 1) < 1e-8
            assert abs(abs(np.vdot(Us[:, i], U[j, i])) - 1) < 1e-8
            assert np.linalg.norm(Rd @ V[j, i] - g[j, i] * U[j, i]) < 1e-8 * g[j, i]
    # both estimators in the history agree with sigma once converged (eq. tildeSig)
    assert np.allclose(hist[-1, :, 0, 1], g[:, 0], rtol=1e-8)


def test_power_iteration_error_decays_at_gain_ratio_rate():
    # Appendix A: with k = 1 the force-mode error falls like (sigma_2/sigma_1)^{2n}; the Rayleigh-Ritz gain
    # error, quadratic in the mode error, like (sigma_2/sigma_1)^{4n}.
    L, _ = tiny_gl()
    w = 0.3
    apply, adj = iteration.dense_rk4_applies(L, H_T, np.array([w]))
    s = dense.gains_and_modes(dense.resolvent_rk4(L, w, H_T), 2)[0]
    rate = (s[1] / s[0]) ** 4
    _, _, _, hist = iteration.block_power_iteration(apply, adj, forcing(10, 1, 1, N_T), 8)
    err = np.abs(hist[:, 0, 0, 0] / s[0] - 1)
    ratios = err[3:7] / err[2:6]
    assert np.all(np.abs(ratios / rate - 1) < 0.2)


def test_stepped_iteration_matches_dense_iteration():
    L, _ = tiny_gl()
    w0, dw, om = _grid3()
    F0 = forcing(11, 3, 2, N_T)
    a1, d1 = iteration.stepped_applies(L, H_T, w0, dw, "transient", tail=13 * P_T)
    a2, d2 = iteration.dense_rk4_applies(L, H_T, om)
    g1 = iteration.block_power_iteration(a1, d1, F0, 3)[0]
    g2 = iteration.block_power_iteration(a2, d2, F0, 3)[0]
    assert np.allclose(g1, g2, rtol=1e-11)


# ---------------------------------------------------------------------------------------------
# Arnoldi (Krylov-subspace) pins.
# ---------------------------------------------------------------------------------------------
def test_arnoldi_on_the_whole_space_is_the_svd():
    # Appendix A: once the orthonormal forcings span the whole space, H = F^H R^H R F is R^H R in that basis, so
    # its eigenvalues are the squared singular values of R_d and F psi are its right singular vectors.
    L, _ = tiny_gl(n=8)
    om = np.array([-0.4, 0.25])
    apply, adj = iteration.dense_rk4_applies(L, H_T, om)
    g, V, U, hist = krylov.block_arnoldi(apply, adj, forcing(31, 2, 2, 8), 4)
    for j, w in enumerate(om):
        Rd = dense.resolvent_rk4(L, w, H_T)
        s, Us, Vs = dense.gains_and_modes(Rd, 2)
        assert np.allclose(g[j], s, rtol=1e-11)
        for i in range(2):
            assert abs(abs(np.vdot(Vs[:, i], V[j, i])) - 1) < 1e-10
            assert abs(abs(np.vdot(Us[:, i], U[j, i])) - 1) < 1e-10
    assert np.allclose(hist[-1], g, rtol=1e-14)


def test_arnoldi_first_block_is_the_rayleigh_quotient():
    # One block: H = F^H R^H R F for the orthonormalised start, whose top eigenvalue is sigma(R F)^2 -- the gain
    # of one power iteration from the same start.
    L, _ = tiny_gl()
    om = np.array([0.1, 0.7])
    apply, adj = iteration.dense_rk4_applies(L, H_T, om)
    F0 = forcing(32, 2, 2, N_T)
    g = krylov.block_arnoldi(apply, adj, F0, 1)[0]
    for j in range(2):
        F = iteration.qr_positive(F0[j].T)[0]
        s = np.linalg.svd(dense.resolvent_rk4(L, om[j], H_T) @ F, compute_uv=False)
        assert np.allclose(g[j], s, rtol=1e-12)


def test_arnoldi_converges_faster_than_the_power_iteration():
    # Appendix A: with small gain separation the Krylov estimate of the suboptimal gain is far ahead of the power
    # iteration after the same number of runs; both approach the SVD from below (Ritz values).
    L, _ = tiny_gl()
    om = np.array([0.2])
    apply, adj = iteration.dense_rk4_applies(L, H_T, om)
    s = dense.gains_and_modes(dense.resolvent_rk4(L, om[0], H_T), 2)[0]
    F0 = forcing(33, 1, 2, N_T)
    gk = krylov.block_arnoldi(apply, adj, F0, 6)[0][0]
    gp = iteration.block_power_iteration(apply, adj, F0, 6)[0][0]
    ek, ep = np.abs(gk / s - 1), np.abs(gp / s - 1)
    assert np.all(gk <= s * (1 + 1e-12))
    assert ek[1] < 0.1 * ep[1] and ek[0] <= ep[0] * (1 + 1e-9)


# ---------------------------------------------------------------------------------------------
# B, C and metric pins.
# ---------------------------------------------------------------------------------------------
def _weights(n, seed):
    g = np.random.default_rng(seed)
    b = np.where(np.arange(n) < 3 * n // 4, 1.0, 0.0) * (0.5 + g.random(n))  # a force mask with amplitudes
    c = np.where(np.arange(n) >= n // 4, 1.0, 0.0)                            # an observation window
    wf = 0.2 + g.random(n)                                                    # quadrature-like weights
    wy = 0.2 + g.random(n)
    return b, c, wf, wy


def test_weighted_adjoint_identity():
    # Sec. 2.1: <R_y f, y>_{W_y} = <f, R_y^dagger y>_{W_f} with R_y^dagger = W_f^{-1} B^H R^H C^H W_y.
    L, _ = tiny_gl()
    om = np.array([-0.2, 0.4])
    a, ad = iteration.dense_rk4_applies(L, H_T, om)
    b, c, wf, wy = _weights(N_T, 50)
    ay, ady = weights.observed_applies(a, ad, b, c, wf, wy)
    F, Y = forcing(51, 2, 1, N_T), forcing(52, 2, 1, N_T)
    lhs = np.sum(np.conj(ay(F)) * wy * Y, axis=-1)
    rhs = np.sum(np.conj(F) * wf * ady(Y), axis=-1)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=0)


def test_weighted_gains_are_the_generalised_singular_values():
    # max ||C R B f||_{W_y} / ||f||_{W_f}: the generalised eigenproblem (R_y^H W_y R_y) v = s^2 W_f v, solved densely,
    # against the SVD of the Euclidean R~ and against the block iteration with R~'s applies.
    import scipy.linalg as sla
    L, _ = tiny_gl()
    om = np.array([0.0, 0.6])
    a, ad = iteration.dense_rk4_applies(L, H_T, om)
    b, c, wf, wy = _weights(N_T, 53)
    ae, ade = weights.euclidean_applies(a, ad, b, c, wf, wy)
    g, V, U, _ = iteration.block_power_iteration(ae, ade, forcing(54, 2, 2, N_T), 80)
    Vw, Uw = weights.modes_from_euclidean(V, U, wf, wy)
    for j, w in enumerate(om):
        Ry = np.diag(c) @ dense.resolvent_rk4(L, w, H_T) @ np.diag(b)
        lam, vec = sla.eigh(Ry.conj().T @ np.diag(wy) @ Ry, np.diag(wf))
        s = np.sqrt(np.maximum(lam[::-1][:2], 0))
        assert np.allclose(g[j], s, rtol=1e-10)
        v1 = vec[:, -1]
        # W_f-normalised leading force mode, up to a phase; its W_y gain is s_1
        assert abs(abs(np.vdot(v1, wf * Vw[j, 0])) / np.sqrt(np.vdot(v1, wf * v1).real) - 1) < 1e-8
        assert abs(np.sqrt(np.sum(wy * np.abs(Ry @ Vw[j, 0]) ** 2)) / s[0] - 1) < 1e-10


# ---------------------------------------------------------------------------------------------
# Gain sensitivity (gradient) pins.
# ---------------------------------------------------------------------------------------------
def test_leading_gain_sensitivity_closed_form_matches_finite_differences():
    n = 24
    x, _ = operators.uniform_interior_grid(n, XL_T, XR_T)
    mu = operators.gl_mu(x, 0.2, -0.01)
    Lmu = lambda m: operators.gl_operator(n, mu=m, xl=XL_T, xr=XR_T)[0].toarray()
    w = -0.2
    sig = lambda m: dense.gains_and_modes(dense.resolvent(Lmu(m), w), 1)[0][0]
    fd = gradient.central_difference_gradient(sig, mu, 1e-6)
    cf = gradient.leading_gain_sensitivity(Lmu(mu), w)
    assert np.linalg.norm(cf - fd) < 1e-7 * np.linalg.norm(fd)


def test_discrete_objective_gradient_tends_to_continuous_sensitivity():
    # With V the leading force mode of R_d, dJ/dmu of the discrete objective approaches the continuous closed
    # form as h -> 0 (both are sigma_1 sensitivities; they differ by the RK4 error only).
    n = 24
    x, _ = operators.uniform_interior_grid(n, XL_T, XR_T)
    mu = operators.gl_mu(x, 0.2, -0.01)
    Lmu = lambda m: operators.gl_operator(n, mu=m, xl=XL_T, xr=XR_T)[0].toarray()
    w, h = -0.2, 0.01
    V1 = dense.gains_and_modes(dense.resolvent_rk4(Lmu(mu), w, h), 1)[2][:, 0]
    J = lambda m: gradient.discrete_objective(Lmu, m, h, [w], V1[None, :], np.array([1.0]))
    fd = gradient.central_difference_gradient(J, mu, 1e-6)
    cf = gradient.leading_gain_sensitivity(Lmu(mu), w)
    assert np.linalg.norm(cf - fd) < 1e-5 * np.linalg.norm(cf)


# ---------------------------------------------------------------------------------------------
# Reverse mode of the time-stepped run (the references for the GPU backward pass).
# ---------------------------------------------------------------------------------------------
def _small_gl(mu0):
    return operators.gl_operator(12, mu0, -0.01, xl=XL_T, xr=XR_T)[0]


@pytest.mark.parametrize("method,kw", [("transient", dict(tail=90)), ("periodic", dict(periods=3, stride=6))])
def test_stepped_vjp_is_the_adjoint_of_the_run(method, kw):
    # <A^H G, d> = <G, A d> for independent random d: a dropped conjugate, a transposed transfer matrix or a
    # wrong unit-forcing index breaks it.
    L = _small_gl(0.2)
    h, P = 0.1, 60
    dw = 2 * np.pi / (P * h)
    G = forcing(31, 3, 2, 12)
    vjp = gradient.stepped_vjp(L, h, -0.4, dw, G, method, **kw)
    for seed in (32, 33):
        d = forcing(seed, 3, 2, 12)
        Ad = stepping.run(L, h, -0.4, dw, d, method, **kw)
        lhs, rhs = np.vdot(vjp, d), np.vdot(G, Ad)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_stepped_vjp_tends_to_dense_adjoint_in_steady_state():
    # Periodic run long after the transient: A is block diagonal with blocks R_d(w_j), so A^H G = R_d^H G.
    L = _small_gl(-0.5)
    h, P = 0.1, 60
    dw = 2 * np.pi / (P * h)
    G = forcing(34, 3, 1, 12)
    vjp = gradient.stepped_vjp(L, h, -0.4, dw, G, "periodic", periods=12, stride=6)
    for j, w in enumerate(stepping.frequencies(-0.4, dw, 3)):
        ref = dense.resolvent_rk4(L, w, h).conj().T @ G[j, 0]
        assert np.linalg.norm(vjp[j, 0] - ref) < 1e-10 * np.linalg.norm(ref)


def test_stepped_mu_gradient_of_diagonal_operator_matches_closed_form():
    # L = diag(lambda): each unknown is a scalar RK4 recurrence whose steady response to F e^{i w t} is
    # r(z) F with r(z) = h q(z) / (e^{i w h} - p(z)), z = h (lambda + mu), p the RK4 step polynomial and q its
    # forcing polynomial; then dJ/dmu_x = Re sum conj(G) h r'(z) F with r' from the quotient rule.
    n, h, P = 6, 0.1, 60
    lam = -0.6 + 1j * np.linspace(-1.0, 1.0, n)
    L0 = sp.diags(lam).tocsr()
    dw = 2 * np.pi / (P * h)
    F, G = forcing(35, 3, 2, n), forcing(36, 3, 2, n)
    fd = gradient.stepped_mu_gradient(L0, np.zeros(n), h, -0.4, dw, F, G, "periodic", eps=1e-5, periods=14,
                                      stride=6)
    p = np.polynomial.Polynomial([1.0, 1.0, 1 / 2, 1 / 6, 1 / 24])
    ref = np.zeros(n)
    for j, w in enumerate(stepping.frequencies(-0.4, dw, 3)):
        a, b = np.exp(0.5j * w * h), np.exp(1j * w * h)
        q = h * np.polynomial.Polynomial([(1 + 4 * a + b) / 6, (1 + 2 * a) / 6, (1 + a) / 12, 1 / 24])
        z = h * lam
        dr = (q.deriv()(z) * (b - p(z)) + q(z) * p.deriv()(z)) / (b - p(z)) ** 2
        ref += np.real(np.sum(np.conj(G[j]) * h * dr * F[j], axis=0))
    assert np.abs(fd - ref).max() < 1e-7 * np.abs(ref).max()


# ---------------------------------------------------------------------------------------------
# The paper's own Ginzburg-Landau model (Sec. 3) and its normalisation ablation.
# ---------------------------------------------------------------------------------------------
def test_paper_gl_operator_matches_pde_on_smooth_function():
    # U = 6, gamma = 1, mu_c = U^2 Re(gamma)/|gamma|^2 = 36, beta = 0.1 on (0, 40): L g must approach
    # -6 g' + g'' + 3.6 (1 - x/20) g at second order in dx (g and g' vanish at both ends).
    errs = []
    for n in (200, 400):
        L, x = operators.paper_gl_operator(n)
        a = np.pi / 40.0
        g = np.sin(a * x) ** 2
        gp = a * np.sin(2 * a * x)
        gpp = 2 * a * a * np.cos(2 * a * x)
        exact = -6.0 * gp + gpp + 3.6 * (1.0 - x / 20.0) * g
        errs.append(np.abs(L @ g - exact).max())
    assert errs[0] < 1e-2 and 3.5 < errs[0] / errs[1] < 4.5


def test_paper_gl_without_growth_has_the_real_toeplitz_spectrum():
    # beta = 0: Dirichlet tridiagonal Toeplitz with sub 1/dx^2 + 3/dx, super 1/dx^2 - 3/dx and diagonal -2/dx^2.
    # For dx < 1/3 the product of the off-diagonals is positive, so the spectrum
    # -2/dx^2 + 2 sqrt((1/dx^2)^2 - 9/dx^2) cos(m pi/(n+1)) is real.  A short domain keeps the matrix only mildly
    # non-normal (the off-diagonal ratio to the power n/2 is 2e5), so LAPACK's eigenvalues are accurate.
    n = 30
    L, x = operators.paper_gl_operator(n, beta=0.0, length=4.0)
    dx = x[1] - x[0]
    m = np.arange(1, n + 1)
    ref = -2 / dx ** 2 + 2 * np.sqrt(1 / dx ** 4 - 9 / dx ** 2) * np.cos(m * np.pi / (n + 1))
    got = np.linalg.eigvals(L.toarray())
    assert np.abs(got.imag).max() < 1e-8 * np.abs(ref).max()
    assert np.abs(np.sort(got.real) - np.sort(ref)).max() < 1e-8 * np.abs(ref).max()
    assert np.abs(L.toarray().imag).max() == 0.0


def test_globally_scaled_iteration_on_scalar_systems_closed_form():
    # N = 1: R f = r_j f, so each estimate is |r_j| and under one common scale the amplitudes grow like |r_j|^{2n}:
    # a_n(j) / a_n(0) = (|r_j| / |r_0|)^{2n} a_0(j) / a_0(0), with the largest kept at 1.
    lam = -0.7 + 0.3j
    om = np.array([0.0, 0.5, 2.0, 6.0])
    r = 1.0 / (1j * om - lam)
    apply = lambda F: F * r[:, None, None]
    adj = lambda G: G * np.conj(r)[:, None, None]
    g, amps = iteration.globally_scaled_power_iteration(apply, adj, forcing(70, 4, 1, 1), 6)
    assert np.allclose(g, np.abs(r)[None, :], rtol=1e-13)
    n = np.arange(6)[:, None]
    ref = (np.abs(r)[None, :] / np.abs(r[0])) ** (2 * n) * (amps[0] / amps[0, 0])[None, :]
    assert np.allclose(amps / amps[:, :1], ref, rtol=1e-12)
    assert np.allclose(amps.max(axis=1), 1.0, rtol=1e-14)


def test_unnormalised_iteration_saturates_on_the_paper_gl():
    # Sec. 3: without per-frequency normalisation all frequencies share one time signal.  Once the ratio of the
    # largest to the smallest spectral amplitude nears the inverse FP64 rounding unit, the small components drown
    # in the rounding of the large ones: the ratio stops growing and the high-frequency estimates drift to the
    # largest gain.  The same scheme on separate per-frequency transfer matrices keeps growing and converging, and
    # the normalised iteration on the same shared march converges.
    n = 200
    L, _ = operators.paper_gl_operator(n)
    dw, P = 5.0, 128  # frequencies 0, 5, 10, 15
    h = 2 * np.pi / (P * dw)
    om = dw * np.arange(4)
    F0 = forcing(71, 4, 1, n)
    a, ad = iteration.stepped_applies(L, h, 0.0, dw, "periodic", periods=12, stride=8)
    da, dad = iteration.dense_rk4_applies(L, h, om)
    gs, ams = iteration.globally_scaled_power_iteration(a, ad, F0, 7)
    gd, amd = iteration.globally_scaled_power_iteration(da, dad, F0, 7)
    exact = np.array([dense.gains_and_modes(dense.resolvent_rk4(L, w, h), 1)[0][0] for w in om])
    cs, cd = ams.max(1) / ams.min(1), amd.max(1) / amd.min(1)
    assert np.allclose(gs[:2], gd[:2], rtol=1e-6)            # amplitude ratio below 1e6: no loss yet
    assert cd[-1] > 1e30 and cs.max() < 1e16                  # the shared march saturates
    assert np.all(np.abs(gs[4:, 3] / exact[0] - 1) < 0.05)    # omega = 15 reads the largest gain
    # normalised on the shared march: the same estimates as the unnormalised scheme on separate frequencies
    hn = iteration.block_power_iteration(a, ad, F0, 7)[3]
    assert np.allclose(hn[:, :, 0, 0], gd, rtol=1e-8)
    assert np.abs(gd[-1, :3] / exact[:3] - 1).max() < 1e-3


# ---------------------------------------------------------------------------------------------
# Time-domain hand-off (Sec. 2.2, App. B, App. C).
# ---------------------------------------------------------------------------------------------
def test_interpolation_reproduces_polynomials():
    # C0 is exact for lines, C1 (second-order derivatives) for quadratics and C2 (five-point derivatives) for
    # quartics, away from the end samples where the one-sided rules apply.
    n = 14
    x = np.arange(n, dtype=float)
    xq = np.linspace(0.0, n - 1.0, 157)
    for scheme, deg, lo, hi in ((0, 1, 0, n - 1), (1, 2, 1, n - 2), (2, 4, 2, n - 3)):
        c = np.random.default_rng(72 + scheme).standard_normal(deg + 1)
        S = np.polyval(c, x)[:, None]
        inner = (xq >= lo) & (xq <= hi)
        got = trm.interpolate(S, xq[inner], scheme)[:, 0]
        assert np.abs(got - np.polyval(c, xq[inner])).max() < 1e-10 * np.abs(S).max()
        if scheme > 0:  # one degree more is not reproduced
            c2 = np.append(c, 0.0) + np.eye(deg + 2)[0]
            S2 = np.polyval(c2, x)[:, None]
            assert np.abs(trm.interpolate(S2, xq[inner], scheme)[:, 0] - np.polyval(c2, xq[inner])).max() > 1e-6


def test_interpolation_errors_per_points_per_cycle():
    # App. C: errors of order 1e-2 need about 4.5 points per cycle (with C2); the error falls at second, third and
    # fifth order in the sample spacing for C0, C1 and C2.
    def err(ppc, scheme):
        n = int(40 * ppc) + 1
        s = np.exp(2j * np.pi * np.arange(n) / ppc)[:, None]
        xq = np.linspace(10, n - 11, 1500)
        return np.abs(trm.interpolate(s, xq, scheme)[:, 0] - np.exp(2j * np.pi * xq / ppc)).max()
    assert 5e-3 < err(4.5, 2) < 5e-2
    for scheme, order in ((0, 2), (1, 3), (2, 5)):
        rate = err(9.0, scheme) / err(18.0, scheme)
        assert abs(np.log2(rate) - order) < 0.35


def test_interpolation_first_spurious_peak():
    # App. C: a sinusoid sampled with p points per cycle and interpolated shows its first spurious spectral peak
    # at p - 1 times its frequency (the image of the sampling frequency).
    p, cycles, fine = 4, 64, 16
    n = p * cycles + 1
    s = np.cos(2 * np.pi * np.arange(n) / p)[:, None]
    xq = np.arange((n - 1) * fine) / fine
    spec = np.abs(np.fft.rfft(trm.interpolate(s, xq, 2)[:, 0]))
    spec[cycles] = 0.0  # the signal itself
    assert np.argmax(spec) == (p - 1) * cycles


def test_signal_march_converges_to_the_scalar_closed_forms():
    # du/dt = lam u + e^{iwt} from rest: u = (e^{iwt} - e^{lam t}) / (iw - lam); the adjoint -dz/dt = conj(lam) z
    # + e^{iwt}, z(T) = 0: z = (e^{(conj(lam) + iw) T - conj(lam) t} - e^{iwt}) / (conj(lam) + iw).  With C2
    # stage forcing the error falls at third order: the first-order one-sided derivative at the end samples (App. C)
    # costs one order against RK4's fourth when the forcing does not vanish there.
    lam, w, Tend = -0.8 + 1.3j, 2.0, 4.0
    L1 = sp.csr_matrix(np.array([[lam]]))
    errs = []
    for h in (0.04, 0.02):
        every = 2
        n = int(round(Tend / (every * h))) + 1
        t = every * h * np.arange(n)
        F = np.exp(1j * w * t)[:, None, None]
        u = trm.march_signal(L1, h, F, every, 2)[:, 0, 0]
        z = trm.march_signal(L1, h, F, every, 2, adjoint=True)[:, 0, 0]
        lb = np.conj(lam)
        u_ex = (np.exp(1j * w * t) - np.exp(lam * t)) / (1j * w - lam)
        z_ex = (np.exp((lb + 1j * w) * Tend - lb * t) - np.exp(1j * w * t)) / (lb + 1j * w)
        errs.append((np.abs(u - u_ex).max(), np.abs(z - z_ex).max()))
    for a, b in zip(errs[0], errs[1]):
        assert a < 1e-4 and 6.5 < a / b < 9.5


def test_fir_design_of_a_flat_response_is_a_delta():
    # A unit response sampled on a whole period inverts to a unit impulse at the centre, where the Hamming window
    # is one: the filter is the identity.
    b = trm.fir_design(40, np.array([-1.0, 1.0]), np.array([1.0, 1.0]))
    ref = np.zeros(41)
    ref[20] = 1.0
    assert np.abs(b - ref).max() < 1e-13


def test_fir_design_is_linear_phase_and_follows_the_response():
    # App. B: a response symmetric in frequency gives real, symmetric taps (linear phase, delay n/2); with the
    # delay removed the filter approximates the desired amplitudes where they vary slowly on its resolution.
    order = 200
    nu = np.linspace(-1, 1, 41)
    D = np.exp(-(nu / 0.3) ** 2)
    b = trm.fir_design(order, nu, D)
    assert np.abs(b.imag).max() < 1e-14 and np.abs(b - b[::-1]).max() < 1e-14
    nq = np.linspace(-0.8, 0.8, 33)
    assert np.abs(trm.fir_response(b, nq) - np.interp(nq, nu, D)).max() < 1e-2


def test_fir_apply_multiplies_an_exponential_by_the_response():
    # y_t = sum_m b_m x_{t+n/2-m}: away from the ends, x_t = e^{i pi nu t} leaves as H(nu) x_t exactly.
    b = trm.fir_design(30, np.array([-1.0, -0.2, 0.4, 1.0]), np.array([0.1, 1.0, 0.3, 0.0]))
    T, nu = 200, 0.37
    x = np.exp(1j * np.pi * nu * np.arange(T))[:, None, None] * np.array([1.0, 2.0 - 1.0j])[None, :, None]
    y = trm.fir_apply(b, x)
    H = trm.fir_response(b, nu)[0]
    assert np.abs(y[15:T - 15] - H * x[15:T - 15]).max() < 1e-13


def test_trm_power_iteration_with_flattening_on_the_paper_gl():
    # Sec. 2.2, Sec. 3: with the flattening filter the spectral amplitudes stay within a small ratio and the gains
    # at omega = 0, 5, 10, 15 (and the modes) converge to the continuous resolvent's; without it the ratio grows with the squared
    # gain ratio (1e6) per iteration until the window's leakage floor, five orders of magnitude above.
    n_x = 200
    L, _ = operators.paper_gl_operator(n_x)
    h, every, n = 0.01, 4, 1501
    dt = every * h
    om = np.linspace(-15, 15, 61)
    sel = [30, 40, 50, 60]
    ex = np.array([dense.gains_and_modes(dense.resolvent(L, w), 1)[0][0] for w in om[sel]])
    F0 = forcing(73, n, 1, n_x)
    kw = dict(order=600, pad=int(12 / dt), ramp=int(6 / dt), margin=3.0, passes=2)
    g, amps, _, V, U = trm.trm_power_iteration(L, h, every, 2, F0, om, 6, want_modes=True, **kw)
    ratio = amps.max(1) / amps.min(1)
    assert ratio[1:].max() < 20
    err = np.abs(g[-1, sel] / ex - 1)
    assert err[:3].max() < 1e-3 and err[3] < 2e-2  # omega = 15: sigma_2 / sigma_1 = 0.8, slow power convergence
    for j in sel[:3]:  # the modes at omega = 0, 5, 10 are those of the continuous resolvent's SVD
        _, Us, Vs = dense.gains_and_modes(dense.resolvent(L, om[j]), 1)
        assert abs(np.vdot(Vs[:, 0], V[j, 0])) > 1 - 1e-3 and abs(np.vdot(Us[:, 0], U[j, 0])) > 1 - 1e-3
    _, amps_u, _ = trm.trm_power_iteration(L, h, every, 2, F0, om, 3, flatten=False, **kw)
    assert (amps_u.max(1) / amps_u.min(1))[-1] > 1e5
