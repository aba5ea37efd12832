"""Sensitivity of resolvent gains to the reaction field mu (test infrastructure only).

The reaction field enters L on its diagonal, L(mu) = L_0 + diag(mu) with mu real.

* ``leading_gain_sensitivity`` -- closed form for the continuous resolvent R = (i w I - L)^{-1} with
  B = C = W = I:  dR = R dL R, R v_1 = sigma_1 u_1 and R^H u_1 = sigma_1 v_1 give
  d sigma_1 = Re(u_1^H dR v_1) = sigma_1^2 Re(v_1^H dL u_1), i.e.
  d sigma_1 / d mu(x) = sigma_1^2 Re(conj(v_1(x)) u_1(x))   (simple leading gain).
* ``discrete_objective``       -- J(mu) = sum_j c_j || R_d(w_j; mu) V_j ||, the objective the autograd path
  differentiates, with the exact RK4 transfer matrix R_d of ``dense`` and fixed forcings V_j.  With V_j the
  leading force mode this is sum_j c_j sigma_1(w_j) and, the mode being stationary, has the same gradient.
* ``central_difference_gradient`` / ``central_difference_directional`` -- brute-force derivatives of any
  scalar function of mu.

Reverse mode of the time-stepped run (the run map A: F -> U of ``stepping.run`` is complex-linear in F, one
column at a time):

* ``stepped_transfer``  -- the matrix of A for one column, assembled column by column from runs on unit forcings
  (one batched run: column c of the batch is the unit forcing of frequency j = c // N at unknown i = c % N);
* ``stepped_vjp``       -- A^H G, the gradient of J = Re sum conj(G) A(F) with respect to F (convention
  dJ/dRe + i dJ/dIm), from that matrix;
* ``stepped_objective`` / ``stepped_mu_gradient`` -- J(mu) = Re sum conj(G) A(mu) F with L(mu) = L_0 + diag(mu)
  and its gradient by central differences, one entry of mu at a time.
"""
import numpy as np
import scipy.sparse as sp

from . import stepping
from .dense import resolvent, gains_and_modes, resolvent_rk4


def leading_gain_sensitivity(L, w):
    s, U, V = gains_and_modes(resolvent(L, w), 1)
    return s[0] ** 2 * np.real(np.conj(V[:, 0]) * U[:, 0])


def discrete_objective(L_of_mu, mu, h, omegas, V, c):
    """V: (n_w, N) forcings; c: (n_w,) weights."""
    L = L_of_mu(mu)
    return float(sum(c[j] * np.linalg.norm(resolvent_rk4(L, w, h) @ V[j]) for j, w in enumerate(omegas)))


def central_difference_gradient(fun, mu, eps):
    mu = np.asarray(mu, float)
    g = np.zeros_like(mu)
    flat = g.reshape(-1)
    for i in range(mu.size):
        e = np.zeros(mu.size)
        e[i] = eps
        e = e.reshape(mu.shape)
        flat[i] = (fun(mu + e) - fun(mu - e)) / (2.0 * eps)
    return g


def central_difference_directional(fun, mu, delta, eps):
    return (fun(mu + eps * delta) - fun(mu - eps * delta)) / (2.0 * eps)


def stepped_transfer(L, h, w0, dw, n_omega, method, **run_kw):
    """(n_omega N) x (n_omega N) matrix T of the time-stepped run of one column: run(F)[j', i'] =
    sum_{j, i} T[j' N + i', j N + i] F[j, i]."""
    N = L.shape[0]
    n = n_omega * N
    E = np.zeros((n_omega, n, N), complex)
    for j in range(n_omega):
        for i in range(N):
            E[j, j * N + i, i] = 1.0
    U = stepping.run(L, h, w0, dw, E, method, **run_kw)  # (n_omega, n, N): column c = response to unit c
    return U.transpose(0, 2, 1).reshape(n, n)


def stepped_vjp(L, h, w0, dw, G, method, **run_kw):
    """A^H G for G (n_omega, k, N): the forcing gradient of Re sum conj(G) run(F)."""
    nw, k, N = G.shape
    T = stepped_transfer(L, h, w0, dw, nw, method, **run_kw)
    out = np.empty_like(G, dtype=complex)
    for b in range(k):
        out[:, b, :] = (T.conj().T @ G[:, b, :].reshape(-1)).reshape(nw, N)
    return out


def expand_node_field(mu_nodes, ncomp):
    """A per-node field acting on every component of a component-outermost state (ncomp blocks of nodes)."""
    return np.tile(np.asarray(mu_nodes, float).ravel(), ncomp)


def stepped_objective(L0, mu, h, w0, dw, F, G, method, ncomp=1, **run_kw):
    """J(mu) = Re sum conj(G) run(L0 + diag(mu), F); with ncomp > 1, mu is a node field shared by the
    components."""
    d = expand_node_field(mu, ncomp)
    L = (sp.csr_matrix(L0) + sp.diags(d)).tocsr()
    U = stepping.run(L, h, w0, dw, F, method, **run_kw)
    return float(np.real(np.sum(np.conj(G) * U)))


def stepped_mu_gradient(L0, mu, h, w0, dw, F, G, method, eps=1e-5, ncomp=1, **run_kw):
    """dJ/dmu of ``stepped_objective`` by central differences, entry by entry."""
    J = lambda m: stepped_objective(L0, m, h, w0, dw, F, G, method, ncomp=ncomp, **run_kw)
    return central_difference_gradient(J, np.asarray(mu, float), eps)


def stepped_mu_directional(L0, mu, delta, h, w0, dw, F, G, method, eps=1e-5, ncomp=1, **run_kw):
    """Directional derivative of ``stepped_objective`` along delta by central differences."""
    J = lambda m: stepped_objective(L0, m, h, w0, dw, F, G, method, ncomp=ncomp, **run_kw)
    return central_difference_directional(J, np.asarray(mu, float), np.asarray(delta, float), eps)
