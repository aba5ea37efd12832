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
"""
import numpy as np

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
