"""Dense ground truth (test infrastructure only).

* ``resolvent``          -- R(w) = (i w I - L)^{-1}.  This is the paper's R = (-i w I + A)^{-1} of
                            Sec. 2.1 (eq. systemFreqDomain) with A = -L, taken with the forcing
                            convention f(t) = sum f_w e^{+i w t}; the paper's Fourier convention
                            (eq. fourier) gives the same operator at -w.
* ``gains_and_modes``    -- SVD R_y = U Sigma V^H: gains sigma_1 >= sigma_2 >= ..., response modes U,
                            force modes V (Sec. 2.1).
* ``rk4_amplification``  -- P(Z) = I + Z + Z^2/2 + Z^3/6 + Z^4/24, the classical RK4 step matrix of
                            du/dt = L u for Z = h L.
* ``rk4_forcing_matrix`` -- h Q_w(Z), the matrix taking a forcing amplitude F (forcing F e^{i w t},
                            evaluated at the RK4 stage times t, t+h/2, t+h/2, t+h) to its contribution to
                            u_{s+1} e^{-i w t_s}.  Derived by expanding the four stages.
* ``resolvent_rk4``      -- R_d(w) = (e^{i w h} I - P(Z))^{-1} h Q_w(Z): the exact steady response of
                            the RK4-discretised system to F e^{i w t}, i.e. the operator the time-stepped
                            method computes once transients have died out.  R_d -> R as h^4.
* ``rk4_steady_residual`` -- e^{i w h} u - P(Z) u - h Q_w(Z) f by matrix-vector products, zero exactly when
                            u = R_d(w) f: checks a steady response at sizes where R_d cannot be formed.
"""
import numpy as np


def _dense(L):
    return L.toarray() if hasattr(L, "toarray") else np.asarray(L)


def resolvent(L, w):
    L = _dense(L).astype(complex)
    n = L.shape[0]
    return np.linalg.inv(1j * w * np.eye(n) - L)


def gains_and_modes(R, k=None):
    """SVD of R: returns (sigma[:k], U[:, :k], V[:, :k]) with R V_i = sigma_i U_i."""
    U, s, Vh = np.linalg.svd(R)
    if k is None:
        k = len(s)
    return s[:k], U[:, :k], Vh.conj().T[:, :k]


def rk4_amplification(Z):
    n = Z.shape[0]
    I = np.eye(n)
    Z2 = Z @ Z
    Z3 = Z2 @ Z
    Z4 = Z3 @ Z
    return I + Z + Z2 / 2.0 + Z3 / 6.0 + Z4 / 24.0


def rk4_forcing_matrix(Z, w, h):
    """h Q_w(Z) with a = e^{i w h/2}, b = e^{i w h}:

        Q_w(Z) = [ (1 + 4a + b) I + (1 + 2a) Z + (1 + a) Z^2 / 2 + Z^3 / 4 ] / 6.

    Expanding the stages with g = h F e^{i w t_s}:  h k1 = g,  h k2 = (Z/2 + a) g,
    h k3 = (Z^2/4 + a Z/2 + a) g,  h k4 = (Z^3/4 + a Z^2/2 + a Z + b) g, and
    u_{s+1} - P(Z) u_s = (h k1 + 2 h k2 + 2 h k3 + h k4)/6 (forcing part).
    """
    n = Z.shape[0]
    I = np.eye(n)
    a = np.exp(1j * w * h / 2.0)
    b = np.exp(1j * w * h)
    Z2 = Z @ Z
    Z3 = Z2 @ Z
    return h * ((1 + 4 * a + b) * I + (1 + 2 * a) * Z + (1 + a) * Z2 / 2.0 + Z3 / 4.0) / 6.0


def resolvent_rk4(L, w, h):
    Z = h * _dense(L).astype(complex)
    n = Z.shape[0]
    return np.linalg.solve(np.exp(1j * w * h) * np.eye(n) - rk4_amplification(Z),
                           rk4_forcing_matrix(Z, w, h))


def rk4_steady_residual(L, w, h, u, f):
    """e^{i w h} u - P(Z) u - h Q_w(Z) f with Z = h L (sparse or dense), the polynomials of rk4_amplification and
    rk4_forcing_matrix applied by repeated products with L."""
    a = np.exp(1j * w * h / 2.0)
    b = np.exp(1j * w * h)
    u = np.asarray(u, dtype=complex)
    f = np.asarray(f, dtype=complex)
    z1 = h * (L @ u)
    z2 = h * (L @ z1)
    z3 = h * (L @ z2)
    z4 = h * (L @ z3)
    Pu = u + z1 + z2 / 2.0 + z3 / 6.0 + z4 / 24.0
    g1 = h * (L @ f)
    g2 = h * (L @ g1)
    g3 = h * (L @ g2)
    Qf = h * ((1 + 4 * a + b) * f + (1 + 2 * a) * g1 + (1 + a) * g2 / 2.0 + g3 / 4.0) / 6.0
    return b * u - Pu - Qf
