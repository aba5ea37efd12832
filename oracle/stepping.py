"""Explicit RK4 time marching of the direct and adjoint systems, all frequencies at once
(test infrastructure only).

What is computed (Sec. 2.1 last paragraphs, Sec. 2.2, Sec. 2.3):

* the forcing is the Fourier sum f(t) = sum_j F_j e^{i w_j t} over a uniform frequency grid
  w_j = w_0 + j dw, j = 0..n_w-1 (the complex branch of eq. forceFseries, written with the
  e^{+i w t} convention of this library), evaluated at the classical RK4 stage times t, t+h/2, t+h/2, t+h;
* the state starts from u = 0 and is marched with classical RK4, dt = h;
* the Fourier coefficients of the response are the sums  U_j = (1/M) sum_s u_s e^{-i w_j t_s}  over a set of
  M' samples (defined below), i.e. a direct evaluation of eq. fourier.

Frequency grid: a period of T = P h with integer P gives dw = 2 pi / (P h) (Sec. 2.3: w_k = 2 pi k / T);
w_0 need not lie on the harmonic grid.

Two schedules:

* transient (TRM with a one-window forcing, Sec. 2.2): the forcing is on for the P steps s = 0..P-1 and off
  afterwards, the run continues for ``tail`` further steps while the response decays, and every step is
  projected: U_j = (1/P) sum_{s=0}^{P+tail-1} u_s e^{-i w_j t_s}.  Because the window holds exactly one period
  of every difference frequency, the Fourier transform of the forcing at w_j is P h F_j, which the 1/P
  normalisation removes; truncation leaves an error proportional to the state at the end (Sec. 2.2).
* periodic (SSRM, Sec. 2.3): the forcing is on throughout ``periods`` periods, the first periods-1 let the
  transient die out, and the last period is projected at every ``stride``-th step:
  U_j = (stride/P) sum_{m} u_{s_m} e^{-i w_j t_{s_m}},  s_m = (periods-1) P + m*stride.
  For a periodic steady state this is exact as long as P/stride >= n_w (no two grid frequencies alias).

Adjoint run (Sec. 2.1, eq. adsystem / adsystemFreqDomain): the same march with L^H and the frequencies
negated, which yields R_d(w)^H applied to the forcing (R_d(-w; L^H) = R_d(w; L)^H because all the matrices
involved are polynomials in one operator).  It replaces the paper's backward-in-time integration by the
equivalent forward march in reversed time tau = T - t.
"""
import numpy as np


def period_steps(domega, h):
    """P with |domega| * P * h = 2 pi; raises if the grid is not commensurate with h."""
    P = int(round(2.0 * np.pi / (abs(domega) * h)))
    if P < 1 or abs(abs(domega) * P * h - 2.0 * np.pi) > 1e-9 * 2.0 * np.pi:
        raise ValueError("frequency spacing is not 2 pi / (P h) for an integer P")
    return P


def snap_grid(wmin, wmax, n_omega, h, stride=1):
    """Nominal n_omega frequencies in [wmin, wmax] -> (w0, dw, P) with dw = 2 pi/(P h), P a multiple of stride."""
    dw_nom = (wmax - wmin) / (n_omega - 1)
    P = stride * int(round(2.0 * np.pi / (dw_nom * h * stride)))
    return wmin, 2.0 * np.pi / (P * h), P


def frequencies(w0, dw, n_omega):
    return w0 + dw * np.arange(n_omega)


def march(L, h, omegas, F, n_steps, forced, projected, norm):
    """Classical RK4 from u = 0 with stage-time forcing sum_j F_j e^{i w_j t} on the steps where
    ``forced(s)`` holds, and Fourier projection of u_s on the steps where ``projected(s)`` holds.

    L: (N, N) sparse or dense;  omegas: (n_w,);  F: (n_w, k, N) complex.  Returns (U (n_w, k, N), u_end).
    """
    nw, k, N = F.shape
    Fm = np.ascontiguousarray(F.transpose(0, 2, 1).reshape(nw, N * k))  # row j = F_j as (N, k)

    def force(t):
        return (np.exp(1j * omegas * t) @ Fm).reshape(N, k)

    u = np.zeros((N, k), complex)
    acc = np.zeros((nw, N * k), complex)
    for s in range(n_steps):
        t = s * h
        if projected(s):
            acc += np.exp(-1j * omegas * t)[:, None] * u.reshape(1, -1)
        if forced(s):
            f0, fh, f1 = force(t), force(t + 0.5 * h), force(t + h)
        else:
            f0 = fh = f1 = 0.0
        k1 = L @ u + f0
        k2 = L @ (u + 0.5 * h * k1) + fh
        k3 = L @ (u + 0.5 * h * k2) + fh
        k4 = L @ (u + h * k3) + f1
        u = u + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    U = (acc / norm).reshape(nw, N, k).transpose(0, 2, 1)
    return np.ascontiguousarray(U), u.T.copy()


def transient_run(L, h, omegas, F, P, tail):
    """One-window transient-response run: force P steps, march P + tail steps, project all of them."""
    return march(L, h, omegas, F, P + tail, lambda s: s < P, lambda s: True, float(P))


def periodic_run(L, h, omegas, F, P, periods, stride=1):
    """Steady-state-response run: force throughout, project the last period every ``stride`` steps."""
    if P % stride != 0:
        raise ValueError("stride must divide P")
    first = (periods - 1) * P
    return march(L, h, omegas, F, periods * P, lambda s: True,
                 lambda s: s >= first and (s - first) % stride == 0, P / stride)


def run(L, h, w0, dw, F, method, adjoint=False, tail=0, periods=2, stride=1):
    """resolvent_apply / resolvent_adjoint_apply of the oracle: R_d(w_j) F_j or R_d(w_j)^H F_j for all j."""
    nw = F.shape[0]
    P = period_steps(dw, h)
    om = frequencies(w0, dw, nw)
    if adjoint:
        L = L.conj().T
        om = -om
    if method == "transient":
        return transient_run(L, h, om, F, P, tail)[0]
    if method == "periodic":
        return periodic_run(L, h, om, F, P, periods, stride)[0]
    raise ValueError(method)
