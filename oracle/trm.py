"""The transient-response method with time-domain hand-off (Sec. 2.2, App. B and App. C); test infrastructure only.

A signal is kept as samples s_i = s(t_i), t_i = i * every * h, i = 0 .. n-1, arrays of shape (n, k, N).

* ``interpolate``: the value between samples (App. C).  With x the position in sample intervals, i the interval
  and u = x - i in [0, 1]:
    C0  linear;
    C1  cubic Hermite on values and first derivatives, the derivatives from second-order central differences
        (first-order one-sided at the two end samples);
    C2  quintic Hermite on values, first and second derivatives, the derivatives from five-point central
        differences; at the end samples a first-order one-sided first derivative and a zero second derivative, at
        the samples next to them second-order central differences.
  Derivatives are per sample interval.
* ``march_signal``: the classical four-stage RK4 from rest, du/dt = L u + f(t), each stage forced by the
  interpolated signal at its own time (t, t + h/2, t + h/2, t + h); returns the state at the sample times.  The
  adjoint run solves -dz/dt = L^H z + g(t) backward in time from z(T) = 0, T = (n - 1) every h (Sec. 2.1, eq.
  adsystem with B = C = I): with tau = T - t it is the forward march of L^H forced by g(T - tau).
* ``fir_design``: a linear-phase FIR filter of even order n (n + 1 taps) approximating a desired amplitude
  response (App. B, the design the paper takes from fir2): the response, given at breakpoints nu in [-1, 1]
  (frequency over the Nyquist frequency pi / dt) and linear between them, is sampled on M uniform frequencies
  nu_q = -1 + 2q/M; the taps are its inverse discrete transform delayed by n/2 samples, times a Hamming window:
      b_m = w_m (1/M) sum_q D(nu_q) e^{i pi nu_q (m - n/2)},   w_m = 0.54 - 0.46 cos(2 pi m / n).
  A response symmetric in nu gives real taps.
* ``fir_apply``: the filter with its n/2-sample delay removed, y_t = sum_m b_m x_{t + n/2 - m} (zero outside the
  series), so that a complex exponential of frequency nu leaves multiplied by H(nu) = sum_m b_m e^{-i pi nu (m-n/2)}.
* ``dft``: X(w) = dt sum_i x_i e^{-i w t_i} at any frequencies.
* ``trm_power_iteration``: the power iteration of Sec. 2.2 / App. A with time-domain hand-off: the direct run's
  response forces the adjoint run, whose output, normalised in frequency by a flattening FIR filter designed from
  its own spectrum (Sec. 2.2, App. B) and tapered to a compact window, forces the next direct run.
"""
import numpy as np


# ---------------------------------------------------------------------------------------------
# App. C: interpolation between samples
# ---------------------------------------------------------------------------------------------
def sample_derivatives(S, scheme):
    """First and second derivatives (per sample interval) at every sample of S (n, ...) for scheme 1 or 2."""
    n = S.shape[0]
    d = np.zeros_like(S)
    dd = np.zeros_like(S)
    if n < 2:
        raise ValueError("need at least two samples")
    d[0] = S[1] - S[0]
    d[n - 1] = S[n - 1] - S[n - 2]
    if scheme == 1:
        for i in range(1, n - 1):
            d[i] = (S[i + 1] - S[i - 1]) / 2.0
    elif scheme == 2:
        for i in range(1, n - 1):
            if i == 1 or i == n - 2:
                d[i] = (S[i + 1] - S[i - 1]) / 2.0
                dd[i] = S[i + 1] - 2.0 * S[i] + S[i - 1]
            else:
                d[i] = (S[i - 2] - 8.0 * S[i - 1] + 8.0 * S[i + 1] - S[i + 2]) / 12.0
                dd[i] = (-S[i - 2] + 16.0 * S[i - 1] - 30.0 * S[i] + 16.0 * S[i + 1] - S[i + 2]) / 12.0
    return d, dd


def interpolate(S, x, scheme):
    """Values of the sampled signal S (n, ...) at fractional sample positions x (1-D array in [0, n-1])."""
    n = S.shape[0]
    d, dd = sample_derivatives(S, scheme) if scheme > 0 else (None, None)
    out = np.empty((len(x),) + S.shape[1:], dtype=np.result_type(S, float))
    for q, xq in enumerate(x):
        i = min(int(np.floor(xq)), n - 2)
        u = xq - i
        if scheme == 0:
            out[q] = (1.0 - u) * S[i] + u * S[i + 1]
        elif scheme == 1:
            h00 = 2 * u ** 3 - 3 * u ** 2 + 1
            h10 = u ** 3 - 2 * u ** 2 + u
            h01 = -2 * u ** 3 + 3 * u ** 2
            h11 = u ** 3 - u ** 2
            out[q] = h00 * S[i] + h10 * d[i] + h01 * S[i + 1] + h11 * d[i + 1]
        else:
            H0 = 1 - 10 * u ** 3 + 15 * u ** 4 - 6 * u ** 5
            H1 = u - 6 * u ** 3 + 8 * u ** 4 - 3 * u ** 5
            H2 = (u ** 2 - 3 * u ** 3 + 3 * u ** 4 - u ** 5) / 2
            H3 = 10 * u ** 3 - 15 * u ** 4 + 6 * u ** 5
            H4 = -4 * u ** 3 + 7 * u ** 4 - 3 * u ** 5
            H5 = (u ** 3 - 2 * u ** 4 + u ** 5) / 2
            out[q] = (H0 * S[i] + H1 * d[i] + H2 * dd[i] + H3 * S[i + 1] + H4 * d[i + 1] + H5 * dd[i + 1])
    return out


# ---------------------------------------------------------------------------------------------
# Direct and adjoint runs forced by a sampled signal
# ---------------------------------------------------------------------------------------------
def march_signal(L, h, F, every, scheme, adjoint=False):
    """State samples (n, k, N) of the run forced by the samples F (n, k, N), from rest (see the module notes)."""
    n, k, N = F.shape
    A = L.conj().T.tocsr() if adjoint else L
    G = F[::-1] if adjoint else F
    S = (n - 1) * every
    half = interpolate(G, np.arange(2 * S + 1) / (2.0 * every), scheme)  # forcing on the half-step grid
    u = np.zeros((N, k), dtype=complex)
    out = np.zeros((n, k, N), dtype=complex)
    for s in range(S):
        fa, fb, fc = half[2 * s].T, half[2 * s + 1].T, half[2 * s + 2].T
        k1 = A @ u + fa
        k2 = A @ (u + 0.5 * h * k1) + fb
        k3 = A @ (u + 0.5 * h * k2) + fb
        k4 = A @ (u + h * k3) + fc
        u = u + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        if (s + 1) % every == 0:
            out[(s + 1) // every] = u.T
    return out[::-1] if adjoint else out


# ---------------------------------------------------------------------------------------------
# App. B: FIR filters
# ---------------------------------------------------------------------------------------------
def fir_grid_size(order):
    """Number of uniform design frequencies over [-1, 1)."""
    return 2 * max(512, 1 << int(np.ceil(np.log2(max(order, 2)))))


def fir_design(order, nu, gain):
    """Complex taps b (order + 1,) for the desired amplitudes `gain` at breakpoints `nu` (ascending, in [-1, 1])."""
    if order < 2 or order % 2:
        raise ValueError("the order must be even and >= 2")
    M = fir_grid_size(order)
    nq = -1.0 + 2.0 * np.arange(M) / M
    D = np.interp(nq, nu, gain)
    m = np.arange(order + 1)
    w = 0.54 - 0.46 * np.cos(2 * np.pi * m / order)
    b = np.array([np.sum(D * np.exp(1j * np.pi * nq * (mm - order / 2))) / M for mm in m])
    return w * b


def fir_response(b, nu):
    """H(nu) = sum_m b_m e^{-i pi nu (m - n/2)} of the delay-compensated filter."""
    n = len(b) - 1
    m = np.arange(n + 1)
    return np.array([np.sum(b * np.exp(-1j * np.pi * v * (m - n / 2))) for v in np.atleast_1d(nu)])


def fir_apply(b, X):
    """y_t = sum_m b_m x_{t + n/2 - m} along axis 0, zero outside the series."""
    n = len(b) - 1
    T = X.shape[0]
    Y = np.zeros(X.shape, dtype=complex)
    for m in range(n + 1):
        sh = n // 2 - m  # y_t += b_m x_{t + sh}
        lo, hi = max(0, -sh), min(T, T - sh)
        if hi > lo:
            Y[lo:hi] += b[m] * X[lo + sh:hi + sh]
    return Y


def dft(X, omegas, dt):
    """X(w_j) = dt sum_i x_i e^{-i w_j t_i}, t_i = i dt, for X (n, ...); returns (n_w, ...)."""
    t = dt * np.arange(X.shape[0])
    E = np.exp(-1j * np.outer(omegas, t))
    return dt * np.tensordot(E, X, axes=(1, 0))


# ---------------------------------------------------------------------------------------------
# Power iteration with time-domain hand-off
# ---------------------------------------------------------------------------------------------
def taper(n, pad, ramp):
    """Window of n samples: zero on the first and last `pad`, raised-cosine ramps of `ramp` samples, one between."""
    w = np.zeros(n)
    for i in range(n):
        a = min(i, n - 1 - i) - pad
        if a < 0:
            w[i] = 0.0
        elif a < ramp:
            w[i] = 0.5 - 0.5 * np.cos(np.pi * (a + 0.5) / ramp)
        else:
            w[i] = 1.0
    return w


def flattening_breakpoints(omegas, Wh_norm, dt, margin):
    """Breakpoints (nu, D) of the flattening response: D = 1/||W(w_j)|| (largest 1) at the analysis frequencies,
    falling linearly to zero `margin` (rad per time unit) outside them and zero beyond."""
    nu = np.asarray(omegas) * dt / np.pi
    D = 1.0 / Wh_norm
    D = D / D.max()
    order = np.argsort(nu)
    nu, D = nu[order], D[order]
    dm = margin * dt / np.pi
    lo, hi = max(-1.0, nu[0] - dm), min(1.0, nu[-1] + dm)
    pts = [(-1.0, 0.0)] if lo > -1.0 else []
    pts += [(lo, 0.0)] + list(zip(nu, D)) + [(hi, 0.0)]
    if hi < 1.0:
        pts.append((1.0, 0.0))
    x = np.array([p[0] for p in pts])
    y = np.array([p[1] for p in pts])
    return x, y


def trm_power_iteration(L, h, every, scheme, F0, omegas, iters, order, pad, ramp, margin, passes=1, flatten=True,
                        want_modes=False, runs=None):
    """Returns (gains (iters, n_w): ||Y(w_j)|| / ||F(w_j)|| of each iteration's forcing, amplitudes (iters, n_w):
    ||F(w_j)|| of each iteration's forcing, F the last forcing series), and with want_modes also the force and
    response modes of the last iteration at the analysis frequencies, V = F(w_j) / ||F(w_j)|| and
    U = Y(w_j) / ||Y(w_j)|| (n_w, k, N).  F0 (n, k, N) is tapered first.  `runs` = (direct, adjoint) maps of
    sample series replace the signal runs of L (e.g. with input and output matrices wrapped around them)."""
    n = F0.shape[0]
    dt = every * h
    win = taper(n, pad, ramp)[:, None, None]
    F = win * F0
    F = F / np.linalg.norm(F)
    gains = np.zeros((iters, len(omegas)))
    amps = np.zeros((iters, len(omegas)))
    if runs is None:
        runs = (lambda X: march_signal(L, h, X, every, scheme),
                lambda X: march_signal(L, h, X, every, scheme, adjoint=True))
    for it in range(iters):
        Y = runs[0](F)
        W = runs[1](Y)
        Fs, Ys = dft(F, omegas, dt), dft(Y, omegas, dt)
        Fh = np.linalg.norm(Fs.reshape(len(omegas), -1), axis=1)
        Yh = np.linalg.norm(Ys.reshape(len(omegas), -1), axis=1)
        Wh = np.linalg.norm(dft(W, omegas, dt).reshape(len(omegas), -1), axis=1)
        gains[it] = Yh / Fh
        amps[it] = Fh
        V, U = Fs / Fh[:, None, None], Ys / Yh[:, None, None]
        if flatten:
            nu, D = flattening_breakpoints(omegas, Wh, dt, margin)
            b = fir_design(order, nu, D ** (1.0 / passes))
            for _ in range(passes):
                W = fir_apply(b, W)
        F = win * W
        F = F / np.linalg.norm(F)
    if want_modes:
        return gains, amps, F, V, U
    return gains, amps, F
