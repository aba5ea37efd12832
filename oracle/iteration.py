"""Block power iteration with frequency-domain normalisation and Rayleigh-Ritz estimates
(test infrastructure only).

The paper's power iteration (Appendix A, eqs. iteration and powerMethod) feeds the adjoint output of one
iteration back as the forcing of the next, f_n = w_{n-1} with w = R^H R f.  The SSRM normalises and
orthogonalises on the Fourier coefficients (Sec. 2.3), and the low-rank representation of R^H R on the span
of the forcings gives gains and modes (Appendix A, eqs. RRFi / arDec and the estimates that follow them).
With k columns per frequency kept orthonormal this is the block (subspace) form of the same iteration:

  1. F  = Q of QR(F_hat)                         (orthonormal forcings, diag R > 0)
  2. Y  = R F                                    (direct run)
  3. Y  = Q_Y R_Y;  R_Y = Phi Sigma Psi^H        (k x k SVD)
       gains = diag Sigma,  V = F Psi (force modes),  U = Q_Y Phi (response modes)
     Since F^H R^H R F = R_Y^H R_Y, Psi and Sigma^2 are the eigenvectors and eigenvalues of the paper's
     H = Q_F^H W R_F^{-1} with R_F = I, so these are its estimates V~ = F psi, U~ = gamma^{-1} R F psi,
     sigma~ = gamma.
  4. Z  = R^H Q_Y                                (adjoint run, forced by the normalised response)
     W  = Z R_Y = R^H R F
  5. F_hat = W Psi                               (next forcing, columns ordered by gain)

The history also keeps the paper's norm-ratio estimate (eq. tildeSig) sqrt(||f_n|| / ||f_{n-1}||) for every
column, which with unit-norm F is sqrt(||F_hat_{:,i}||).
``apply`` / ``adjoint_apply`` map (n_w, k, N) arrays of per-frequency forcings to responses; they can be the
time-stepped runs of ``stepping`` or the dense R_d of ``dense``.
"""
import numpy as np


def qr_positive(A):
    """Householder QR (LAPACK) of A (N, k) with the diagonal of R made real and non-negative."""
    Q, R = np.linalg.qr(A)
    d = np.diag(R)
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1.0), 1.0)
    return Q * ph[None, :], R * ph.conj()[:, None]


def block_power_iteration(apply, adjoint_apply, F0, iters):
    """Returns (gains (n_w, k), V (n_w, k, N), U (n_w, k, N), hist (iters, n_w, k, 2))."""
    nw, k, N = F0.shape
    Fhat = np.array(F0, dtype=complex)
    hist = np.zeros((iters, nw, k, 2))
    gains = np.zeros((nw, k))
    V = np.zeros((nw, k, N), complex)
    U = np.zeros((nw, k, N), complex)
    for n in range(iters):
        F = np.empty_like(Fhat)
        for j in range(nw):
            F[j] = qr_positive(Fhat[j].T)[0].T
        Y = apply(F)
        QY = np.empty_like(Y)
        RY = np.empty((nw, k, k), complex)
        Psi = np.empty((nw, k, k), complex)
        for j in range(nw):
            Q, Rj = qr_positive(Y[j].T)
            Phi, S, PsiH = np.linalg.svd(Rj)
            gains[j] = S
            Psi[j] = PsiH.conj().T
            RY[j] = Rj
            QY[j] = Q.T
            U[j] = (Q @ Phi).T
            V[j] = (F[j].T @ Psi[j]).T
        Z = adjoint_apply(QY)
        for j in range(nw):
            W = Z[j].T @ RY[j]
            Fhat[j] = (W @ Psi[j]).T
        hist[n, :, :, 0] = gains
        hist[n, :, :, 1] = np.sqrt(np.linalg.norm(Fhat, axis=2))
    return gains, V, U, hist


def globally_scaled_power_iteration(apply, adjoint_apply, F0, iters):
    """The power iteration without frequency normalisation, the unregularised scheme of Sec. 3: w = R^H R f is
    handed back as the next forcing with one common scale for all frequencies, as a hand-off of the adjoint run's
    time signal does (the scale only keeps the largest frequency's norm at 1).  One column per frequency
    (F0 of shape (n_w, 1, N)).  Returns (gains (iters, n_w), amplitudes (iters, n_w)): the estimate
    ||R f_j|| / ||f_j|| and the norm ||f_j|| of the forcing each iteration starts from."""
    nw, k, N = F0.shape
    if k != 1:
        raise ValueError("one column per frequency")
    F = np.array(F0, dtype=complex)
    F /= np.linalg.norm(F, axis=2).max()
    gains = np.zeros((iters, nw))
    amps = np.zeros((iters, nw))
    for n in range(iters):
        amps[n] = np.linalg.norm(F[:, 0], axis=1)
        Y = apply(F)
        gains[n] = np.linalg.norm(Y[:, 0], axis=1) / amps[n]
        W = adjoint_apply(Y)
        F = W / np.linalg.norm(W, axis=2).max()
    return gains, amps


def dense_rk4_applies(L, h, omegas):
    """(apply, adjoint_apply) with the exact RK4 transfer matrices R_d(w_j) (see ``dense.resolvent_rk4``)."""
    from .dense import resolvent_rk4
    Rd = [resolvent_rk4(L, w, h) for w in omegas]

    def apply(F):
        return np.stack([(Rd[j] @ F[j].T).T for j in range(len(Rd))])

    def adjoint_apply(G):
        return np.stack([(Rd[j].conj().T @ G[j].T).T for j in range(len(Rd))])

    return apply, adjoint_apply


def stepped_applies(L, h, w0, dw, method, **run_kw):
    """(apply, adjoint_apply) with the explicit time-stepped runs of ``stepping.run``."""
    from .stepping import run

    def apply(F):
        return run(L, h, w0, dw, F, method, adjoint=False, **run_kw)

    def adjoint_apply(G):
        return run(L, h, w0, dw, G, method, adjoint=True, **run_kw)

    return apply, adjoint_apply
