"""Arnoldi (Krylov-subspace) estimates of resolvent gains and modes on the steady-state response method
(test infrastructure only).

Appendix A: instead of feeding w_{n-1} = R^H R f_{n-1} back unchanged (the power iteration), the Arnoldi
algorithm takes as the next forcing f_n the part of w_{n-1} orthogonal to all earlier forcings (eq. freqOrt,
Euclidean weight), normalised.  With the forcings orthonormal, F = Q_F and R_F = I, so the low-rank
representation of R^H R on span(F) is H = F^H W (eq. arDec), and its eigen-decomposition H Psi = Gamma^2 Psi
gives the estimates (the equations after eq. arDec)

    V~_i = F psi_i,    U~_i = gamma_i^{-1} R F psi_i,    sigma~_i = gamma_i.

Block form, as the power iteration here: each f_n is a block of k orthonormal columns per frequency (k = 1 is
the paper's sequence).  The orthogonalisation is classical Gram-Schmidt applied twice, then a QR of what is
left.  H is Hermitian in exact arithmetic; it is formed from the coefficients B_i^H W_j with i <= j (its upper
block triangle) and mirrored.  ``apply`` / ``adjoint_apply`` map (n_w, k, N) arrays to (n_w, k, N) arrays (the
time-stepped runs of ``stepping`` or the dense R_d of ``dense``).
"""
import numpy as np

from .iteration import qr_positive


def hermitian_from_upper(T):
    """The Hermitian matrix whose upper triangle (diagonal included, imaginary part of the diagonal dropped) is
    that of T."""
    H = np.triu(T) + np.triu(T, 1).conj().T
    H[np.diag_indices_from(H)] = np.real(np.diag(T))
    return H


def ritz(T, k):
    """Top-k eigenpairs of the Hermitian completion of T: (gamma (k,), Psi (n, k)), gamma = sqrt(eigenvalue)."""
    lam, Psi = np.linalg.eigh(hermitian_from_upper(T))
    order = np.argsort(lam)[::-1][:k]
    return np.sqrt(np.maximum(lam[order], 0.0)), Psi[:, order]


def block_arnoldi(apply, adjoint_apply, F0, blocks):
    """Returns (gains (n_w, k), V (n_w, k, N), U (n_w, k, N), hist (blocks, n_w, k)): the top-k estimates after
    `blocks` blocks of k forcings (blocks direct and blocks adjoint runs), and those after each block."""
    nw, k, N = F0.shape
    if blocks * k > N:
        raise ValueError("more basis columns than unknowns")
    basis = [[qr_positive(np.asarray(F0[j], complex).T)[0]] for j in range(nw)]  # per frequency: N x k blocks
    Ys = []
    T = np.zeros((nw, blocks * k, blocks * k), complex)
    hist = np.zeros((blocks, nw, k))
    for i in range(blocks):
        Bi = np.stack([basis[j][i].T for j in range(nw)])
        Y = apply(Bi)
        W = adjoint_apply(Y)
        Ys.append(Y)
        for j in range(nw):
            Q = np.hstack(basis[j])
            w = W[j].T
            C = Q.conj().T @ w
            T[j, :(i + 1) * k, i * k:(i + 1) * k] = C
            hist[i, j] = ritz(T[j, :(i + 1) * k, :(i + 1) * k], k)[0]
            if i + 1 < blocks:
                w = w - Q @ C
                w = w - Q @ (Q.conj().T @ w)
                basis[j].append(qr_positive(w)[0])
    gains = np.zeros((nw, k))
    V = np.zeros((nw, k, N), complex)
    U = np.zeros((nw, k, N), complex)
    for j in range(nw):
        g, Psi = ritz(T[j], k)
        Q = np.hstack(basis[j])
        Yj = np.hstack([Ys[i][j].T for i in range(blocks)])
        gains[j] = g
        V[j] = (Q @ Psi).T
        U[j] = (Yj @ Psi / np.where(g > 0, g, 1.0)[None, :]).T
    return gains, V, U, hist
