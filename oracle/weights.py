"""Input and output matrices B, C and the force / observation metrics W_f, W_y of the resolvent problem (Sec. 2.1),
for diagonal B, C, W (masks, weights and non-uniform-grid quadrature); test infrastructure only.

The observed response is y = C R B f.  With <a, b>_f = a^H W_f b on forces and <a, b>_y = a^H W_y b on
observations, the gains are sigma = max ||C R B f||_y / ||f||_f and the adjoint of R_y = C R B in these metrics is
R_y^dagger = W_f^{-1} B^H R^H C^H W_y (the W_u of the state space cancels: the paper's A^dagger = W_u^{-1} A^H W_u
enters between B^dagger = W_f^{-1} B^H W_u and C^dagger = W_u^{-1} C^H W_y; the paper prints the last one as
W_y^{-1} C^H W_u, which maps the wrong way for an output matrix).  The gains and modes are the SVD of the Euclidean
operator R~ = W_y^{1/2} C R B W_f^{-1/2}: sigma(R~), force modes V = W_f^{-1/2} V~ (W_f-orthonormal), response
modes U = W_y^{-1/2} U~.

``apply`` / ``adjoint_apply`` act on (n_w, k, N) arrays (Euclidean R and R^H); b, c, wf, wy are real (N,) arrays.
"""
import numpy as np


def observed_applies(apply, adjoint_apply, b, c, wf, wy):
    """(y = C R B f, R_y^dagger y = W_f^{-1} B R^H C W_y y) for real diagonal B = diag(b), C = diag(c)."""
    def app(F):
        return c * apply(b * F)

    def adj(Y):
        return (b / wf) * adjoint_apply(c * wy * Y)

    return app, adj


def euclidean_applies(apply, adjoint_apply, b, c, wf, wy):
    """(R~ f, R~^H g) with R~ = W_y^{1/2} C R B W_f^{-1/2}: the operator whose Euclidean SVD gives the gains."""
    sin, sout = b / np.sqrt(wf), c * np.sqrt(wy)

    def app(F):
        return sout * apply(sin * F)

    def adj(G):
        return sin * adjoint_apply(sout * G)

    return app, adj


def modes_from_euclidean(V, U, wf, wy):
    """Force and response modes in the problem's metrics from the Euclidean modes of R~."""
    return V / np.sqrt(wf), U / np.sqrt(wy)
