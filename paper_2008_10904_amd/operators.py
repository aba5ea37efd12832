"""Stencil coefficients of the model operators, handed to the library through the C ABI.

These are the library's own builders (host NumPy, set-up only); they produce the coefficient arrays of
``resolvent_op_desc`` from the physical parameters:

* linearised Ginzburg-Landau  L = -nu d/dx + gamma d2/dx2 + mu(x),  mu(x) = (mu0 - c_mu^2) + mu2 x^2 / 2,
  second-order central differences on N interior nodes of [xl, xr] with u = 0 at both ends;
* the same for a batch of independent instances placed back to back.
"""
import numpy as np

GL_NU = 2.0 + 0.4j
GL_GAMMA = 1.0 - 1.0j
GL_CMU2 = 0.04


def gl_nodes(n, xl=-50.0, xr=50.0):
    dx = (xr - xl) / (n + 1)
    return xl + dx * (1.0 + np.arange(n)), dx


def gl_reaction(x, mu0, mu2, cmu2=GL_CMU2):
    return (mu0 - cmu2) + 0.5 * mu2 * x ** 2


def gl_coefficients(n, mu0=None, mu2=None, nu=GL_NU, gamma=GL_GAMMA, xl=-50.0, xr=50.0, mu=None):
    """(lower, diag, upper) complex arrays of the three-point GL operator: (L u)_i = lo_i u_{i-1} + d_i u_i + up_i u_{i+1}."""
    x, dx = gl_nodes(n, xl, xr)
    if mu is None:
        mu = gl_reaction(x, mu0, mu2)
    adv = nu / (2.0 * dx)       # -nu (u_{i+1} - u_{i-1}) / (2 dx)
    dif = gamma / (dx * dx)     # gamma (u_{i+1} - 2 u_i + u_{i-1}) / dx^2
    lower = np.full(n, adv + dif, dtype=np.complex128)
    upper = np.full(n, -adv + dif, dtype=np.complex128)
    diag = -2.0 * dif + np.asarray(mu, dtype=np.complex128)
    lower[0] = 0.0
    upper[-1] = 0.0
    return lower, diag, upper


def gl_batched_coefficients(instances, nu=GL_NU, gamma=GL_GAMMA, xl=-50.0, xr=50.0):
    """Concatenated coefficients and offsets [ninst+1] of independent instances [(n, mu0, mu2), ...]."""
    parts = [gl_coefficients(n, mu0, mu2, nu, gamma, xl, xr) for (n, mu0, mu2) in instances]
    lower = np.concatenate([p[0] for p in parts])
    diag = np.concatenate([p[1] for p in parts])
    upper = np.concatenate([p[2] for p in parts])
    offsets = np.zeros(len(instances) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([n for (n, _, _) in instances])
    return lower, diag, upper, offsets


def snap_grid(wmin, wmax, n_omega, h, stride=1):
    """Uniform grid of n_omega frequencies starting at wmin whose spacing is 2 pi / (P h) with P a multiple of
    ``stride`` closest to the nominal spacing (wmax - wmin)/(n_omega - 1).  Returns (omega0, domega, P)."""
    dw_nom = (wmax - wmin) / (n_omega - 1)
    P = stride * int(round(2.0 * np.pi / (dw_nom * h * stride)))
    return float(wmin), 2.0 * np.pi / (P * h), P
