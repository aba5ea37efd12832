"""Stencil coefficients of the model operators, handed to the library through the C ABI.

These are the library's own builders (host NumPy, set-up only); they produce the coefficient arrays of
``resolvent_op_desc`` from the physical parameters:

* linearised Ginzburg-Landau  L = -nu d/dx + gamma d2/dx2 + mu(x),  mu(x) = (mu0 - c_mu^2) + mu2 x^2 / 2,
  second-order central differences on N interior nodes of [xl, xr] with u = 0 at both ends;
* the same for a batch of independent instances placed back to back;
* the paper's own real Ginzburg-Landau model of Sec. 3 (U = 6, gamma = 1, mu(x) = beta mu_c (1 - x/20) on (0, 40)).
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


def paper_gl_coefficients(n, beta=0.1, U=6.0, gamma=1.0, length=40.0):
    """Three-point coefficients of the Sec. 3 model L = -U d/dx + gamma d2/dx2 + mu(x), u(0) = u(length) = 0, with
    mu(x) = beta mu_c (1 - x/20) and mu_c = U^2 Re(gamma)/|gamma|^2 (real coefficients, stored as complex)."""
    x, _ = gl_nodes(n, 0.0, length)
    mu_c = U * U * np.real(gamma) / abs(gamma) ** 2
    return gl_coefficients(n, nu=U, gamma=gamma, xl=0.0, xr=length, mu=beta * mu_c * (1.0 - x / 20.0))


def snap_grid(wmin, wmax, n_omega, h, stride=1):
    """Uniform grid of n_omega frequencies starting at wmin whose spacing is 2 pi / (P h) with P a multiple of
    ``stride`` closest to the nominal spacing (wmax - wmin)/(n_omega - 1).  Returns (omega0, domega, P)."""
    dw_nom = (wmax - wmin) / (n_omega - 1)
    P = stride * int(round(2.0 * np.pi / (dw_nom * h * stride)))
    return float(wmin), 2.0 * np.pi / (P * h), P


# ------------------------------------------------------------------------------------------------------------
# 2-D advection-diffusion-reaction and 3-D three-component advection-diffusion with shear coupling
# ------------------------------------------------------------------------------------------------------------
def _ramp(s, lo, hi, frac=0.1):
    """Sponge ramp: 0 away from the ends of [lo, hi], rising linearly to 1 over the last `frac` of each end."""
    w = frac * (hi - lo)
    return np.clip((w - np.minimum(s - lo, hi - s)) / w, 0.0, 1.0)


def adr2d_coefficients(nx, ny, Re=200.0, mu=None, mu_base=-0.1, mu_amp=0.08, mu_xc=10.0, mu_w2=4.0, nu_s=1.0,
                       Lx=40.0, ylo=-10.0, yhi=10.0):
    """Five-point coefficients of  L q = -U(y) q_x + (q_xx + q_yy)/Re + (mu(x,y) - sponge(x,y)) q,  U = tanh(y),
    on nx * ny interior nodes of [0, Lx] x [ylo, yhi] with q = 0 on the boundary (x fastest).

    mu: array (ny, nx) or None for mu_base + mu_amp exp(-((x - mu_xc)^2 + y^2)/mu_w2).  The sponge is
    nu_s * max(rx, ry)^2 with rx, ry the linear ramps over the outer tenth of each direction.
    Returns dict(cxm, cxp, cym, cyp [ny], dfield [ny*nx], mu [ny, nx])."""
    dx = Lx / (nx + 1)
    dy = (yhi - ylo) / (ny + 1)
    x = dx * (1.0 + np.arange(nx))
    y = ylo + dy * (1.0 + np.arange(ny))
    X, Y = np.meshgrid(x, y, indexing="xy")
    if mu is None:
        mu = mu_base + mu_amp * np.exp(-((X - mu_xc) ** 2 + Y ** 2) / mu_w2)
    sponge = nu_s * np.maximum(_ramp(X, 0.0, Lx), _ramp(Y, ylo, yhi)) ** 2
    U = np.tanh(y)
    dif_x, dif_y = 1.0 / (Re * dx * dx), 1.0 / (Re * dy * dy)
    return dict(cxm=U / (2 * dx) + dif_x, cxp=-U / (2 * dx) + dif_x, cym=np.full(ny, dif_y), cyp=np.full(ny, dif_y),
                dfield=(-2 * dif_x - 2 * dif_y + np.asarray(mu) - sponge).ravel(), mu=np.asarray(mu), sponge=sponge)


def wake_profile(y, z, amp, delta, y0, z0):
    """U = 1 - amp exp(-((y - y0)^2 + (z - z0)^2)/delta^2) with its analytic derivatives (U, dU/dy, dU/dz)."""
    g = np.exp(-((y - y0) ** 2 + (z - z0) ** 2) / delta ** 2)
    return 1.0 - amp * g, 2.0 * amp * g * (y - y0) / delta ** 2, 2.0 * amp * g * (z - z0) / delta ** 2


def adr3d3c_coefficients(nx, ny, nz, wake, Re=200.0, mu=None, mu_const=-0.05, nu_s=1.0, Lx=40.0, lo=-10.0,
                         hi=10.0):
    """Seven-point coefficients of the three-component operator on (nz, ny, nx) interior nodes, q = 0 on the
    boundary:  du/dt = -U u_x - U_y v - U_z w + lap(u)/Re + (mu - s) u,  dv/dt = -U v_x + lap(v)/Re + (mu - s) v,
    dw/dt = -U w_x + lap(w)/Re + (mu - s) w,  with U(y, z) the wake profile of ``wake``.
    Returns dict(cxm, cxp, cym, cyp, czm, czp [nz*ny], dfield [nz*ny*nx], coupling [nz*ny, 3, 3], mu)."""
    dx = Lx / (nx + 1)
    dy = (hi - lo) / (ny + 1)
    dz = (hi - lo) / (nz + 1)
    x = dx * (1.0 + np.arange(nx))
    y = lo + dy * (1.0 + np.arange(ny))
    z = lo + dz * (1.0 + np.arange(nz))
    Zl, Yl = np.meshgrid(z, y, indexing="ij")  # line index l = iz * ny + iy
    U, Uy, Uz = wake_profile(Yl, Zl, **wake)
    Z3, Y3, X3 = np.meshgrid(z, y, x, indexing="ij")
    if mu is None:
        mu = np.full((nz, ny, nx), mu_const)
    sponge = nu_s * np.maximum(np.maximum(_ramp(X3, 0.0, Lx), _ramp(Y3, lo, hi)), _ramp(Z3, lo, hi)) ** 2
    ax, ay, az = 1.0 / (Re * dx * dx), 1.0 / (Re * dy * dy), 1.0 / (Re * dz * dz)
    nl = ny * nz
    K = np.zeros((nl, 3, 3))
    K[:, 0, 1] = -Uy.ravel()
    K[:, 0, 2] = -Uz.ravel()
    return dict(cxm=(U / (2 * dx) + ax).ravel(), cxp=(-U / (2 * dx) + ax).ravel(), cym=np.full(nl, ay),
                cyp=np.full(nl, ay), czm=np.full(nl, az), czp=np.full(nl, az),
                dfield=(-2 * (ax + ay + az) + np.asarray(mu) - sponge).ravel(), coupling=K, mu=np.asarray(mu))
