"""Linear operators L of du/dt = L u + f, built from their PDE definitions (test infrastructure only).

The paper writes the system as du/dt + A u = B f (Sec. 2.1, eq. system); here L = -A and B = C = I,
the choice the paper also makes for its Ginzburg-Landau study (Sec. 3).  Each builder writes the
continuous operator out term by term with second-order central differences on a uniform grid of
interior nodes and homogeneous Dirichlet values just outside it.

* ``gl_operator``      -- linearised Ginzburg-Landau  L = -nu d/dx + gamma d2/dx2 + mu(x)
                          (complex nu, gamma; the model family of Sec. 3 in the form with complex
                          coefficients used by the 1-D workloads).
* ``paper_gl_operator`` -- the paper's own real Ginzburg-Landau model of Sec. 3 (U = 6, gamma = 1,
                          mu(x) = beta mu_c (1 - x/20) on (0, 40)).
* ``adr2d_operator``   -- 2-D advection-diffusion-reaction  L q = -U(y) q_x + Re^-1 lap q + (mu - s) q.
* ``adr3d3c_operator`` -- 3-D three-component advection-diffusion with shear coupling
                          L (u,v,w) = (-U u_x - v U_y - w U_z, -U v_x, -U w_x) + Re^-1 lap + (mu - s).

Index order: x fastest, then y, then z; components outermost (comp-major).
"""
import numpy as np
import scipy.sparse as sp


def uniform_interior_grid(n, lo, hi):
    """n interior nodes of [lo, hi] with the end points excluded (Dirichlet nodes)."""
    d = (hi - lo) / (n + 1)
    return lo + d * np.arange(1, n + 1), d


def _first_derivative(n, d):
    # (q[i+1] - q[i-1]) / (2 d), q = 0 outside
    return sp.diags([-np.ones(n - 1), np.ones(n - 1)], [-1, 1], shape=(n, n)) / (2.0 * d)


def _second_derivative(n, d):
    # (q[i+1] - 2 q[i] + q[i-1]) / d^2, q = 0 outside
    return sp.diags([np.ones(n - 1), -2.0 * np.ones(n), np.ones(n - 1)], [-1, 0, 1],
                    shape=(n, n)) / (d * d)


# ----------------------------------------------------------------------------------------------
# 1-D Ginzburg-Landau
# ----------------------------------------------------------------------------------------------
GL_NU = 2.0 + 0.4j
GL_GAMMA = 1.0 - 1.0j
GL_CMU2 = 0.04  # c_mu^2 of mu(x) = (mu0 - c_mu^2) + mu2 x^2 / 2


def gl_mu(x, mu0, mu2, cmu2=GL_CMU2):
    """Reaction profile mu(x) = (mu0 - c_mu^2) + mu2 * x^2 / 2."""
    return (mu0 - cmu2) + 0.5 * mu2 * x * x


def gl_operator(n, mu0=None, mu2=None, nu=GL_NU, gamma=GL_GAMMA, xl=-50.0, xr=50.0, mu=None):
    """L = -nu d/dx + gamma d2/dx2 + mu(x) on n interior nodes of [xl, xr], u(xl) = u(xr) = 0.

    Either (mu0, mu2) or an explicit array ``mu`` (length n, real or complex) gives the reaction term.
    Returns (L as CSR complex128, x).
    """
    x, dx = uniform_interior_grid(n, xl, xr)
    if mu is None:
        mu = gl_mu(x, mu0, mu2)
    D1 = _first_derivative(n, dx).astype(complex).tocsr()
    D2 = _second_derivative(n, dx).astype(complex).tocsr()
    L = -nu * D1 + gamma * D2 + sp.diags(np.asarray(mu, complex)).tocsr()
    return L.tocsr().astype(np.complex128), x


def paper_gl_operator(n, beta=0.1, U=6.0, gamma=1.0, length=40.0):
    """The Ginzburg-Landau model of Sec. 3 (eq. GL_timeDomain): A = U d/dx - mu(x) - gamma d2/dx2 on (0, length)
    with u = 0 at both ends, mu(x) = beta mu_c (1 - x/20) and mu_c = U^2 Re(gamma) / |gamma|^2.  All
    coefficients are real.  Returns (L = -A as CSR complex128, x)."""
    x, _ = uniform_interior_grid(n, 0.0, length)
    mu_c = U * U * np.real(gamma) / abs(gamma) ** 2
    return gl_operator(n, nu=U, gamma=gamma, xl=0.0, xr=length, mu=beta * mu_c * (1.0 - x / 20.0))


# ----------------------------------------------------------------------------------------------
# 2-D advection-diffusion-reaction with a sponge
# ----------------------------------------------------------------------------------------------
def sponge_ramp(s, lo, hi, frac=0.1):
    """0 in the interior, rising as ((w - dist)/w)^1 to 1 at the edges of [lo, hi]; w = frac*(hi-lo)."""
    w = frac * (hi - lo)
    dist = np.minimum(s - lo, hi - s)
    return np.clip((w - dist) / w, 0.0, 1.0)


def adr2d_fields(nx, ny, Lx=40.0, ylo=-10.0, yhi=10.0, nu_s=1.0, frac=0.1):
    """Grid, base flow U(y) = tanh(y), sponge s(x,y) = nu_s * max(rx, ry)^2."""
    x, dx = uniform_interior_grid(nx, 0.0, Lx)
    y, dy = uniform_interior_grid(ny, ylo, yhi)
    X, Y = np.meshgrid(x, y, indexing="xy")  # shape (ny, nx): x fastest
    rx = sponge_ramp(X, 0.0, Lx, frac)
    ry = sponge_ramp(Y, ylo, yhi, frac)
    sponge = nu_s * np.maximum(rx, ry) ** 2
    return dict(x=x, y=y, dx=dx, dy=dy, X=X, Y=Y, U=np.tanh(y), sponge=sponge)


def adr2d_mu_default(X, Y, base=-0.1, amp=0.08, xc=10.0, width2=4.0):
    """Default reaction field mu(x,y) = base + amp * exp(-((x-xc)^2 + y^2)/width2)."""
    return base + amp * np.exp(-((X - xc) ** 2 + Y ** 2) / width2)


def adr2d_operator(nx, ny, Re=200.0, mu=None, Lx=40.0, ylo=-10.0, yhi=10.0, nu_s=1.0):
    """L q = -U(y) dq/dx + (1/Re)(q_xx + q_yy) + (mu(x,y) - sponge(x,y)) q, Dirichlet on all edges.

    ``mu``: array (ny, nx) or None for the default field.  Returns (L CSR complex128, fields dict).
    """
    f = adr2d_fields(nx, ny, Lx, ylo, yhi, nu_s)
    if mu is None:
        mu = adr2d_mu_default(f["X"], f["Y"])
    Ix, Iy = sp.identity(nx), sp.identity(ny)
    Dx = sp.kron(Iy, _first_derivative(nx, f["dx"]))
    Dxx = sp.kron(Iy, _second_derivative(nx, f["dx"]))
    Dyy = sp.kron(_second_derivative(ny, f["dy"]), Ix)
    Uflat = np.repeat(f["U"], nx)  # U(y) on every node of row y
    L = (-sp.diags(Uflat) @ Dx + (Dxx + Dyy) / Re
         + sp.diags(np.asarray(mu).ravel() - f["sponge"].ravel()))
    f["mu"] = np.asarray(mu)
    return L.tocsr().astype(np.complex128), f


# ----------------------------------------------------------------------------------------------
# 3-D three-component advection-diffusion with shear coupling
# ----------------------------------------------------------------------------------------------
def wake_profile(Y, Z, amp, delta, y0, z0):
    """U(y,z) = 1 - amp * exp(-((y-y0)^2 + (z-z0)^2)/delta^2) and its analytic y, z derivatives."""
    g = np.exp(-((Y - y0) ** 2 + (Z - z0) ** 2) / delta ** 2)
    U = 1.0 - amp * g
    Uy = amp * g * 2.0 * (Y - y0) / delta ** 2
    Uz = amp * g * 2.0 * (Z - z0) / delta ** 2
    return U, Uy, Uz


def adr3d3c_fields(nx, ny, nz, wake, Lx=40.0, lo=-10.0, hi=10.0, nu_s=1.0, frac=0.1):
    x, dx = uniform_interior_grid(nx, 0.0, Lx)
    y, dy = uniform_interior_grid(ny, lo, hi)
    z, dz = uniform_interior_grid(nz, lo, hi)
    Zg, Yg, Xg = np.meshgrid(z, y, x, indexing="ij")  # shape (nz, ny, nx)
    U, Uy, Uz = wake_profile(Yg[:, :, 0], Zg[:, :, 0], **wake)  # (nz, ny): constant along x
    r = np.maximum(np.maximum(sponge_ramp(Xg, 0.0, Lx, frac), sponge_ramp(Yg, lo, hi, frac)),
                   sponge_ramp(Zg, lo, hi, frac))
    return dict(x=x, y=y, z=z, dx=dx, dy=dy, dz=dz, X=Xg, Y=Yg, Z=Zg, U=U, Uy=Uy, Uz=Uz,
                sponge=nu_s * r ** 2)


def adr3d3c_operator(nx, ny, nz, wake, Re=200.0, mu=None, Lx=40.0, lo=-10.0, hi=10.0, nu_s=1.0):
    """Three velocity-like components q = (u, v, w) on an (nz, ny, nx) grid, Dirichlet on all faces:

        du/dt = -U du/dx - v dU/dy - w dU/dz + (1/Re) lap u + (mu - s) u
        dv/dt = -U dv/dx                     + (1/Re) lap v + (mu - s) v
        dw/dt = -U dw/dx                     + (1/Re) lap w + (mu - s) w

    ``mu``: array (nz, ny, nx) or None (constant -0.05).  Returns (L CSR complex128, fields dict).
    """
    f = adr3d3c_fields(nx, ny, nz, wake, Lx, lo, hi, nu_s)
    if mu is None:
        mu = np.full((nz, ny, nx), -0.05)
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    Dx = sp.kron(Iz, sp.kron(Iy, _first_derivative(nx, f["dx"])))
    Dxx = sp.kron(Iz, sp.kron(Iy, _second_derivative(nx, f["dx"])))
    Dyy = sp.kron(Iz, sp.kron(_second_derivative(ny, f["dy"]), Ix))
    Dzz = sp.kron(_second_derivative(nz, f["dz"]), sp.kron(Iy, Ix))
    Ufl = np.repeat(f["U"].ravel(), nx)
    S = (-sp.diags(Ufl) @ Dx + (Dxx + Dyy + Dzz) / Re
         + sp.diags(np.asarray(mu).ravel() - f["sponge"].ravel()))
    Cy = sp.diags(-np.repeat(f["Uy"].ravel(), nx))
    Cz = sp.diags(-np.repeat(f["Uz"].ravel(), nx))
    Zr = None
    L = sp.bmat([[S, Cy, Cz], [Zr, S, Zr], [Zr, Zr, S]])
    f["mu"] = np.asarray(mu)
    return L.tocsr().astype(np.complex128), f
