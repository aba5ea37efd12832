"""Seeded synthetic workloads for the resolvent hot path.

Holds only problem parameters and random draws -- none of the method's arithmetic.  Both the CPU oracle
(through the tests) and the HIP library (through the tests, ``bench.py`` and ``__graft_entry__``) take their
inputs from here, and each side builds its own operator and frequency grid from these numbers.

Workloads (the paper publishes no data set; every input is synthetic):

* ``GL_TRANSIENT``  1-D linearised Ginzburg-Landau, N = 200, complex128, transient method, 64 frequencies in
                    [-2, 2], k = 1, 20 iterations.  mu0 = 0.30 (the literal mu0 = 0.38 gives an unstable
                    operator at N = 200, kept as ``GL_TRANSIENT_UNSTABLE`` for the error path).
* ``GL_PERIODIC``   same operator family at N = 2000 (mu0 = 0.38), periodic method, 256 frequencies in [-3, 3],
                    k = 4, 10 periods per run, 30 iterations, dt = 0.001 (0.005 is beyond RK4's stability limit).
* ``GL_BATCHED``    64 GL instances with seeded (mu0, mu2, N), N in {256, 512, 1024, 2048}, 128 frequencies in
                    [-2, 2], k = 2, mixed precision; the accepted draws are stored in
                    ``tests/golden/gl_batched_instances.json`` (see the script beside it).
* ``ADR2D``         2-D advection-diffusion-reaction, 1024 x 512, complex64 state, U(y) = tanh(y), Re = 200,
                    128 frequencies in [0, 2], k = 2, transient method with a 300-time-unit tail.
* ``GL_PAPER``      the paper's own real Ginzburg-Landau model (Sec. 3): U = 6, gamma = 1, beta = 0.1 on (0, 40),
                    N = 200, 77 frequencies 0, 15/76, ..., 15 (the band of the paper's study), P = 3200 so that
                    h = 2 pi 76 / (15 * 3200) = 0.00995 (the paper's step is 0.01), periodic method with 2 periods
                    (the transient decays like exp(-4.8 t), 1e-66 after one period), k = 1.
* ``GL_PAPER_TRM``  the same model with the transient-response method and time-domain hand-off at the paper's
                    settings (Sec. 3, App. B): h = 0.01 sampled every step, 6001 samples (60 time units; forcing
                    tapered to zero on the first and last 12 with 6-unit ramps), FIR flattening filters of order 3000
                    (resolution about 0.2 rad per time unit) applied in two passes, 61 analysis frequencies in
                    [-15, 15], C2 interpolation, k = 1.
* ``ADR3D``         3-D three-component advection-diffusion with shear coupling, 256 x 128 x 128, FP32 state,
                    96 frequencies in [0, pi/2] (P = 3,800 steps of h = 0.1), k = 3, periodic method with three
                    periods, the last one projected every 38th step (100 samples for 96 frequencies), checkpoints
                    every 64 steps for the gradient.

``gl_weights`` gives diagonal B, C, W_f, W_y (forcing window, observation window, grid quadrature) on the GL grid.

Random forcings are complex with independent N(0,1) real and imaginary parts from NumPy's PCG64 with the
workload seed (seed = 20081090 + index).
"""
import json
import math
import os

import numpy as np

SEED_BASE = 20081090
_HERE = os.path.dirname(os.path.abspath(__file__))
BATCHED_INSTANCES_JSON = os.path.join(_HERE, "tests", "golden", "gl_batched_instances.json")

GL_NU = (2.0, 0.4)
GL_GAMMA = (1.0, -1.0)
GL_CMU2 = 0.04
GL_DOMAIN = (-50.0, 50.0)

GL_TRANSIENT = dict(name="gl_transient_n200", kind="gl", N=200, mu0=0.30, mu2=-0.01, h=0.01,
                    wmin=-2.0, wmax=2.0, n_omega=64, method="transient", tail=20000, stride=1,
                    periods=1, k=1, iters=20, precision="fp64", seed=SEED_BASE + 0)
GL_TRANSIENT_UNSTABLE = dict(GL_TRANSIENT, name="gl_transient_n200_literal", mu0=0.38)

GL_PERIODIC = dict(name="gl_periodic_n2000", kind="gl", N=2000, mu0=0.38, mu2=-0.01, h=0.001,
                   wmin=-3.0, wmax=3.0, n_omega=256, method="periodic", periods=10, stride=256,
                   tail=0, k=4, iters=30, precision="fp64", seed=SEED_BASE + 1)

GL_BATCHED = dict(name="gl_batched_64", kind="gl_batched", ninst=64, sizes=(256, 512, 1024, 2048),
                  mu0_range=(0.2, 0.5), mu2_range=(-0.02, -0.005), stability_margin=-0.01, h=0.001,
                  wmin=-2.0, wmax=2.0, n_omega=128, method="periodic", periods=10, stride=128, tail=0,
                  k=2, iters=20, precision="mixed", seed=SEED_BASE + 2)

ADR2D = dict(name="adr2d_1024x512", kind="adr2d", nx=1024, ny=512, Re=200.0, h=0.02,
             wmin=0.0, wmax=2.0, n_omega=128, method="transient", tail=15000, stride=1, periods=1,
             k=2, iters=10, precision="mixed", mu_base=-0.1, mu_amp=0.08, mu_xc=10.0, mu_w2=4.0,
             nu_s=1.0, seed=SEED_BASE + 3)

GL_PAPER = dict(name="gl_paper_n200", kind="gl_paper", N=200, U=6.0, gamma=1.0, beta=0.1, length=40.0,
                w0=0.0, dw=15.0 / 76, n_omega=77, P=3200, h=2 * math.pi * 76 / (15.0 * 3200), method="periodic",
                periods=2, stride=32, tail=0, k=1, iters=15, precision="fp64", seed=SEED_BASE + 5)

GL_PAPER_TRM = dict(name="gl_paper_trm_n200", kind="gl_paper", N=200, U=6.0, gamma=1.0, beta=0.1, length=40.0,
                    h=0.01, every=1, n_samples=6001, wmax=15.0, n_omega=61, order=3000, passes=2, pad=1200, ramp=600,
                    margin=3.0, scheme="C2", k=1, iters=8, precision="fp64", seed=SEED_BASE + 6)

ADR3D = dict(name="adr3d3c_256x128x128", kind="adr3d3c", nx=256, ny=128, nz=128, Re=200.0, h=0.1,
             wmin=0.0, wmax=math.pi / 2, n_omega=96, method="periodic", periods=3, stride=38, tail=0,
             k=3, iters=1, precision="mixed", mu_const=-0.05, nu_s=1.0, checkpoint_every=64,
             seed=SEED_BASE + 4)


def gl_weights(n, xl=GL_DOMAIN[0], xr=GL_DOMAIN[1]):
    """Diagonal input, output and metric weights on the n interior nodes of the GL grid (x_i = xl + (i + 1) dx,
    dx = (xr - xl) / (n + 1)): B a smooth window over the upstream 60 % of the domain (where forcing may act), C a
    smooth window over the downstream 60 % (where the response is observed), W_f = W_y = dx (the quadrature of the
    uniform grid).  The windows overlap: disjoint ones (forcing upstream of the observed region only) make C R B
    so nearly low-rank that the four leading gains span more than 1e7 at w = 0.  Returns (b, c, wf, wy) as float64
    arrays."""
    dx = (xr - xl) / (n + 1)
    x = xl + dx * np.arange(1, n + 1)
    t = (x - xl) / (xr - xl)

    def window(a, b, w):
        return 0.5 * (np.tanh((t - a) / w) - np.tanh((t - b) / w))

    b = window(0.0, 0.6, 0.05)
    c = window(0.4, 1.0, 0.05)
    w = np.full(n, dx)
    return b, c, w, w.copy()


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def random_forcing(seed, n_omega, k, n, dtype=np.complex128):
    """F[j, c, :] with independent N(0,1) real and imaginary parts, shape (n_omega, k, n)."""
    g = rng(seed)
    re = g.standard_normal((n_omega, k, n))
    im = g.standard_normal((n_omega, k, n))
    return (re + 1j * im).astype(dtype)


def random_forcing_device(seed, n_omega, k, n, dtype, device):
    """F[j, c, :] with independent N(0,1) real and imaginary parts drawn on the device by torch's Philox generator
    seeded with `seed`, one frequency at a time (for inputs too large to draw on the host, such as the 3-D
    workload's 96 x 3 x 12.6 M forcing).  dtype: torch.complex64 or torch.complex128."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    real = torch.float32 if dtype == torch.complex64 else torch.float64
    out = torch.empty((n_omega, k, n), dtype=dtype, device=device)
    for j in range(n_omega):
        re = torch.randn((k, n), generator=g, dtype=real, device=device)
        im = torch.randn((k, n), generator=g, dtype=real, device=device)
        out[j] = torch.complex(re, im)
    return out


def batched_draws(cfg, count):
    """Candidate (N, mu0, mu2) triples in draw order (stability screening happens in the golden script)."""
    g = rng(cfg["seed"])
    out = []
    for _ in range(count):
        mu0 = float(g.uniform(*cfg["mu0_range"]))
        mu2 = float(g.uniform(*cfg["mu2_range"]))
        n = int(cfg["sizes"][int(g.integers(0, len(cfg["sizes"])))])
        out.append((n, mu0, mu2))
    return out


def batched_instances():
    """The 64 accepted GL instances [(N, mu0, mu2), ...] of ``GL_BATCHED``."""
    with open(BATCHED_INSTANCES_JSON) as f:
        data = json.load(f)
    return [tuple(x) for x in data["instances"]]


def wake_parameters(seed):
    """Seeded smooth wake-profile parameters of ``ADR3D``: U = 1 - amp exp(-((y-y0)^2+(z-z0)^2)/delta^2)."""
    g = rng(seed)
    return dict(amp=float(g.uniform(0.4, 0.6)), delta=float(g.uniform(1.5, 2.5)),
                y0=float(g.uniform(-0.5, 0.5)), z0=float(g.uniform(-0.5, 0.5)))
