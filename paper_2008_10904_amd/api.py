"""Python face of the resolvent library: a handle class over the C ABI.  PyTorch provides device memory and the
stream; the computation is entirely in libresolvent.so (no CPU fallback: without the library or a GPU the
calls raise)."""
import ctypes

import numpy as np

from . import _lib
from ._lib import Grid, OpDesc, Run, check

_METHODS = {"transient": _lib.RES_TRANSIENT, "periodic": _lib.RES_PERIODIC}
_PREC = {"fp64": _lib.RES_FP64, "mixed": _lib.RES_MIXED}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the resolvent library needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


class ResolventOp:
    """A linear operator L with its RK4 step h, uploaded to the GPU.

    precision: "fp64" (complex128 I/O, FP64 everywhere) or "mixed" (complex64 I/O, FP32 stepping and phase
    GEMMs with FP64 accumulation, FP64 QR and gains)."""

    def __init__(self, desc, keep, precision, stream=None):
        self._lib = _lib.load()
        torch = _torch()
        self.precision = precision
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        self._keep = keep
        self._stream = stream
        h = ctypes.c_void_p()
        check(self._lib.resolvent_op_create(ctypes.byref(desc), self._stream_ptr(), ctypes.byref(h)))
        self._h = h
        self.n = int(self._lib.resolvent_op_size(h))
        self.h = desc.h
        self.ninst = int(desc.ninst)
        self.offsets = np.array(keep.get("offsets", [0, self.n]), dtype=np.int64)

    # ---- construction helpers ---------------------------------------------------------------------------
    @classmethod
    def tridiagonal(cls, lower, diag, upper, h, precision="fp64", offsets=None, probe=False, probe_tol=1e-9,
                    probe_tmax=2000.0, probe_seed=12345, stream=None):
        lower = np.ascontiguousarray(np.asarray(lower, np.complex128)).view(np.float64)
        diag = np.ascontiguousarray(np.asarray(diag, np.complex128)).view(np.float64)
        upper = np.ascontiguousarray(np.asarray(upper, np.complex128)).view(np.float64)
        n = diag.size // 2
        keep = dict(lower=lower, diag=diag, upper=upper)
        d = OpDesc()
        d.kind = _lib.RES_OP_TRIDIAG
        d.precision = _PREC[precision]
        d.h = float(h)
        if offsets is not None:
            off = np.ascontiguousarray(np.asarray(offsets, np.int64))
            keep["offsets"] = off
            d.ninst = len(off) - 1
            d.inst_offsets = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        else:
            d.ninst = 1
            d.nx = n
        d.lower, d.diag, d.upper = _dptr(lower), _dptr(diag), _dptr(upper)
        d.probe = 1 if probe else 0
        d.probe_tol = probe_tol
        d.probe_tmax = probe_tmax
        d.probe_seed = probe_seed
        return cls(d, keep, precision, stream)

    @classmethod
    def grid_operator(cls, kind, nx, ny, nz, coef, h, precision="fp64", probe=False, probe_tol=1e-9,
                      probe_tmax=2000.0, probe_seed=12345, stream=None):
        """2-D five-point (kind "adr2d") or 3-D three-component (kind "adr3d3c") operator from the coefficient
        dict of ``operators.adr2d_coefficients`` / ``operators.adr3d3c_coefficients``."""
        three = kind == "adr3d3c"
        keep = {}
        d = OpDesc()
        d.kind = _lib.RES_OP_ADR3D3C if three else _lib.RES_OP_ADR2D
        d.precision = _PREC[precision]
        d.h = float(h)
        d.ninst = 1
        d.nx, d.ny, d.nz = int(nx), int(ny), int(nz if three else 1)
        for name in ("cxm", "cxp", "cym", "cyp", "czm", "czp", "dfield", "coupling"):
            if name in coef and (three or name not in ("czm", "czp", "coupling")):
                a = np.ascontiguousarray(np.asarray(coef[name], np.float64)).ravel()
                keep[name] = a
                setattr(d, name, _dptr(a))
        d.probe = 1 if probe else 0
        d.probe_tol = probe_tol
        d.probe_tmax = probe_tmax
        d.probe_seed = probe_seed
        op = cls(d, keep, precision, stream)
        op.grid_shape = (int(nz if three else 1), int(ny), int(nx))
        op.ncomp = 3 if three else 1
        return op

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.resolvent_op_destroy(h)
            self._h = None

    def _stream_ptr(self):
        torch = _torch()
        s = self._stream if self._stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    @property
    def decay_time(self):
        return float(self._lib.resolvent_op_decay_time(self._h))

    # ---- arguments ----------------------------------------------------------------------------------------
    @staticmethod
    def grid(omega0, domega, n_omega):
        return Grid(float(omega0), float(domega), int(n_omega))

    @staticmethod
    def run(method, tail=0, periods=1, stride=1):
        return Run(_METHODS[method], int(tail), int(periods), int(stride))

    def _check_io(self, x, nw, k):
        torch = _torch()
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == self.cdtype and x.is_contiguous()):
            raise TypeError("expected a contiguous %s CUDA tensor" % self.cdtype)
        if tuple(x.shape) != (nw, k, self.n):
            raise ValueError("expected shape (n_omega, k, N) = %s, got %s" % ((nw, k, self.n), tuple(x.shape)))

    # ---- calls ------------------------------------------------------------------------------------------------
    def apply(self, f_hat, grid, run, out=None):
        """u_hat[j] = R_d(w_j) f_hat[j] for all frequencies in one direct run."""
        return self._apply(f_hat, grid, run, out, adjoint=False)

    def apply_noalloc(self, f_hat, grid, run, out):
        """apply(f_hat, grid, run) through resolvent_apply_noalloc: the library allocates nothing and takes its
        workspace from its fixed per-GPU scratch array; `out` (like f_hat) must be given.  Calls that overlap on one
        GPU race on that array."""
        nw, k = grid.n_omega, f_hat.shape[1]
        self._check_io(f_hat, nw, k)
        self._check_io(out, nw, k)
        check(self._lib.resolvent_apply_noalloc(self._h, ctypes.byref(grid), ctypes.byref(run), k,
                                                ctypes.c_void_p(f_hat.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                                self._stream_ptr()))
        return out

    def workspace_size(self, grid, run, k):
        """Smallest device workspace (bytes) apply_noalloc needs for this grid, run and column count (host
        computation; compare with _lib.NOALLOC_SCRATCH_BYTES)."""
        n = ctypes.c_size_t(0)
        check(self._lib.resolvent_workspace_size(self._h, ctypes.byref(grid), ctypes.byref(run), int(k),
                                                 ctypes.byref(n)))
        return int(n.value)

    def adjoint_apply(self, g_hat, grid, run, out=None):
        """z_hat[j] = R_d(w_j)^H g_hat[j] in one adjoint run."""
        return self._apply(g_hat, grid, run, out, adjoint=True)

    def _apply(self, x, grid, run, out, adjoint):
        torch = _torch()
        nw, k = grid.n_omega, x.shape[1]
        self._check_io(x, nw, k)
        if out is None:
            out = torch.empty_like(x)
        self._check_io(out, nw, k)
        fn = self._lib.resolvent_adjoint_apply if adjoint else self._lib.resolvent_apply
        check(fn(self._h, ctypes.byref(grid), ctypes.byref(run), k, ctypes.c_void_p(x.data_ptr()),
                 ctypes.c_void_p(out.data_ptr()), self._stream_ptr()))
        return out

    def modes(self, f0_hat, grid, run, iters, want_modes=True, want_hist=True):
        """Block power iteration; returns (gains [ninst, nw, k], V, U, hist [iters, ninst, nw, k, 2])."""
        torch = _torch()
        nw, k = grid.n_omega, f0_hat.shape[1]
        self._check_io(f0_hat, nw, k)
        gains = np.zeros((self.ninst, nw, k))
        hist = np.zeros((iters, self.ninst, nw, k, 2)) if want_hist else None
        V = torch.empty_like(f0_hat) if want_modes else None
        U = torch.empty_like(f0_hat) if want_modes else None
        check(self._lib.resolvent_modes(
            self._h, ctypes.byref(grid), ctypes.byref(run), k, int(iters), ctypes.c_void_p(f0_hat.data_ptr()),
            _dptr(gains), ctypes.c_void_p(V.data_ptr()) if V is not None else None,
            ctypes.c_void_p(U.data_ptr()) if U is not None else None, _dptr(hist), self._stream_ptr()))
        return gains, V, U, hist

    def krylov(self, f0_hat, grid, run, blocks, want_modes=True, want_hist=True):
        """Block Arnoldi estimates from `blocks` blocks of k forcings (k = f0_hat.shape[1]); returns (gains
        [ninst, nw, k], V, U, hist [blocks, ninst, nw, k]) like modes."""
        torch = _torch()
        nw, k = grid.n_omega, f0_hat.shape[1]
        self._check_io(f0_hat, nw, k)
        gains = np.zeros((self.ninst, nw, k))
        hist = np.zeros((blocks, self.ninst, nw, k)) if want_hist else None
        V = torch.empty_like(f0_hat) if want_modes else None
        U = torch.empty_like(f0_hat) if want_modes else None
        check(self._lib.resolvent_krylov(
            self._h, ctypes.byref(grid), ctypes.byref(run), k, int(blocks), ctypes.c_void_p(f0_hat.data_ptr()),
            _dptr(gains), ctypes.c_void_p(V.data_ptr()) if V is not None else None,
            ctypes.c_void_p(U.data_ptr()) if U is not None else None, _dptr(hist), self._stream_ptr()))
        return gains, V, U, hist

    def krylov_polished(self, op_fp64, f0_hat, grid, run, blocks):
        """Mixed-precision block Arnoldi with an FP64 Rayleigh-Ritz finish on its k leading Ritz vectors (one FP64
        direct and adjoint run on op_fp64, as modes_polished).  Returns (gains, V, U) with V, U complex128."""
        torch = _torch()
        if self.precision != "mixed" or op_fp64.precision != "fp64" or op_fp64.n != self.n:
            raise ValueError("krylov_polished needs this handle in mixed precision and op_fp64 in fp64, same size")
        if getattr(self, "weights", None) is not None:
            op_fp64.set_weights(*self.weights)
        _, V, _, _ = self.krylov(f0_hat, grid, run, blocks, want_modes=True, want_hist=False)
        gains, V2, U2, _ = op_fp64.modes(V.to(torch.complex128).contiguous(), grid, run, 1, want_hist=False)
        return gains, V2, U2

    def modes_polished(self, op_fp64, f0_hat, grid, run, iters, want_hist=True):
        """Mixed-precision block power iteration with an FP64 Rayleigh-Ritz finish.

        The iterations run on this (mixed-precision) handle; then one FP64 run on op_fp64 (the same operator built
        with precision "fp64") takes the Rayleigh-Ritz values on the final force-mode subspace.  Those gains are
        stationary at the modes, so their error is second order in the mixed-precision subspace error, while every
        iteration keeps the mixed-precision speed (the finish costs one FP64 iteration).  Returns (gains, V, U,
        hist) as modes, with V, U complex128 from the FP64 finish and hist the mixed iterations' history whose last
        row carries the finished gains."""
        torch = _torch()
        if self.precision != "mixed" or op_fp64.precision != "fp64" or op_fp64.n != self.n:
            raise ValueError("modes_polished needs this handle in mixed precision and op_fp64 in fp64, same size")
        if getattr(self, "weights", None) is not None:
            op_fp64.set_weights(*self.weights)
        _, V, _, hist = self.modes(f0_hat, grid, run, iters, want_modes=True, want_hist=want_hist)
        gains, V2, U2, _ = op_fp64.modes(V.to(torch.complex128).contiguous(), grid, run, 1, want_hist=False)
        if want_hist:
            hist[-1, ..., 0] = gains
        return gains, V2, U2, hist

    def diag_size(self):
        """Length of the diagonal that set_diagonal and the reverse mode address: N for a tridiagonal operator,
        nz*ny*nx (one value per node, shared by the components) for a grid operator."""
        if hasattr(self, "grid_shape"):
            nz, ny, nx = self.grid_shape
            return nz * ny * nx
        return self.n

    def apply_backward(self, f_hat, g_hat, grid, run, checkpoint_every=0, want_f=True, want_mu=True):
        """Reverse mode of apply(f_hat, grid, run): given g_hat = dJ/du_hat of a real objective J (convention
        dJ/dRe + i dJ/dIm), returns (f_grad like f_hat or None, mu_grad float64 [diag_size()] or None) with
        mu_grad = dJ/d(real part of L's diagonal).  The forward trajectory is recomputed from checkpoints taken
        every `checkpoint_every` steps (0: about sqrt of the run length)."""
        torch = _torch()
        nw, k = grid.n_omega, f_hat.shape[1]
        self._check_io(f_hat, nw, k)
        self._check_io(g_hat, nw, k)
        f_grad = torch.empty_like(f_hat) if want_f else None
        mu_grad = torch.empty(self.diag_size(), dtype=torch.float64, device=f_hat.device) if want_mu else None
        mu_ptr = ctypes.cast(ctypes.c_void_p(mu_grad.data_ptr()), ctypes.POINTER(ctypes.c_double)) if want_mu else None
        check(self._lib.resolvent_apply_backward(
            self._h, ctypes.byref(grid), ctypes.byref(run), k, ctypes.c_void_p(f_hat.data_ptr()),
            ctypes.c_void_p(g_hat.data_ptr()), ctypes.c_void_p(f_grad.data_ptr()) if want_f else None, mu_ptr,
            int(checkpoint_every), self._stream_ptr()))
        return f_grad, mu_grad

    def set_diagonal(self, diag):
        """Replace the operator's diagonal (host array): complex [N] for a tridiagonal operator, real
        [nz*ny*nx] (the dfield) for a grid operator."""
        if hasattr(self, "grid_shape"):
            d = np.ascontiguousarray(np.asarray(diag, np.float64)).ravel()
        else:
            d = np.ascontiguousarray(np.asarray(diag, np.complex128)).view(np.float64)
        check(self._lib.resolvent_op_set_diagonal(self._h, _dptr(d), 0, self._stream_ptr()))

    def set_graphs(self, enable=True):
        """resolvent_modes replays its middle iterations from one captured HIP graph."""
        check(self._lib.resolvent_op_set_graphs(self._h, 1 if enable else 0))

    def set_backward_rows(self, fp64=True):
        """Row precision of apply_backward for a mixed-precision operator: FP64 rows (fp64=True) or FP32 rows (the
        default); the arithmetic and the gradient accumulation are FP64 either way."""
        check(self._lib.resolvent_op_set_backward_rows(self._h, 1 if fp64 else 0))

    # ---- stepper plan and autotuner (1-D operators) ------------------------------------------------------------
    def get_plan(self):
        """(configuration, owned unknowns per workgroup, steps between exchanges, persistent) in effect."""
        p = (ctypes.c_int32 * 4)()
        check(self._lib.resolvent_op_get_plan(self._h, p))
        return tuple(int(x) for x in p)

    def set_plan(self, plan):
        p = (ctypes.c_int32 * 4)(*[int(x) for x in plan])
        check(self._lib.resolvent_op_set_plan(self._h, p))
        return self.get_plan()

    def set_weights(self, b=None, c=None, wf=None, wy=None):
        """Diagonal B, C and metrics W_f, W_y (real arrays of the N unknowns, None = identity): apply returns
        C R B f, adjoint_apply W_f^-1 B^H R^H C^H W_y y, and modes / krylov maximise ||C R B f||_Wy / ||f||_Wf."""
        arrs = []
        for a in (b, c, wf, wy):
            arrs.append(None if a is None else np.ascontiguousarray(np.asarray(a, np.float64).ravel()))
        for a in arrs:
            if a is not None and a.shape != (self.n,):
                raise ValueError("weights must have the operator's %d unknowns" % self.n)
        check(self._lib.resolvent_op_set_weights(self._h, *[_dptr(a) for a in arrs]))
        self.weights = None if all(a is None for a in arrs) else tuple(arrs)

    def set_step_power(self, m):
        """RK4 steps per kernel step of the 1-D march (1, 2 or 4): the band P(Z)^m and the combined forcing of m
        steps; runs whose period, projection samples and exchange interval are multiples of m use it."""
        check(self._lib.resolvent_op_set_step_power(self._h, int(m)))

    def get_step_power(self):
        m = ctypes.c_int32()
        check(self._lib.resolvent_op_get_step_power(self._h, ctypes.byref(m)))
        return int(m.value)

    def tune(self, k, steps=2048):
        """Time every candidate stepper plan for k columns and keep the fastest; returns (plan, us per step)."""
        p = (ctypes.c_int32 * 4)()
        us = ctypes.c_double()
        check(self._lib.resolvent_op_tune(self._h, int(k), int(steps), p, ctypes.byref(us), self._stream_ptr()))
        return tuple(int(x) for x in p), us.value

    def set_timing(self, enable=True):
        check(self._lib.resolvent_op_set_timing(self._h, 1 if enable else 0))

    def timing(self, kind):
        """(total device ms, launches) of a kernel class since the last query (synchronises the stream)."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(self._lib.resolvent_op_get_timing(self._h, int(kind), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def check(self):
        check(self._lib.resolvent_op_check(self._h, self._stream_ptr()))

    # ---- transient-response method with time-domain hand-off ----------------------------------------------------
    _SCHEMES = {"C0": 0, "C1": 1, "C2": 2}

    def _check_series(self, x):
        torch = _torch()
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == self.cdtype and x.is_contiguous()):
            raise TypeError("expected a contiguous %s CUDA tensor" % self.cdtype)
        if x.dim() != 3 or x.shape[2] != self.n:
            raise ValueError("expected shape (n_samples, k, N) with N = %d, got %s" % (self.n, tuple(x.shape)))

    def signal_run(self, f, every, scheme="C2", adjoint=False, out=None):
        """State samples [n, k, N] of the run forced by the samples f [n, k, N] (sample i at t = i every h), from
        rest; adjoint=True runs -dz/dt = L^H z + f backward from z(T) = 0.  scheme: "C0", "C1" or "C2"."""
        torch = _torch()
        self._check_series(f)
        if out is None:
            out = torch.empty_like(f)
        check(self._lib.resolvent_signal_run(self._h, int(f.shape[1]), int(f.shape[0]), int(every),
                                             self._SCHEMES[scheme], 1 if adjoint else 0, ctypes.c_void_p(f.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), self._stream_ptr()))
        return out

    def trm_modes(self, f0, omegas, iters, every, scheme="C2", order=600, passes=2, pad=0, ramp=0, margin=0.0,
                  want_forcing=False, want_modes=False):
        """Power iteration with time-domain hand-off and FIR flattening (resolvent_trm_modes).  Returns (gains
        [iters, n_omega], amplitudes [iters, n_omega], last forcing [n, k, N] or None), and with want_modes also
        the force and response modes of the last iteration, V and U [n_omega, k, N]."""
        torch = _torch()
        self._check_series(f0)
        om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
        gains = np.zeros((int(iters), len(om)))
        amps = np.zeros((int(iters), len(om)))
        fo = torch.empty_like(f0) if want_forcing else None
        V = torch.empty((len(om), f0.shape[1], self.n), dtype=self.cdtype, device=f0.device) if want_modes else None
        U = torch.empty_like(V) if want_modes else None
        check(self._lib.resolvent_trm_modes(
            self._h, int(f0.shape[1]), int(f0.shape[0]), int(every), self._SCHEMES[scheme],
            ctypes.c_void_p(f0.data_ptr()), len(om), _dptr(om), int(iters), int(order), int(passes), int(pad),
            int(ramp), float(margin), _dptr(gains), _dptr(amps),
            ctypes.c_void_p(fo.data_ptr()) if fo is not None else None,
            ctypes.c_void_p(V.data_ptr()) if V is not None else None,
            ctypes.c_void_p(U.data_ptr()) if U is not None else None, self._stream_ptr()))
        if want_modes:
            return gains, amps, fo, V, U
        return gains, amps, fo


def grid_from_omegas(omegas, h, stride=1):
    """(Grid, P) for an array of uniformly spaced analysis frequencies: the spacing snapped to 2 pi / (P h) with P
    the multiple of `stride` nearest 2 pi / (|domega| h); host computation in the library."""
    lib = _lib.load()
    w = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64).ravel())
    g = Grid()
    P = ctypes.c_int64(0)
    check(lib.resolvent_grid_from_omegas(_dptr(w), len(w), float(h), int(stride), ctypes.byref(g), ctypes.byref(P)))
    return g, int(P.value)


def fir_design(order, nu, gain):
    """Taps (complex128, order + 1) of the linear-phase FIR filter for the amplitudes `gain` at breakpoints `nu`
    (frequency over Nyquist, non-decreasing in [-1, 1]); host computation in the library."""
    lib = _lib.load()
    nu = np.ascontiguousarray(np.asarray(nu, dtype=np.float64))
    gain = np.ascontiguousarray(np.asarray(gain, dtype=np.float64))
    if nu.shape != gain.shape:
        raise ValueError("nu and gain must have the same length")
    taps = np.zeros(int(order) + 1, dtype=np.complex128)
    out = taps.view(np.float64)
    check(lib.resolvent_fir_design(int(order), len(nu), _dptr(nu), _dptr(gain), _dptr(out)))
    return taps


def fir_apply(taps, x, out=None):
    """Delay-compensated FIR filtering along the first axis of the CUDA tensor x [n_t, ...] (complex128 or
    complex64) with complex taps (order + 1, even order)."""
    torch = _torch()
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.is_contiguous()
            and x.dtype in (torch.complex128, torch.complex64)):
        raise TypeError("expected a contiguous complex CUDA tensor")
    t = torch.as_tensor(np.asarray(taps, dtype=np.complex128)).to(x.device).contiguous()
    if out is None:
        out = torch.empty_like(x)
    ncols = int(x.numel() // x.shape[0])
    check(_lib.load().resolvent_fir_apply(1 if x.dtype == torch.complex128 else 0, int(x.shape[0]), ncols,
                                          int(t.numel()) - 1, ctypes.c_void_p(t.data_ptr()),
                                          ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out
