#!/usr/bin/env python3
"""Resolvent sweeps/s of the time-stepping resolvent method on one MI355X.

Workload: linearised Ginzburg-Landau, N = 2000 unknowns, k = 4 forcing columns per frequency, 256 frequencies in
[-3, 3], steady-state-response (periodic) method with 10 forcing periods per run (the last one projected every
256 steps), RK4 with h = 0.001 (P = 267,008 steps per period), complex128.  One benchmark step is one iteration
of the block power iteration: a direct run, an adjoint run, two per-frequency QR factorisations and the k x k
SVDs.  Sweeps/s = N * k * n_omega * (time steps of the direct and adjoint runs) / seconds.

The same step is also timed in the mixed form (FP32 stepping and phase GEMMs, FP64 accumulation/QR/gains), with
the largest relative gain difference to the FP64 GPU run reported beside it.  The CPU baseline is the FP64
oracle marching the same operator and forcing for a bounded number of steps (the oracle is slow; its rate is
scaled to the same unit).  Inputs are synthetic and seeded; no data set is involved.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK = 256 * 4 * 16 * 2 * 2.4e9  # CUs x SIMDs x FP64 lanes x (FMA = 2 flop) x clock = 78.6 TFLOP/s
STEP_FLOP_PER_UNKNOWN = 9 * 8 + 8  # nine complex multiply-adds of the step stencil + the forcing term


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="gl_periodic_n2000",
                    choices=["gl_periodic_n2000", "gl_batched_64", "adr2d_1024x512", "adr3d3c_256x128x128",
                             "gl_paper_n200"],
                    help="gl_periodic_n2000 (default, the headline line), gl_batched_64 (64 uneven GL instances, "
                         "mixed precision, reported beside its FP64 form), the 2-D and 3-D grid operators, or "
                         "gl_paper_n200 (the paper's own real GL model of Sec. 3, with its power vs Arnoldi study)")
    ap.add_argument("--plan", default=None,
                    help="1-D stepper plan: 'tuned' (autotuner, cached per problem; tuning is set-up, not timed), "
                         "'default' (the library's default plan) or 'cfg,chunk,block,persist'.  Default: 'default' "
                         "for gl_periodic_n2000 (the plan its profiles were taken with; the tuner lands on it or on "
                         "one within noise), 'tuned' for gl_batched_64")
    ap.add_argument("--step-power", type=int, default=None, choices=[1, 2, 4],
                    help="1-D workloads: RK4 steps per kernel step (band P(Z)^m and the combined forcing of m "
                         "steps); default: the library's default (4)")
    ap.add_argument("--algorithm", default="power", choices=["power", "krylov", "trm"],
                    help="gl_periodic_n2000: 'power' (block power iteration, the headline line) or 'krylov' (block "
                         "Arnoldi with --krylov-blocks blocks of k forcings; one step = one call); gl_paper_n200: "
                         "'trm' (transient-response method with time-domain hand-off and FIR flattening; one step = "
                         "one iteration)")
    ap.add_argument("--krylov-blocks", type=int, default=10)
    ap.add_argument("--trm-every", type=int, default=1,
                    help="--algorithm trm: RK4 steps between samples (1: the paper's every-step sampling); the window, "
                         "taper and FIR resolution stay the same (order 3000 / every), and the march takes four "
                         "steps per kernel step when every is a multiple of four")
    ap.add_argument("--weighted", action="store_true",
                    help="gl_periodic_n2000 with diagonal B (forcing window over the upstream 60 %%), C (observation "
                         "window over the downstream 60 %%) and metrics W_f = W_y = dx")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for the HBM byte counters)")
    return ap.parse_args()


def calibrate_copy():
    """A plain copy of known size: 2^30 bytes read and 2^30 bytes written per launch, three launches."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": src.numel() * 4, "launches": 3}), flush=True)


def build_op(cfg, precision):
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import gl_coefficients
    lo, d, up = gl_coefficients(cfg["N"], cfg["mu0"], cfg["mu2"])
    return ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision=precision)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "step1d_gl_periodic_n2000_traffic.md")
STEPPER_SOURCES = ("step1d_kernel.h", "common.h")  # the stepper kernel and the helpers it inlines


def measured_traffic(plan=None, step_power=1):
    """HBM bytes per stepper launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the
    stepper's sources have changed since those counters were taken (their hash is recorded beside the figure) or
    when the run uses a different stepper plan or step power than the profiled one."""
    import hashlib
    h = hashlib.sha256()
    for f in STEPPER_SOURCES:
        with open(os.path.join(ROOT, "paper_2008_10904_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    value, digest, prof_plan, prof_power = None, None, None, 1
    try:
        with open(TRAFFIC_PROFILE) as fh:
            for line in fh:
                if line.startswith("traffic_bytes_per_launch:"):
                    value = float(line.split(":", 1)[1])
                elif line.startswith("source-sha256"):
                    digest = line.rsplit(":", 1)[1].strip()
                elif line.startswith("plan:"):
                    prof_plan = [int(x) for x in line.split(":", 1)[1].split(",")]
                elif line.startswith("step_power:"):
                    prof_power = int(line.split(":", 1)[1])
    except OSError:
        return None
    if digest != h.hexdigest() or (plan is not None and list(plan) != prof_plan) or step_power != prof_power:
        return None
    return value


def choose_plan(op, k, how, search_power=False):
    """Apply the requested stepper plan (see --plan) and return the plan in effect.  A tuned plan with
    search_power also chooses the step power (4, 2 or 1 RK4 steps per kernel step)."""
    from paper_2008_10904_amd import autotune
    if how == "tuned":
        return autotune.tuned(op, k, powers=(4, 2, 1) if search_power else None)[0]
    if how == "default":
        return op.get_plan()
    return op.set_plan([int(x) for x in how.split(",")])


def time_steps(op, f0, grid, run, K, W):
    import torch
    from paper_2008_10904_amd import _lib as L
    for _ in range(W):
        g, _, _, _ = op.modes(f0, grid, run, 1, want_modes=False, want_hist=False)
    torch.cuda.synchronize()
    op.set_timing(True)
    for kind in range(4):
        op.timing(kind)  # reset the counters
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        g, _, _, _ = op.modes(f0, grid, run, 1, want_modes=False, want_hist=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = {name: op.timing(kind) for name, kind in (("stepper", L.RES_TIMING_STEPPER),
                                                   ("synthesis", L.RES_TIMING_SYNTHESIS),
                                                   ("projection", L.RES_TIMING_PROJECTION),
                                                   ("qr", L.RES_TIMING_QR))}
    op.set_timing(False)
    return (t1 - t0) / K, g, kt


def cpu_baseline(cfg, w0, dw, F, seconds):
    """The oracle's explicit RK4 march of the same operator and forcing, timed for a bounded sample of steps."""
    import numpy as np
    from oracle import operators as O_ops
    if cfg["kind"] == "gl_paper":
        L, _ = O_ops.paper_gl_operator(cfg["N"], cfg["beta"], cfg["U"], cfg["gamma"], cfg["length"])
    else:
        L, _ = O_ops.gl_operator(cfg["N"], cfg["mu0"], cfg["mu2"])
    om = w0 + dw * np.arange(cfg["n_omega"])
    from oracle.stepping import march
    march(L, cfg["h"], om, F, 3, lambda s: True, lambda s: False, 1.0)  # warm caches and BLAS threads
    # time-boxed sample: chunks of 200 forced steps until `seconds` have elapsed
    n, t = 0, time.perf_counter()
    while time.perf_counter() - t < seconds:
        march(L, cfg["h"], om, F, 200, lambda s: True, lambda s: False, 1.0)
        n += 200
    dt = time.perf_counter() - t
    sweeps = cfg["N"] * cfg["k"] * cfg["n_omega"] * n / dt
    threads = os.environ.get("OMP_NUM_THREADS") or os.environ.get("OPENBLAS_NUM_THREADS") or str(os.cpu_count())
    return dict(value=sweeps, unit="resolvent sweeps/s", cores=int(threads), kind="oracle",
                sample="%d forced RK4 steps of the N=%d, k=%d, %d-frequency periodic run (FP64 NumPy/SciPy), "
                       "%.1f s" % (n, cfg["N"], cfg["k"], cfg["n_omega"], dt))


def bench_batched(args):
    """One block-power iteration of the batched workload (64 GL instances packed back to back, k = 2, 128
    frequencies, periodic method, mixed precision), with the FP64 form of the same iteration beside it."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import gl_batched_coefficients, snap_grid

    cfg = W.GL_BATCHED
    inst = W.batched_instances()
    lo, d, up, off = gl_batched_coefficients(inst)
    ntot = int(off[-1])
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"], cfg["stride"])
    steps_per_run = cfg["periods"] * P
    F = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], ntot)
    sweeps_per_step = ntot * cfg["k"] * cfg["n_omega"] * 2 * steps_per_run
    res, plans, powers = {}, {}, {}
    for prec, dtype in (("mixed", torch.complex64), ("fp64", torch.complex128)):
        op = ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision=prec, offsets=off)
        if args.step_power:
            op.set_step_power(args.step_power)
        plans[prec] = choose_plan(op, cfg["k"], args.plan, search_power=args.step_power is None)
        powers[prec] = op.get_step_power()
        grid = op.grid(w0, dw, cfg["n_omega"])
        run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
        f = torch.from_numpy(F).to(dtype).cuda()
        res[prec] = time_steps(op, f, grid, run, args.steps, args.warmup)
        del op, f
        torch.cuda.empty_cache()
    dtm, gm, ktm = res["mixed"]
    dt64, g64, kt64 = res["fp64"]
    out = {
        "metric": "resolvent sweeps/s (N*k*Nw*Nt per s)",
        "value": sweeps_per_step / dtm,
        "unit": "resolvent sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dtm * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 step/GEMM, f64 acc",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "instances": len(inst), "N_total": ntot, "k": cfg["k"],
                   "n_omega": cfg["n_omega"], "P": P, "h": cfg["h"], "method": "periodic",
                   "periods": cfg["periods"], "stride": cfg["stride"], "step": "one block-power iteration",
                   "time_steps_per_step": 2 * steps_per_run},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in ktm.items()},
        "fp64": {"value": sweeps_per_step / dt64, "ms_per_step": dt64 * 1e3, "dtype": "f64",
                 "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt64.items()}},
        "max_rel_gain_diff_mixed_vs_fp64": float(np.abs(gm / g64 - 1).max()),
        "stepper_plan": {k: list(v) for k, v in plans.items()},
        "step_power": powers,
    }
    print(json.dumps(out), flush=True)


HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s


def grid_op(cfg, precision):
    import numpy as np
    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import adr2d_coefficients, adr3d3c_coefficients
    if cfg["kind"] == "adr2d":
        c = adr2d_coefficients(cfg["nx"], cfg["ny"], Re=cfg["Re"], mu_base=cfg["mu_base"], mu_amp=cfg["mu_amp"],
                               mu_xc=cfg["mu_xc"], mu_w2=cfg["mu_w2"], nu_s=cfg["nu_s"])
        return ResolventOp.grid_operator("adr2d", cfg["nx"], cfg["ny"], 1, c, cfg["h"], precision=precision)
    wake = W.wake_parameters(cfg["seed"])
    c = adr3d3c_coefficients(cfg["nx"], cfg["ny"], cfg["nz"], wake, Re=cfg["Re"],
                             mu=np.full((cfg["nz"], cfg["ny"], cfg["nx"]), cfg["mu_const"]), nu_s=cfg["nu_s"])
    return ResolventOp.grid_operator("adr3d3c", cfg["nx"], cfg["ny"], cfg["nz"], c, cfg["h"], precision=precision)


def bench_grid(args):
    """Grid workloads.  adr2d_1024x512: one full block-power iteration (transient method, mixed precision).
    adr3d3c_256x128x128: the full-size state does not leave room for a whole iteration's FP64 blocks in one GPU's
    memory, so the stepping is measured alone: one apply of 64 forced steps at the full grid (8 frequencies,
    P = 64), reported per step; the Fourier work scales with the frequency count and is reported separately by
    the iteration of the 2-D workload.  Both report the HBM roofline of the Horner-stage kernel against the
    algorithmic bytes of a step (read and write the state, read one forcing row)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd import _lib as L
    from paper_2008_10904_amd.operators import snap_grid

    cfg = W.ADR2D if args.workload == "adr2d_1024x512" else W.ADR3D
    op = grid_op(cfg, cfg["precision"])
    ncomp = 3 if cfg["kind"] == "adr3d3c" else 1
    nodes = cfg["nx"] * cfg["ny"] * cfg.get("nz", 1)
    N = ncomp * nodes
    k = cfg["k"]
    csize = 8  # complex64 state
    if cfg["kind"] == "adr2d":
        w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"], cfg["stride"])
        nw = cfg["n_omega"]
        run = op.run("transient", tail=cfg["tail"])
        steps_per_run = P + cfg["tail"]
        F = W.random_forcing(cfg["seed"], nw, k, N, dtype=np.complex64)
        f = torch.from_numpy(F).cuda()
        grid = op.grid(w0, dw, nw)
        dt, gains, kt = time_steps(op, f, grid, run, args.steps, args.warmup)
        time_steps_total = 2 * steps_per_run * args.steps
        value = N * k * nw * 2 * steps_per_run / dt
        step_desc = "one block-power iteration"
        # forward plus reverse mode (the C4 gradient path): one apply and one apply_backward with the forcing and
        # mu gradients, checkpoints every ~sqrt(steps), timed outside the iteration above
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = op.apply(f, grid, run)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = (u / u.abs().clamp_min(1e-30)).contiguous()  # dJ/du_hat of J = sum |u_hat| (leading-mode objective)
        op.apply_backward(f, g, grid, run)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        op.apply_backward(f, g, grid, run, want_mu=False)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        autograd = {"forward_s": t1 - t0, "backward_s": t2 - t1, "backward_forcing_only_s": t3 - t2,
                    "note": "one apply and one apply_backward (forcing and mu gradients) of the full workload; "
                            "then the forcing gradient alone (adjoint recursion only)"}
    else:
        nw, P = 8, 64
        dw = 2 * np.pi / (P * cfg["h"])
        F = W.random_forcing(cfg["seed"], nw, k, N, dtype=np.complex64)
        f = torch.from_numpy(F).cuda()
        del F
        grid = op.grid(cfg["wmin"], dw, nw)
        run = op.run("transient", tail=0)
        out_u = op.apply(f, grid, run)
        torch.cuda.synchronize()
        op.set_timing(True)
        for kind in range(4):
            op.timing(kind)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            op.apply(f, grid, run, out=out_u)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        kt = {name: op.timing(kind) for name, kind in (("stepper", L.RES_TIMING_STEPPER),
                                                       ("synthesis", L.RES_TIMING_SYNTHESIS),
                                                       ("projection", L.RES_TIMING_PROJECTION))}
        op.set_timing(False)
        time_steps_total = P * args.steps
        steps_per_run = P
        value = N * k * cfg["n_omega"] * P / (kt["stepper"][0] / 1e3 / args.steps)
        step_desc = "stepping of one 64-step apply (value: sweeps/s of the stepping alone at 96 frequencies)"
    kernel_name = ("grid_step2d_kernel (one RK4 step per launch)" if cfg["kind"] == "adr2d"
                   else "grid_pair3d_kernel x2 (one RK4 step: two launches of two Horner stages)")
    step_s = kt["stepper"][0] / 1e3 / time_steps_total
    alg_bytes = 3 * csize * N * k  # read u, write u, read one forcing row
    achieved = alg_bytes / step_s
    out = {
        "metric": "resolvent sweeps/s (N*k*Nw*Nt per s)", "value": value, "unit": "resolvent sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 step/GEMM, f64 acc",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": [cfg["nx"], cfg["ny"], cfg.get("nz", 1)], "components": ncomp,
                   "k": k, "n_omega": nw, "P": P, "h": cfg["h"], "step": step_desc,
                   "time_steps_per_step": time_steps_total // args.steps},
        "roofline": {"bound": "hbm", "kernel": kernel_name, "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": None,
                     "us_per_time_step": step_s * 1e6, "algorithmic_bytes_per_step": alg_bytes},
        "kernel_ms_per_step": {kk: v[0] / args.steps for kk, v in kt.items()},
    }
    if cfg["kind"] == "adr2d":
        out["autograd"] = autograd
    else:
        del f, out_u
        op = None
        torch.cuda.empty_cache()
        out["autograd"] = grad3d_half(cfg)
    print(json.dumps(out), flush=True)


def grad3d_half(cfg):
    """Forward plus reverse mode of the 3-D workload's gradient pattern: one apply of the periodic method (all
    periods, 96 frequencies, k = 3) and one apply_backward with forcing and mu gradients, checkpoints every 64
    steps.  The reverse mode keeps FP64 rows (forcing, seed and gradient blocks, 64-step segments, checkpoints),
    which at the full grid need more memory than one GPU holds, so this runs the same operator on the grid
    halved in each direction (128 x 64 x 64, one eighth of the state)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd.operators import snap_grid

    half = dict(cfg, nx=cfg["nx"] // 2, ny=cfg["ny"] // 2, nz=cfg["nz"] // 2)
    op = grid_op(half, cfg["precision"])
    N = 3 * half["nx"] * half["ny"] * half["nz"]
    nw, k = cfg["n_omega"], cfg["k"]
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], nw, cfg["h"], cfg["stride"])
    f = torch.from_numpy(W.random_forcing(cfg["seed"], nw, k, N, dtype=np.complex64)).cuda()
    grid = op.grid(w0, dw, nw)
    run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = op.apply(f, grid, run)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = (u / u.abs().clamp_min(1e-30)).contiguous()  # dJ/du_hat of J = sum |u_hat|
    del u
    fg, mg = op.apply_backward(f, g, grid, run, checkpoint_every=cfg["checkpoint_every"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ok = bool(torch.isfinite(fg).all().item()) and bool(np.isfinite(mg.cpu().numpy()).all())
    del fg, mg
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    op.apply_backward(f, g, grid, run, checkpoint_every=cfg["checkpoint_every"], want_mu=False)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    return {"grid": [half["nx"], half["ny"], half["nz"]], "n_omega": nw, "k": k, "P": P,
            "time_steps": cfg["periods"] * P, "checkpoint_every": cfg["checkpoint_every"],
            "forward_s": t1 - t0, "backward_s": t2 - t1, "backward_forcing_only_s": t4 - t3, "finite": ok,
            "note": "one apply and one apply_backward (forcing and mu gradients), periodic method, on the grid "
                    "halved in each direction"}


def bench_krylov(args):
    """gl_periodic_n2000 with the block Arnoldi estimates: one step is one resolvent_krylov call of
    --krylov-blocks blocks of k = 4 forcings (that many direct and adjoint runs), FP64 and mixed.  The power
    iteration's gains after the same number of runs are reported beside it, with both compared on their
    largest suboptimal-gain change over the last block (a convergence indicator)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd import _lib as L
    from paper_2008_10904_amd.operators import snap_grid

    cfg = W.GL_PERIODIC
    nb = args.krylov_blocks
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"], cfg["stride"])
    steps_per_run = cfg["periods"] * P
    F = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], cfg["N"])
    sweeps = cfg["N"] * cfg["k"] * cfg["n_omega"] * 2 * steps_per_run * nb
    res = {}
    for prec, dtype in (("fp64", torch.complex128), ("mixed", torch.complex64)):
        op = build_op(cfg, prec)
        if args.step_power:
            op.set_step_power(args.step_power)
        grid = op.grid(w0, dw, cfg["n_omega"])
        run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
        f = torch.from_numpy(F).to(dtype).cuda()
        for _ in range(args.warmup):
            op.krylov(f, grid, run, nb, want_modes=False, want_hist=False)
        torch.cuda.synchronize()
        op.set_timing(True)
        for kind in range(4):
            op.timing(kind)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g, _, _, hist = op.krylov(f, grid, run, nb, want_modes=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        kt = {name: op.timing(kind)[0] / args.steps for name, kind in (("stepper", L.RES_TIMING_STEPPER),
                                                                       ("synthesis", L.RES_TIMING_SYNTHESIS),
                                                                       ("projection", L.RES_TIMING_PROJECTION),
                                                                       ("arnoldi_and_qr", L.RES_TIMING_QR))}
        op.set_timing(False)
        gp, _, _, hp = op.modes(f, grid, run, nb, want_modes=False)
        torch.cuda.synchronize()
        if prec == "mixed":
            op64 = build_op(cfg, "fp64")
            if args.step_power:
                op64.set_step_power(args.step_power)
            g_fin = op.krylov_polished(op64, f, grid, run, nb)[0]
            torch.cuda.synchronize()
            del op64
        else:
            g_fin = None
        res[prec] = dict(value=sweeps / dt, ms_per_step=dt * 1e3, kernel_ms_per_step=kt, gains=g, power_gains=gp,
                         finished_gains=g_fin,
                         krylov_last_change=float(np.abs(hist[-1] / hist[-2] - 1).max()) if nb > 1 else None,
                         power_last_change=float(np.abs(hp[-1, ..., 0] / hp[-2, ..., 0] - 1).max()) if nb > 1 else None)
        del op, f
        torch.cuda.empty_cache()
    r64, rm = res["fp64"], res["mixed"]
    out = {
        "metric": "resolvent sweeps/s (N*k*Nw*Nt per s)", "value": r64["value"], "unit": "resolvent sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "N": cfg["N"], "k": cfg["k"], "n_omega": cfg["n_omega"], "P": P,
                   "h": cfg["h"], "method": "periodic", "periods": cfg["periods"], "stride": cfg["stride"],
                   "step": "one block Arnoldi call of %d blocks" % nb, "time_steps_per_step": 2 * steps_per_run * nb},
        "kernel_ms_per_step": r64["kernel_ms_per_step"],
        "krylov_vs_power_same_runs": {
            "max_rel_gain_diff": float(np.abs(r64["gains"] / r64["power_gains"] - 1).max()),
            "krylov_last_block_change": r64["krylov_last_change"],
            "power_last_iteration_change": r64["power_last_change"]},
        "mixed": {"value": rm["value"], "ms_per_step": rm["ms_per_step"], "kernel_ms_per_step": rm["kernel_ms_per_step"],
                  "max_rel_gain_diff_vs_fp64": float(np.abs(rm["gains"] / r64["gains"] - 1).max()),
                  "with_fp64_finish": {
                      "max_rel_gain_diff_vs_fp64": float(np.abs(rm["finished_gains"] / r64["gains"] - 1).max()),
                      "leading_gain": float(np.abs(rm["finished_gains"][..., 0] / r64["gains"][..., 0] - 1).max())},
                  "leading_gain_diff_vs_fp64": float(np.abs(rm["gains"][..., 0] / r64["gains"][..., 0] - 1).max())},
    }
    print(json.dumps(out), flush=True)


def bench_paper(args):
    """gl_paper_n200, the paper's own Ginzburg-Landau study (Sec. 3): N = 200, k = 1, 77 frequencies from 0 to 15,
    periodic method with 2 periods of P = 3200 steps, FP64.  One step is one block-power iteration.  Beside it, the
    paper's comparison after the same 15 direct and adjoint runs: one resolvent_modes call of 15 iterations and one
    resolvent_krylov call of 15 blocks, with their omega = 15 gains and the change over their last run."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import paper_gl_coefficients

    cfg = W.GL_PAPER
    N, k, nw, P = cfg["N"], cfg["k"], cfg["n_omega"], cfg["P"]
    steps_per_run = cfg["periods"] * P
    F = W.random_forcing(cfg["seed"] + 1, nw, k, N)
    sweeps_per_step = N * k * nw * 2 * steps_per_run
    lo, d, up = paper_gl_coefficients(N, cfg["beta"], cfg["U"], cfg["gamma"], cfg["length"])
    op = ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision="fp64")
    if args.step_power:
        op.set_step_power(args.step_power)
    plan = choose_plan(op, k, args.plan)
    grid = op.grid(cfg["w0"], cfg["dw"], nw)
    run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
    f = torch.from_numpy(F).cuda()
    dt, _, kt = time_steps(op, f, grid, run, args.steps, args.warmup)
    stepper_ms, stepper_n = kt["stepper"]
    avg_launch_s = stepper_ms / 1e3 / max(stepper_n, 1)
    steps_per_launch = 2 * steps_per_run * args.steps / max(stepper_n, 1)
    achieved = STEP_FLOP_PER_UNKNOWN * N * k * steps_per_launch / avg_launch_s / 1e12
    peak = FP64_VECTOR_PEAK / 1e12
    n = cfg["iters"]
    study = {"runs": n}
    for name, call in (("power", lambda: op.modes(f, grid, run, n, want_modes=False)),
                       ("arnoldi", lambda: op.krylov(f, grid, run, n, want_modes=False))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g, _, _, hist = call()
        torch.cuda.synchronize()
        h15 = hist[..., 0] if name == "power" else hist
        study[name] = {"seconds": time.perf_counter() - t0, "gain_omega0": float(g[0, 0, 0]),
                       "gain_omega15": float(g[0, -1, 0]),
                       "last_run_change_omega15": float(abs(h15[-1, 0, -1, 0] / h15[-2, 0, -1, 0] - 1))}
    out = {
        "metric": "resolvent sweeps/s (N*k*Nw*Nt per s)", "value": sweeps_per_step / dt, "unit": "resolvent sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "N": N, "k": k, "n_omega": nw, "omega0": cfg["w0"], "domega": cfg["dw"],
                   "P": P, "h": cfg["h"], "method": "periodic", "periods": cfg["periods"], "stride": cfg["stride"],
                   "U": cfg["U"], "gamma": cfg["gamma"], "beta": cfg["beta"], "step": "one block-power iteration",
                   "time_steps_per_step": 2 * steps_per_run},
        "roofline": {"bound": "alu", "kernel": "step1d_kernel (fused RK4 step, FP64)", "achieved": achieved,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "avg_launch_ms": avg_launch_s * 1e3, "launches": stepper_n, "steps_per_launch": steps_per_launch},
        "kernel_ms_per_step": {kk: v[0] / args.steps for kk, v in kt.items()},
        "stepper_plan": list(plan), "step_power": op.get_step_power(),
        "power_vs_arnoldi_same_runs": study,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, cfg["w0"], cfg["dw"], F, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_trm(args):
    """gl_paper_trm_n200: the transient-response method with time-domain hand-off on the paper's GL model at its
    own settings (h = 0.01 sampled every step, FIR order 3000 in two passes, 61 analysis frequencies in [-15, 15],
    6001 samples).  One step is one iteration: the direct and adjoint signal runs (6000 RK4 steps each), the
    spectra of F, Y and W, the filter design (host) and the two filter passes.  The roofline object is that of the
    kernel with the larger share of the device time, the FIR filter or the stepper, timed with HIP events on the
    stream it runs on."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd import _lib as L
    from paper_2008_10904_amd.api import fir_apply, fir_design
    from paper_2008_10904_amd.operators import paper_gl_coefficients

    cfg = dict(W.GL_PAPER_TRM)
    e = max(1, args.trm_every)
    if e != cfg["every"]:  # same window, taper and filter resolution with samples e steps apart
        if (cfg["n_samples"] - 1) % e or cfg["order"] % (2 * e) or cfg["pad"] % e or cfg["ramp"] % e:
            print("--trm-every must divide 6000, 1500, 1200 and 600", file=sys.stderr)
            sys.exit(2)
        cfg.update(every=e, n_samples=(cfg["n_samples"] - 1) // e + 1, order=cfg["order"] // e, pad=cfg["pad"] // e,
                   ramp=cfg["ramp"] // e, name=cfg["name"] + "_every%d" % e)
    N, k, n, every = cfg["N"], cfg["k"], cfg["n_samples"], cfg["every"]
    om = np.linspace(-cfg["wmax"], cfg["wmax"], cfg["n_omega"])
    steps_per_run = (n - 1) * every
    sweeps_per_step = N * k * cfg["n_omega"] * 2 * steps_per_run
    lo, d, up = paper_gl_coefficients(N, cfg["beta"], cfg["U"], cfg["gamma"], cfg["length"])
    op = ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision="fp64")
    F0 = W.random_forcing(cfg["seed"], n, k, N)
    f0 = torch.from_numpy(F0).cuda()
    kw = dict(order=cfg["order"], passes=cfg["passes"], pad=cfg["pad"], ramp=cfg["ramp"], margin=cfg["margin"])
    for _ in range(args.warmup):
        op.trm_modes(f0, om, 1, every, cfg["scheme"], **kw)
    torch.cuda.synchronize()
    op.set_timing(True)
    for kind in range(4):
        op.timing(kind)
    iters = max(args.steps, 2)
    t0 = time.perf_counter()
    gains, amps, _ = op.trm_modes(f0, om, iters, every, cfg["scheme"], **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    kt = {name: op.timing(kind) for name, kind in (("stepper", L.RES_TIMING_STEPPER),
                                                   ("prefilter", L.RES_TIMING_SYNTHESIS),
                                                   ("spectra", L.RES_TIMING_PROJECTION),
                                                   ("fir_and_normalise", L.RES_TIMING_QR))}
    op.set_timing(False)
    # the FIR kernel alone at the same shape, on torch's current stream (the stream fir_apply launches on)
    b = fir_design(cfg["order"], [-1.0, -0.2, 0.0, 0.2, 1.0], [0.0, 0.0, 1.0, 0.0, 0.0])
    y = fir_apply(b, f0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 5
    ev[0].record()
    for _ in range(reps):
        fir_apply(b, f0, out=y)
    ev[1].record()
    torch.cuda.synchronize()
    fir_s = ev[0].elapsed_time(ev[1]) / 1e3 / reps
    fir_flop = 8.0 * (cfg["order"] + 1) * n * k * N  # complex multiply-adds of the taps per output
    st_ms, st_n = kt["stepper"]
    peak = FP64_VECTOR_PEAK / 1e12
    fir_share = cfg["passes"] * fir_s * 1e3 * (iters - 1)
    if fir_share >= st_ms:
        roof = {"bound": "alu", "kernel": "fir_kernel (delay-compensated FIR, FP64, order %d)" % cfg["order"],
                "achieved": fir_flop / fir_s / 1e12, "peak": peak, "unit": "TFLOP/s",
                "frac": fir_flop / fir_s / 1e12 / peak, "traffic": None, "avg_launch_ms": fir_s * 1e3}
    else:
        avg = st_ms / 1e3 / max(st_n, 1)
        spl = 2 * steps_per_run * iters / max(st_n, 1)
        ach = STEP_FLOP_PER_UNKNOWN * N * k * spl / avg / 1e12
        roof = {"bound": "alu", "kernel": "step1d_kernel (fused RK4 step, FP64)", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": None, "avg_launch_ms": avg * 1e3,
                "launches": st_n, "steps_per_launch": spl}
    sel = [int(np.argmin(np.abs(om - w))) for w in (0.0, 5.0, 10.0, 15.0)]
    out = {
        "metric": "resolvent sweeps/s (N*k*Nw*Nt per s)", "value": sweeps_per_step / dt, "unit": "resolvent sweeps/s",
        "n_gpus": 1, "steps": iters, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "N": N, "k": k, "n_omega": cfg["n_omega"], "band": [-cfg["wmax"], cfg["wmax"]],
                   "h": cfg["h"], "samples": n, "every": every, "fir_order": cfg["order"], "fir_passes": cfg["passes"],
                   "interpolation": cfg["scheme"], "method": "transient, time-domain hand-off",
                   "step": "one TRM iteration", "time_steps_per_step": 2 * steps_per_run},
        "roofline": roof,
        "kernel_ms_per_step": {kk: v[0] / iters for kk, v in kt.items()},
        "step_power": op.get_step_power(),
        "fir_kernel_ms": fir_s * 1e3,
        "gains_last_iteration": {"omega": [float(om[j]) for j in sel], "gain": [float(gains[-1, j]) for j in sel]},
        "amplitude_ratio_per_iteration": [float(a.max() / a.min()) for a in amps],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_trm(cfg, F0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline_trm(cfg, F0, seconds):
    """The oracle's signal run (RK4 with C2 stage forcing) of the same operator, timed on growing prefixes of the
    forcing until about `seconds` have passed; rate in the same unit as the GPU line."""
    from oracle import operators as O_ops
    from oracle import trm as O_trm
    L, _ = O_ops.paper_gl_operator(cfg["N"], cfg["beta"], cfg["U"], cfg["gamma"], cfg["length"])
    scheme = {"C0": 0, "C1": 1, "C2": 2}[cfg["scheme"]]
    O_trm.march_signal(L, cfg["h"], F0[:3], cfg["every"], scheme)  # warm up
    steps, t, m = 0, time.perf_counter(), 101
    while time.perf_counter() - t < seconds:
        O_trm.march_signal(L, cfg["h"], F0[:m], cfg["every"], scheme)
        steps += (m - 1) * cfg["every"]
    dt = time.perf_counter() - t
    threads = os.environ.get("OMP_NUM_THREADS") or os.environ.get("OPENBLAS_NUM_THREADS") or str(os.cpu_count())
    return dict(value=cfg["N"] * cfg["k"] * cfg["n_omega"] * steps / dt, unit="resolvent sweeps/s",
                cores=int(threads), kind="oracle",
                sample="%d RK4 steps of the oracle's signal run (C2 stage forcing, N=%d, k=%d; the spectra at %d "
                       "frequencies counted as in the GPU line), %.1f s" % (steps, cfg["N"], cfg["k"],
                                                                          cfg["n_omega"], dt))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.plan is None:
        args.plan = "tuned" if args.workload == "gl_batched_64" else "default"
    if args.weighted and (args.workload != "gl_periodic_n2000" or args.algorithm != "power"):
        print("--weighted measures the block-power iteration of gl_periodic_n2000", file=sys.stderr)
        sys.exit(2)
    if args.algorithm == "trm":
        if args.workload != "gl_paper_n200":
            print("--algorithm trm measures gl_paper_n200", file=sys.stderr)
            sys.exit(2)
        bench_trm(args)
        return
    if args.algorithm == "krylov":
        if args.workload != "gl_periodic_n2000":
            print("--algorithm krylov measures gl_periodic_n2000", file=sys.stderr)
            sys.exit(2)
        bench_krylov(args)
        return
    if args.workload == "gl_batched_64":
        bench_batched(args)
        return
    if args.workload == "gl_paper_n200":
        bench_paper(args)
        return
    if args.workload in ("adr2d_1024x512", "adr3d3c_256x128x128"):
        bench_grid(args)
        return
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd.operators import snap_grid

    cfg = W.GL_PERIODIC
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], cfg["n_omega"], cfg["h"], cfg["stride"])
    steps_per_run = cfg["periods"] * P
    F = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], cfg["N"])
    sweeps_per_step = cfg["N"] * cfg["k"] * cfg["n_omega"] * 2 * steps_per_run

    weights = W.gl_weights(cfg["N"]) if args.weighted else None
    op = build_op(cfg, "fp64")
    if weights is not None:
        op.set_weights(*weights)
    if args.step_power:
        op.set_step_power(args.step_power)
    plan64 = choose_plan(op, cfg["k"], args.plan)  # set-up: the stepper plan
    power = op.get_step_power()
    grid = op.grid(w0, dw, cfg["n_omega"])
    run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
    f64 = torch.from_numpy(F).cuda()
    dt, gains64, kt = time_steps(op, f64, grid, run, args.steps, args.warmup)
    stepper_ms, stepper_n = kt["stepper"]
    avg_launch_s = stepper_ms / 1e3 / max(stepper_n, 1)
    steps_per_launch = 2 * steps_per_run * args.steps / max(stepper_n, 1)
    flop_per_launch = STEP_FLOP_PER_UNKNOWN * cfg["N"] * cfg["k"] * steps_per_launch
    achieved = flop_per_launch / avg_launch_s / 1e12
    peak = FP64_VECTOR_PEAK / 1e12
    out = {
        "metric": "resolvent sweeps/s (N*k*Nw*Nt per s)",
        "value": sweeps_per_step / dt,
        "unit": "resolvent sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "N": cfg["N"], "k": cfg["k"], "n_omega": cfg["n_omega"],
                   "omega0": w0, "domega": dw, "P": P, "h": cfg["h"], "method": "periodic",
                   "periods": cfg["periods"], "stride": cfg["stride"], "step": "one block-power iteration",
                   "time_steps_per_step": 2 * steps_per_run},
        "roofline": {"bound": "alu", "kernel": "step1d_kernel (fused RK4 step, FP64)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(plan64, power), "avg_launch_ms": avg_launch_s * 1e3, "launches": stepper_n,
                     "steps_per_launch": steps_per_launch},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
        "stepper_plan": list(plan64),
        "step_power": power,
    }
    if weights is not None:
        out["config"]["weights"] = ("B: window over the upstream 60 %, C: window over the downstream 60 %, "
                                    "W_f = W_y = dx (gains of C R B in the W norms)")
    del op, f64
    torch.cuda.empty_cache()
    if not args.no_mixed:
        opm = build_op(cfg, "mixed")
        if weights is not None:
            opm.set_weights(*weights)
        if args.step_power:
            opm.set_step_power(args.step_power)
        planm = choose_plan(opm, cfg["k"], args.plan)
        f32 = torch.from_numpy(F).to(torch.complex64).cuda()
        dtm, gainsm, ktm = time_steps(opm, f32, grid, run, args.steps, args.warmup)
        out["mixed"] = {"value": sweeps_per_step / dtm, "ms_per_step": dtm * 1e3, "dtype": "f32 step/GEMM, f64 acc",
                        "max_rel_gain_diff_vs_fp64": float(np.abs(gainsm / gains64 - 1).max()),
                        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in ktm.items()},
                        "stepper_plan": list(planm)}
        del opm, f32
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, w0, dw, F, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
