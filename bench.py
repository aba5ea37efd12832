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
    ap.add_argument("--accuracy-iters", type=int, default=None,
                    help="iterations of the untimed accuracy pass against the oracle (default: the workload's own "
                         "iteration count; 0 skips it).  The gains and modes at sampled frequencies are compared "
                         "with the CPU oracle's same iteration, which runs in the CPU-baseline leg")
    ap.add_argument("--accuracy-every", type=int, default=8,
                    help="gl_batched_64: compare every n-th instance with the oracle (8: eight instances, all four "
                         "sizes; 1: all 64, a few minutes of oracle work)")
    ap.add_argument("--workload", default="gl_periodic_n2000",
                    choices=["gl_periodic_n2000", "gl_transient_n200", "gl_batched_64", "adr2d_1024x512",
                             "adr3d3c_256x128x128", "gl_paper_n200"],
                    help="gl_periodic_n2000 (default, the headline line), gl_transient_n200 (the transient-response "
                         "method's iteration on the N = 200 GL operator), gl_batched_64 (64 uneven GL instances, "
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
    ap.add_argument("--no-autograd", action="store_true",
                    help="grid workloads: skip the reverse-mode part (apply_backward) after the timed iterations")
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


def measured_traffic(plan=None, step_power=1, steps_per_launch=None):
    """HBM bytes per stepper launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the
    stepper's sources have changed since those counters were taken (their hash is recorded beside the figure) or
    when the run uses a different stepper plan or step power than the profiled one.  The profiled launches march
    whole periods; launches of another average length (the first period marched in chunks beside the table's
    synthesis) scale the figure by their RK4 steps (the traffic is the forcing rows and the exchanges, both
    per step)."""
    import hashlib
    h = hashlib.sha256()
    for f in STEPPER_SOURCES:
        with open(os.path.join(ROOT, "paper_2008_10904_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    value, digest, prof_plan, prof_power, prof_steps = None, None, None, 1, None
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
                elif line.startswith("rk4_steps_per_launch:"):
                    prof_steps = float(line.split(":", 1)[1])
    except OSError:
        return None
    if digest != h.hexdigest() or (plan is not None and list(plan) != prof_plan) or step_power != prof_power:
        return None
    if steps_per_launch is not None and prof_steps:
        return value * steps_per_launch / prof_steps
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


def progress(msg):
    """One progress line on stderr (the JSON line stays alone on stdout)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def time_steps(op, f0, grid, run, K, W):
    import torch
    from paper_2008_10904_amd import _lib as L
    for i in range(W):
        g, _, _, _ = op.modes(f0, grid, run, 1, want_modes=False, want_hist=False)
        torch.cuda.synchronize()
        progress("warmup step %d of %d done" % (i + 1, W))
    torch.cuda.synchronize()
    op.set_timing(True)
    for kind in range(4):
        op.timing(kind)  # reset the counters
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        g, _, _, _ = op.modes(f0, grid, run, 1, want_modes=False, want_hist=False)
        if K > 1 and i + 1 < K and (time.perf_counter() - t0) > 30.0:
            progress("timed step %d of %d queued" % (i + 1, K))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress("%d timed steps done" % K)
    kt = {name: op.timing(kind) for name, kind in (("stepper", L.RES_TIMING_STEPPER),
                                                   ("synthesis", L.RES_TIMING_SYNTHESIS),
                                                   ("projection", L.RES_TIMING_PROJECTION),
                                                   ("qr", L.RES_TIMING_QR))}
    op.set_timing(False)
    return (t1 - t0) / K, g, kt


def graph_replay(op, f0, grid, run, iters):
    """Wall time per iteration of one resolvent_modes call of `iters` iterations, eager and with the middle
    iterations replayed from one captured HIP graph (resolvent_op_set_graphs), each after a warm call of two
    iterations; and whether the two give the same gains bit for bit."""
    import numpy as np
    import torch
    out = {"iterations": iters}
    gains = {}
    for name, on in (("eager", False), ("graph", True)):
        op.set_graphs(on)
        op.modes(f0, grid, run, 2, want_modes=False, want_hist=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g, _, _, _ = op.modes(f0, grid, run, iters, want_modes=False, want_hist=False)
        torch.cuda.synchronize()
        out[name + "_ms_per_iteration"] = (time.perf_counter() - t0) / iters * 1e3
        gains[name] = g
    op.set_graphs(False)
    out["same_gains"] = bool(np.array_equal(gains["eager"], gains["graph"]))
    progress("graph replay timed")
    return out


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
    return dict(value=sweeps, unit="resolvent sweeps/s", cores=oracle_threads(), kind="oracle", host=host_cpu(),
                sample="%d forced RK4 steps of the N=%d, k=%d, %d-frequency periodic run (FP64 NumPy/SciPy), "
                       "%.1f s" % (n, cfg["N"], cfg["k"], cfg["n_omega"], dt))


def host_cpu():
    """Model name and L3 size of the host CPU (lscpu), for the CPU baseline's record."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            key, _, val = line.partition(":")
            if key.strip() in ("Model name", "L3 cache", "CPU(s)"):
                info[key.strip()] = val.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return {"model": info.get("Model name"), "l3": info.get("L3 cache"), "logical_cpus": info.get("CPU(s)")}


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS") or os.environ.get("OPENBLAS_NUM_THREADS") or os.cpu_count())


def mode_errors(X, Y, gains, gap=1e-6):
    """Per-mode error of modes X (k, N) against reference modes Y (k, N) with reference gains (k,) sorted
    descending: min over phases of ||x e^{i phi} - y|| for unit vectors; modes in a cluster of gains closer than
    `gap` (relative) get the 2-norm distance between the cluster's subspaces instead (a mode is unique only up to
    a phase, and a degenerate one only as a subspace)."""
    import numpy as np
    X = np.asarray(X, complex)
    Y = np.asarray(Y, complex)
    k = X.shape[0]
    Xn = X / np.linalg.norm(X, axis=1, keepdims=True)
    Yn = Y / np.linalg.norm(Y, axis=1, keepdims=True)
    out = np.zeros(k)
    i = 0
    while i < k:
        j = i + 1
        while j < k and (gains[j - 1] - gains[j]) < gap * gains[j - 1]:
            j += 1
        if j == i + 1:
            c = np.vdot(Xn[i], Yn[i])
            out[i] = np.linalg.norm(Xn[i] * (c / abs(c) if abs(c) > 0 else 1.0) - Yn[i])
        else:
            Qx = np.linalg.qr(X[i:j].T)[0]
            Qy = np.linalg.qr(Y[i:j].T)[0]
            out[i:j] = np.linalg.norm(Qy - Qx @ (Qx.conj().T @ Qy), 2)
        i = j
    return out


def accuracy(g, V, U, g_ref, V_ref, U_ref, labels):
    """Error of every sampled gain and mode against the oracle: per sample, the relative gain errors and the mode
    errors (mode_errors), and their maxima."""
    import numpy as np
    rows = []
    for i, lab in enumerate(labels):
        rows.append({"sample": lab, "gain_rel_err": [float(x) for x in np.abs(g[i] / g_ref[i] - 1)],
                     "force_mode_err": [float(x) for x in mode_errors(V[i], V_ref[i], g_ref[i])],
                     "response_mode_err": [float(x) for x in mode_errors(U[i], U_ref[i], g_ref[i])]})
    return {"max_gain_rel_err": max(max(r["gain_rel_err"]) for r in rows),
            "max_leading_gain_rel_err": max(r["gain_rel_err"][0] for r in rows),
            "max_force_mode_err": max(max(r["force_mode_err"]) for r in rows),
            "max_response_mode_err": max(max(r["response_mode_err"]) for r in rows),
            "per_sample": rows}


def gpu_modes_sampled(op, f0, grid, run, iters, js, sl=None, inst=0, finish_op=None):
    """GPU block power iteration of `iters` iterations (with the FP64 Rayleigh-Ritz finish on finish_op when given);
    gains, force and response modes at the frequencies js (and unknowns sl of instance inst)."""
    import numpy as np
    if finish_op is not None:
        g, V, U, _ = op.modes_polished(finish_op, f0, grid, run, iters, want_hist=False)
    else:
        g, V, U, _ = op.modes(f0, grid, run, iters, want_hist=False)
    V = V.cpu().numpy().astype(complex)
    U = U.cpu().numpy().astype(complex)
    sl = slice(None) if sl is None else sl
    return g[inst][js], V[js][:, :, sl], U[js][:, :, sl]


def oracle_sampled_reference(L, h, omegas, F_sel, iters):
    """The CPU oracle's block power iteration (App. A) at the sampled frequencies only, from the same start, with
    the RK4 transfer matrices R_d(w_j) from its dense solve (frequencies are independent in the block iteration,
    and after the settle periods the periodic run applies R_d exactly).  F_sel: (n_sel, k, N).  Returns
    (gains, V, U).  Part of the CPU-baseline leg: the oracle runs on the host, outside the timed region."""
    from oracle.iteration import block_power_iteration, dense_rk4_applies
    a, ad = dense_rk4_applies(L, h, omegas)
    g, V, U, _ = block_power_iteration(a, ad, F_sel, iters)
    return g, V, U


TRANSIENT_REFERENCE = os.path.join(ROOT, "tests", "golden", "gl_transient_reference.json")


def bench_transient(args):
    """gl_transient_n200: the transient-response method (one forcing window of P = 9,896 steps and a 20,000-step
    tail) on the N = 200 GL operator, 64 frequencies in [-2, 2], k = 1.  One step is one block-power iteration
    (direct and adjoint run of 29,896 steps each, QR and gains), FP64, with the mixed form beside it.  The accuracy
    pass runs the workload's 20 iterations and compares every gain, and the modes at the stored frequencies, with
    the oracle's same iteration stored in tests/golden/gl_transient_reference.json (written by the script beside
    it, which calls only the oracle).  The oracle is timed on whole iterations of its explicit RK4 runs."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd.operators import snap_grid

    cfg = W.GL_TRANSIENT
    N, k, nw = cfg["N"], cfg["k"], cfg["n_omega"]
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], nw, cfg["h"])
    S = P + cfg["tail"]
    F = W.random_forcing(cfg["seed"], nw, k, N)
    sweeps_per_step = N * k * nw * 2 * S
    iters = cfg["iters"] if args.accuracy_iters is None else args.accuracy_iters
    with open(TRANSIENT_REFERENCE) as fh:
        ref = json.load(fh)
    js = ref["sampled"]
    g_ref = np.array(ref["gains"])
    V_ref = np.array(ref["V_re"]) + 1j * np.array(ref["V_im"])
    U_ref = np.array(ref["U_re"]) + 1j * np.array(ref["U_im"])
    res = {}
    for prec, dtype in (("fp64", torch.complex128), ("mixed", torch.complex64)):
        op = build_op(cfg, prec)
        plan = choose_plan(op, k, args.plan)
        grid = op.grid(w0, dw, nw)
        run = op.run("transient", tail=cfg["tail"])
        f = torch.from_numpy(F).to(dtype).cuda()
        dt, _, kt = time_steps(op, f, grid, run, args.steps, args.warmup)
        if prec == "fp64":
            replay = graph_replay(op, f, grid, run, 20)
        acc = None
        if iters == ref["iters"]:
            g, V, U, _ = op.modes(f, grid, run, iters, want_hist=False)
            V = V.cpu().numpy().astype(complex)
            U = U.cpu().numpy().astype(complex)
            acc = accuracy(g[0][js], V[js], U[js], g_ref[js], V_ref, U_ref, js)
            acc["max_gain_rel_err_all_frequencies"] = float(np.abs(g[0] / g_ref - 1).max())
            del acc["per_sample"]
        res[prec] = (dt, kt, plan, op.get_step_power(), acc)
        del op, f
        torch.cuda.empty_cache()
    dt, kt, plan, power, acc64 = res["fp64"]
    stepper_ms, stepper_n = kt["stepper"]
    avg = stepper_ms / 1e3 / max(stepper_n, 1)
    spl = 2 * S * args.steps / max(stepper_n, 1)
    achieved = STEP_FLOP_PER_UNKNOWN * N * k * spl / avg / 1e12
    peak = FP64_VECTOR_PEAK / 1e12
    dtm, ktm, planm, _, accm = res["mixed"]
    out = {
        "metric": "resolvent sweeps/s (N*k*Nw*Nt per s)", "value": sweeps_per_step / dt, "unit": "resolvent sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "N": N, "mu0": cfg["mu0"], "k": k, "n_omega": nw, "omega0": w0,
                   "domega": dw, "P": P, "tail": cfg["tail"], "h": cfg["h"], "method": "transient",
                   "step": "one block-power iteration", "time_steps_per_step": 2 * S},
        "roofline": {"bound": "alu", "kernel": "step1d_kernel (fused RK4 step, FP64)", "achieved": achieved,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "avg_launch_ms": avg * 1e3, "launches": stepper_n, "steps_per_launch": spl,
                     "ns_per_time_step": avg / spl * 1e9},
        "kernel_ms_per_step": {kk: v[0] / args.steps for kk, v in kt.items()},
        "stepper_plan": list(plan), "step_power": power,
        "mixed": {"value": sweeps_per_step / dtm, "ms_per_step": dtm * 1e3, "dtype": "f32 step/GEMM, f64 acc",
                  "kernel_ms_per_step": {kk: v[0] / args.steps for kk, v in ktm.items()}, "stepper_plan": list(planm)},
        "accuracy_vs_oracle": {"iterations": iters, "sampled_omega_index": js, "fp64": acc64, "mixed": accm,
                               "reference": "tests/golden/gl_transient_reference.json (the oracle's 20 iterations)"},
        "graph_replay_fp64": replay,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_transient(cfg, w0, dw, F, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline_transient(cfg, w0, dw, F, seconds):
    """The oracle's block power iteration on the same workload (explicit RK4 direct and adjoint runs of
    P + tail steps, NumPy QR and SVD), timed on whole iterations from the same start until `seconds` have passed
    (at least one)."""
    from oracle.iteration import block_power_iteration, stepped_applies
    from oracle.operators import gl_operator
    from oracle.stepping import period_steps
    L, _ = gl_operator(cfg["N"], cfg["mu0"], cfg["mu2"])
    a, ad = stepped_applies(L, cfg["h"], w0, dw, "transient", tail=cfg["tail"])
    S = period_steps(dw, cfg["h"]) + cfg["tail"]
    n, t = 0, time.perf_counter()
    while n == 0 or time.perf_counter() - t < seconds:
        block_power_iteration(a, ad, F, 1)
        n += 1
    dt = time.perf_counter() - t
    return dict(value=cfg["N"] * cfg["k"] * cfg["n_omega"] * 2 * S * n / dt, unit="resolvent sweeps/s",
                cores=oracle_threads(), kind="oracle", host=host_cpu(),
                sample="%d whole iteration(s) of the oracle's block power iteration (two explicit RK4 runs of %d "
                       "steps, N=%d, %d frequencies), %.1f s" % (n, S, cfg["N"], cfg["n_omega"], dt))


FP32_VECTOR_PEAK = 157.3e12  # MI355X FP32 vector peak (packed FP32 issue; the build issues unpacked FP32)


def bench_batched(args):
    """One block-power iteration of the batched workload (64 GL instances packed back to back, k = 2, 128
    frequencies, periodic method, mixed precision), with the FP64 form of the same iteration beside it.  The
    accuracy pass runs the workload's 20 iterations (mixed, mixed with the FP64 Rayleigh-Ritz finish, FP64) and
    compares gains and modes at every eighth instance (eight, all four sizes) and three frequencies with the
    oracle's same iteration.  The CPU baseline times the oracle's march on one instance of each size."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd.operators import gl_batched_coefficients, snap_grid

    cfg = W.GL_BATCHED
    inst = W.batched_instances()
    lo, d, up, off = gl_batched_coefficients(inst)
    ntot = int(off[-1])
    k, nw = cfg["k"], cfg["n_omega"]
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], nw, cfg["h"], cfg["stride"])
    steps_per_run = cfg["periods"] * P
    F = W.random_forcing(cfg["seed"], nw, k, ntot)
    sweeps_per_step = ntot * k * nw * 2 * steps_per_run
    iters = cfg["iters"] if args.accuracy_iters is None else args.accuracy_iters
    picks = list(range(0, len(inst), max(1, args.accuracy_every)))  # default: every eighth, all four sizes
    js = [0, 64, 127]
    res, plans, powers, sampled = {}, {}, {}, {}
    V_mixed = None
    for prec, dtype in (("mixed", torch.complex64), ("fp64", torch.complex128)):
        op = ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision=prec, offsets=off)
        if args.step_power:
            op.set_step_power(args.step_power)
        plans[prec] = choose_plan(op, k, args.plan, search_power=args.step_power is None)
        powers[prec] = op.get_step_power()
        grid = op.grid(w0, dw, nw)
        run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
        f = torch.from_numpy(F).to(dtype).cuda()
        res[prec] = time_steps(op, f, grid, run, args.steps, args.warmup)
        if prec == "mixed":
            replay = graph_replay(op, f, grid, run, 6)
        if iters > 0:
            g, V, U, _ = op.modes(f, grid, run, iters, want_hist=False)
            if prec == "mixed":
                V_mixed = V.to(torch.complex128).contiguous()  # the subspace of the FP64 finish below
            sampled[prec] = (g, V.cpu().numpy().astype(complex), U.cpu().numpy().astype(complex))
            del V, U
            if prec == "fp64":
                g, V, U, _ = op.modes(V_mixed, grid, run, 1, want_hist=False)  # Rayleigh-Ritz on the mixed subspace
                sampled["mixed_fp64_finish"] = (g, V.cpu().numpy().astype(complex), U.cpu().numpy().astype(complex))
                del V, U, V_mixed
        del op, f
        torch.cuda.empty_cache()
    dtm, gm, ktm = res["mixed"]
    dt64, g64, kt64 = res["fp64"]
    st_ms, st_n = ktm["stepper"]
    avg = st_ms / 1e3 / max(st_n, 1)
    spl = 2 * steps_per_run * args.steps / max(st_n, 1)
    achieved = STEP_FLOP_PER_UNKNOWN * ntot * k * spl / avg
    out = {
        "metric": "resolvent sweeps/s (N*k*Nw*Nt per s)",
        "value": sweeps_per_step / dtm,
        "unit": "resolvent sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dtm * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 step/GEMM, f64 acc",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "instances": len(inst), "N_total": ntot, "k": k,
                   "n_omega": nw, "P": P, "h": cfg["h"], "method": "periodic",
                   "periods": cfg["periods"], "stride": cfg["stride"], "step": "one block-power iteration",
                   "time_steps_per_step": 2 * steps_per_run},
        "roofline": {"bound": "alu", "kernel": "step1d_kernel (fused RK4 steps, FP32, all instances in one launch)",
                     "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK, "traffic": None, "avg_launch_ms": avg * 1e3,
                     "launches": st_n, "steps_per_launch": spl},
        "kernel_ms_per_step": {k_: v[0] / args.steps for k_, v in ktm.items()},
        "fp64": {"value": sweeps_per_step / dt64, "ms_per_step": dt64 * 1e3, "dtype": "f64",
                 "kernel_ms_per_step": {k_: v[0] / args.steps for k_, v in kt64.items()}},
        "stepper_plan": {k_: list(v) for k_, v in plans.items()},
        "graph_replay_mixed": replay,
        "step_power": powers,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(cfg, inst, w0, dw, args.cpu_seconds)
        if sampled:
            out["accuracy_vs_oracle"] = batched_accuracy(cfg, inst, off, w0, dw, F, picks, js, iters, sampled)
    print(json.dumps(out), flush=True)


def batched_accuracy(cfg, inst, off, w0, dw, F, picks, js, iters, sampled):
    """Sampled instances and frequencies of the batched GPU iterations against the oracle's same iteration."""
    import numpy as np
    from oracle.operators import gl_operator
    t = time.perf_counter()
    out = {"iterations": iters, "instances": picks, "sampled_omega_index": js}
    refs = {}
    for i, m in enumerate(picks):
        n, mu0, mu2 = inst[m]
        L, _ = gl_operator(n, mu0, mu2)
        if i % 8 == 7:
            progress("oracle references: %d of %d instances" % (i + 1, len(picks)))
        sl = slice(int(off[m]), int(off[m + 1]))
        om = w0 + dw * np.asarray(js)
        for kind in ("fp64", "mixed"):
            Fin = F[js][:, :, sl] if kind == "fp64" else F[js][:, :, sl].astype(np.complex64).astype(np.complex128)
            refs[(m, kind)] = oracle_sampled_reference(L, cfg["h"], om, Fin, iters)
    for prec, (g, V, U) in sampled.items():
        kind = "fp64" if prec == "fp64" else "mixed"
        rows = {}
        for m in picks:
            sl = slice(int(off[m]), int(off[m + 1]))
            g_ref, V_ref, U_ref = refs[(m, kind)]
            rows["instance %d (N=%d)" % (m, inst[m][0])] = accuracy(g[m][js], V[js][:, :, sl], U[js][:, :, sl],
                                                                      g_ref, V_ref, U_ref, js)
        out[prec] = {"max_gain_rel_err": max(r["max_gain_rel_err"] for r in rows.values()),
                     "max_leading_gain_rel_err": max(r["max_leading_gain_rel_err"] for r in rows.values()),
                     "max_force_mode_err": max(r["max_force_mode_err"] for r in rows.values()),
                     "max_response_mode_err": max(r["max_response_mode_err"] for r in rows.values()),
                     "per_instance": {kk: {x: v for x, v in r.items() if x != "per_sample"} for kk, r in rows.items()}}
    out["oracle_seconds"] = time.perf_counter() - t
    out["targets"] = {"fp64_gain": 1e-8, "mixed_gain": 1e-4}
    return out


def cpu_baseline_batched(cfg, inst, w0, dw, seconds):
    """The oracle's forced march (the batch's 128 frequencies, k = 2) on one instance of each size, each timed for
    a quarter of `seconds`; the batch's oracle time per step is the sum over its instances of their sizes' step
    times, and the rate is the batch's sweeps per step over that."""
    import numpy as np
    import workloads as W
    from oracle.operators import gl_operator
    from oracle.stepping import march
    om = w0 + dw * np.arange(cfg["n_omega"])
    per_step = {}
    for n in sorted({x[0] for x in inst}):
        _, mu0, mu2 = next(x for x in inst if x[0] == n)
        L, _ = gl_operator(n, mu0, mu2)
        F = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], n)
        march(L, cfg["h"], om, F, 3, lambda s: True, lambda s: False, 1.0)
        steps, t = 0, time.perf_counter()
        while time.perf_counter() - t < seconds / 4:
            march(L, cfg["h"], om, F, 100, lambda s: True, lambda s: False, 1.0)
            steps += 100
        per_step[n] = (time.perf_counter() - t) / steps
    t_step = sum(per_step[x[0]] for x in inst)
    ntot = sum(x[0] for x in inst)
    return dict(value=ntot * cfg["k"] * cfg["n_omega"] / t_step, unit="resolvent sweeps/s", cores=oracle_threads(),
                kind="oracle", host=host_cpu(),
                sample="forced RK4 steps of one instance of each size (%s), %.1f s each; batch time per step = sum "
                       "over the 64 instances (%.3g s)" % (",".join(str(n) for n in per_step), seconds / 4, t_step))


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
    """Grid workloads, one step = one block-power iteration (direct and adjoint run, QR and gains), mixed precision.
    adr2d_1024x512: transient method (P = 19,949 plus a 15,000-step tail), 128 frequencies, k = 2; then one forward
    apply and its reverse mode (forcing and mu gradients).  adr3d3c_256x128x128: the 3-D workload's own run shape:
    96 frequencies, k = 3, periodic method with three periods of P = 3,800 steps, the last projected every 38th
    step; its forcing is drawn on the device (workloads.random_forcing_device).  Both report the HBM roofline of
    the step kernel against the algorithmic bytes of a step (read and write the state, read one forcing row)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd.operators import snap_grid

    three = args.workload != "adr2d_1024x512"
    cfg = W.ADR3D if three else W.ADR2D
    op = grid_op(cfg, cfg["precision"])
    ncomp = 3 if three else 1
    nodes = cfg["nx"] * cfg["ny"] * cfg.get("nz", 1)
    N = ncomp * nodes
    k, nw = cfg["k"], cfg["n_omega"]
    csize = 8  # complex64 state
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], nw, cfg["h"], cfg["stride"])
    if three:
        run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
        steps_per_run = cfg["periods"] * P
        f = W.random_forcing_device(cfg["seed"], nw, k, N, torch.complex64, "cuda")
    else:
        run = op.run("transient", tail=cfg["tail"])
        steps_per_run = P + cfg["tail"]
        f = torch.from_numpy(W.random_forcing(cfg["seed"], nw, k, N, dtype=np.complex64)).cuda()
    grid = op.grid(w0, dw, nw)
    dt, gains, kt = time_steps(op, f, grid, run, args.steps, args.warmup)
    time_steps_total = 2 * steps_per_run * args.steps
    value = N * k * nw * 2 * steps_per_run / dt
    autograd = None
    if not three and not args.no_autograd:
        # forward plus reverse mode (the 2-D gradient path): one apply and one apply_backward with the forcing and
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
    kernel_name = ("grid_step2d_kernel (two RK4 steps per launch)" if not three
                   else "grid_step3d_kernel (one RK4 step per launch: the four Horner stages pipelined along z)")
    step_s = kt["stepper"][0] / 1e3 / time_steps_total
    alg_bytes = 3 * csize * N * k  # read u, write u, read one forcing row
    achieved = alg_bytes / step_s
    out = {
        "metric": "resolvent sweeps/s (N*k*Nw*Nt per s)", "value": value, "unit": "resolvent sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 step/GEMM, f64 acc",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": [cfg["nx"], cfg["ny"], cfg.get("nz", 1)], "components": ncomp,
                   "k": k, "n_omega": nw, "P": P, "h": cfg["h"], "method": cfg["method"],
                   "periods": cfg["periods"] if three else None, "tail": None if three else cfg["tail"],
                   "stride": cfg["stride"], "step": "one block-power iteration",
                   "time_steps_per_step": 2 * steps_per_run},
        "roofline": {"bound": "hbm", "kernel": kernel_name, "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": None,
                     "us_per_time_step": step_s * 1e6, "algorithmic_bytes_per_step": alg_bytes},
        "kernel_ms_per_step": {kk: v[0] / args.steps for kk, v in kt.items()},
    }
    del f
    op = None
    torch.cuda.empty_cache()
    if autograd is not None:
        out["autograd"] = autograd
    elif three and not args.no_autograd:
        out["autograd"] = grad3d(cfg)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_grid(cfg, w0, dw, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline_grid(cfg, w0, dw, seconds):
    """The oracle's forced RK4 march (sparse L, all frequencies synthesised per stage) of the grid workload, timed
    on chunks of steps until `seconds` have passed.  The 2-D workload runs at full size; the 3-D one on the grid
    halved in each direction (one eighth of the unknowns: its full-size forcing, 58 GB in FP64, and the oracle's
    copies of it do not fit the host's memory), which leaves the oracle's rate per unknown unchanged (every part
    of its step is linear in the unknowns)."""
    import numpy as np
    import workloads as W
    from oracle import operators as O_ops
    from oracle.stepping import march
    if cfg["kind"] == "adr2d":
        f = O_ops.adr2d_fields(cfg["nx"], cfg["ny"], nu_s=cfg["nu_s"])
        mu = O_ops.adr2d_mu_default(f["X"], f["Y"], base=cfg["mu_base"], amp=cfg["mu_amp"], xc=cfg["mu_xc"],
                                    width2=cfg["mu_w2"])
        L, _ = O_ops.adr2d_operator(cfg["nx"], cfg["ny"], Re=cfg["Re"], mu=mu, nu_s=cfg["nu_s"])
        shape = (cfg["nx"], cfg["ny"], 1)
    else:
        shape = (cfg["nx"] // 2, cfg["ny"] // 2, cfg["nz"] // 2)
        L, _ = O_ops.adr3d3c_operator(*shape, W.wake_parameters(cfg["seed"]), Re=cfg["Re"],
                                      mu=np.full(shape[::-1], cfg["mu_const"]), nu_s=cfg["nu_s"])
    N = L.shape[0]
    F = W.random_forcing(cfg["seed"], cfg["n_omega"], cfg["k"], N)
    om = w0 + dw * np.arange(cfg["n_omega"])
    march(L, cfg["h"], om, F, 1, lambda s: True, lambda s: False, 1.0)
    steps, t = 0, time.perf_counter()
    while steps == 0 or time.perf_counter() - t < seconds:
        march(L, cfg["h"], om, F, 2, lambda s: True, lambda s: False, 1.0)
        steps += 2
    dt = time.perf_counter() - t
    return dict(value=N * cfg["k"] * cfg["n_omega"] * steps / dt, unit="resolvent sweeps/s", cores=oracle_threads(),
                kind="oracle", host=host_cpu(),
                sample="%d forced RK4 steps of the oracle on the %s grid (%d unknowns, k=%d, %d frequencies), %.1f s"
                       % (steps, "x".join(map(str, shape)), N, cfg["k"], cfg["n_omega"], dt))


def grad3d(cfg):
    """Forward plus reverse mode of the 3-D workload's gradient pattern on its full grid: one apply of the periodic
    method (all periods, 96 frequencies, k = 3) and one apply_backward with forcing and mu gradients, checkpoints
    every 64 steps, mixed precision (FP32 rows, FP64 arithmetic and accumulation; the mode runs the columns in
    chunks when the rows of all three do not fit beside the inputs).  With g = u / |u| (dJ/du_hat of
    J = sum |u_hat|) the duality <A^H g, f> = <g, A f> = J checks the forcing gradient at no extra cost."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2008_10904_amd.operators import snap_grid

    op = grid_op(cfg, cfg["precision"])
    N = 3 * cfg["nx"] * cfg["ny"] * cfg["nz"]
    nw, k = cfg["n_omega"], cfg["k"]
    w0, dw, P = snap_grid(cfg["wmin"], cfg["wmax"], nw, cfg["h"], cfg["stride"])
    f = W.random_forcing_device(cfg["seed"], nw, k, N, torch.complex64, "cuda")
    grid = op.grid(w0, dw, nw)
    run = op.run("periodic", periods=cfg["periods"], stride=cfg["stride"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = op.apply(f, grid, run)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress("gradient: forward apply done")
    J = sum(float(u[j].abs().to(torch.float64).sum().item()) for j in range(nw))
    g = torch.empty_like(u)
    for j in range(nw):  # dJ/du_hat of J = sum |u_hat|, one frequency at a time (no full-size temporaries)
        g[j] = u[j] / u[j].abs().clamp_min(1e-30)
    del u
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t1b = time.perf_counter()
    fg, mg = op.apply_backward(f, g, grid, run, checkpoint_every=cfg["checkpoint_every"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    progress("gradient: backward (forcing and mu) done")
    dual = sum(complex(torch.vdot(fg[j].flatten().to(torch.complex128), f[j].flatten().to(torch.complex128)).item())
               for j in range(nw))
    ok = bool(torch.isfinite(fg).all().item()) and bool(np.isfinite(mg.cpu().numpy()).all())
    del fg, mg
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    op.apply_backward(f, g, grid, run, checkpoint_every=cfg["checkpoint_every"], want_mu=False)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    return {"grid": [cfg["nx"], cfg["ny"], cfg["nz"]], "n_omega": nw, "k": k, "P": P,
            "time_steps": cfg["periods"] * P, "checkpoint_every": cfg["checkpoint_every"], "rows": "fp32",
            "forward_s": t1 - t0, "backward_s": t2 - t1b, "backward_forcing_only_s": t4 - t3, "finite": ok,
            "duality_rel": abs(dual - J) / J,
            "note": "one apply and one apply_backward (forcing and mu gradients), periodic method, full grid"}


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
    replay = graph_replay(op, f, grid, run, 50)
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
        "graph_replay": replay,
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
    if args.workload == "gl_transient_n200":
        bench_transient(args)
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
                     "traffic": measured_traffic(plan64, power, steps_per_launch), "avg_launch_ms": avg_launch_s * 1e3,
                     "launches": stepper_n,
                     "steps_per_launch": steps_per_launch},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
        "stepper_plan": list(plan64),
        "step_power": power,
    }
    out["roofline"]["ns_per_rk4_step"] = avg_launch_s / steps_per_launch * 1e9
    floor = latency_floor(cfg, power)
    floor["headline_over_floor"] = out["roofline"]["ns_per_rk4_step"] / floor["ns_per_rk4_step"]
    out["roofline"]["latency_floor"] = floor
    if weights is not None:
        out["config"]["weights"] = ("B: window over the upstream 60 %, C: window over the downstream 60 %, "
                                    "W_f = W_y = dx (gains of C R B in the W norms)")
    iters = cfg["iters"] if args.accuracy_iters is None else args.accuracy_iters
    js = [0, 101, 128, 255]  # both band edges, an inner frequency and the centre (omega ~ 0)
    sampled = {}
    if iters > 0:
        sampled["fp64"] = gpu_modes_sampled(op, f64, grid, run, iters, js)
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
                        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in ktm.items()},
                        "stepper_plan": list(planm)}
        if iters > 0:
            sampled["mixed"] = gpu_modes_sampled(opm, f32, grid, run, iters, js)
        del opm, f32
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, w0, dw, F, args.cpu_seconds)
        if sampled and weights is None:
            out["accuracy_vs_oracle"] = headline_accuracy(cfg, w0, dw, F, js, iters, sampled)
    print(json.dumps(out), flush=True)


def latency_floor(cfg, step_power):
    """The 1-D stepper's dependent-step latency without neighbour exchange: a column of 256 unknowns of the same GL
    family (one workgroup per column: no halo, no exchange), k = 4, the same step power and precision (FP64),
    marched through one forced period of P = 65,536 steps with 16 frequencies.  Returns ns per RK4 step of the
    stepper launches (HIP events on the library's stream).  The headline march differs from it by the neighbour
    exchange and the halo's redundant work, so the ratio of the two says how far the stepper is from its own
    latency bound."""
    import numpy as np
    import torch
    from paper_2008_10904_amd import ResolventOp
    from paper_2008_10904_amd import _lib as L
    from paper_2008_10904_amd.operators import gl_coefficients
    n, P, nw = 256, 65536, 16
    lo, d, up = gl_coefficients(n, cfg["mu0"], cfg["mu2"])
    op = ResolventOp.tridiagonal(lo, d, up, cfg["h"], precision="fp64")
    op.set_step_power(step_power)
    grid = op.grid(-1.0, 2 * np.pi / (P * cfg["h"]), nw)
    run = op.run("periodic", periods=1, stride=P // nw)
    f = torch.ones((nw, cfg["k"], n), dtype=torch.complex128, device="cuda")
    op.apply(f, grid, run)  # warm-up
    torch.cuda.synchronize()
    op.set_timing(True)
    op.timing(L.RES_TIMING_STEPPER)
    op.apply(f, grid, run)
    ms, launches = op.timing(L.RES_TIMING_STEPPER)
    op.set_timing(False)
    return {"ns_per_rk4_step": ms * 1e6 / P, "unknowns": n, "k": cfg["k"], "step_power": step_power,
            "note": "one workgroup per column, no neighbour exchange: the latency of the dependent step chain"}


def headline_accuracy(cfg, w0, dw, F, js, iters, sampled):
    """Gains and modes of the GPU iterations at the sampled frequencies against the oracle's same iteration (FP64;
    the mixed path's oracle starts from the complex64-rounded forcing it was given)."""
    import numpy as np
    from oracle import operators as O_ops
    L, _ = O_ops.gl_operator(cfg["N"], cfg["mu0"], cfg["mu2"])
    om = w0 + dw * np.asarray(js)
    t = time.perf_counter()
    out = {"iterations": iters, "sampled_omega_index": list(js), "sampled_omega": [float(w) for w in om]}
    for prec, (g, V, U) in sampled.items():
        F_sel = F[js] if prec == "fp64" else F[js].astype(np.complex64).astype(np.complex128)
        g_ref, V_ref, U_ref = oracle_sampled_reference(L, cfg["h"], om, F_sel, iters)
        out[prec] = accuracy(g, V, U, g_ref, V_ref, U_ref, [int(j) for j in js])
    out["oracle_seconds"] = time.perf_counter() - t
    out["targets"] = {"fp64_gain": 1e-8, "mixed_gain": 1e-4}
    return out


if __name__ == "__main__":
    main()
