"""Persistent cache of tuned stepper plans.

``tuned(op, k)`` applies the plan stored for this problem (device, operator size and batch layout, column count,
precision, step power) if the cache holds one, and otherwise runs the library's autotuner (``ResolventOp.tune``)
and stores its choice.  The cache is a JSON file: ``$RESOLVENT_PLAN_CACHE`` if set, else
``~/.cache/resolvent/stepper_plans.json``.  Plans only change how the march is laid out on the device; results
are bit for bit the same under every plan.  ``tuned(op, k, powers=(4, 2, 1))`` also chooses the step power (RK4
steps per kernel step) among those given; the power changes results at the rounding level only.
"""
import json
import os


def cache_path():
    return os.environ.get("RESOLVENT_PLAN_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "resolvent",
                                                                  "stepper_plans.json")


def problem_key(device, op, k, powers=None):
    offsets = list(getattr(op, "offsets", [0, op.n]))
    sizes = sorted({int(b) - int(a) for a, b in zip(offsets[:-1], offsets[1:])})
    key = "%s|N=%d|inst=%d|sizes=%s|k=%d|%s" % (device, op.n, len(offsets) - 1, ",".join(map(str, sizes)), k,
                                                op.precision)
    if powers is not None:
        return key + "|m in " + ",".join(str(int(m)) for m in powers)
    m = op.get_step_power() if hasattr(op, "get_step_power") else 1
    return key if m == 1 else key + "|m=%d" % m


def load(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save(entries, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(op, k, steps=2048, device=None, path=None, retune=False, powers=None):
    """Apply the cached plan for (op, k) or tune and cache one; returns (plan, us per step or None if cached).
    With powers (a sequence of step powers) the plan is tuned at each and the fastest (power, plan) is kept."""
    if device is None:
        import torch
        device = torch.cuda.get_device_name()
    key = problem_key(device, op, k, powers)
    entries = load(path)
    if not retune and key in entries:
        if powers is not None:
            op.set_step_power(entries[key]["step_power"])
        return op.set_plan(entries[key]["plan"]), None
    best = None
    for m in (powers if powers is not None else [None]):
        if m is not None:
            op.set_step_power(m)
        plan, us = op.tune(k, steps)
        if best is None or us < best[2]:
            best = (m, plan, us)
    m, plan, us = best
    if m is not None:
        op.set_step_power(m)
        plan = op.set_plan(plan)
    entries[key] = {"plan": list(plan), "us_per_step": us, "steps": steps}
    if m is not None:
        entries[key]["step_power"] = int(m)
    save(entries, path)
    return plan, us
