"""Persistent cache of tuned stepper plans.

``tuned(op, k)`` applies the plan stored for this problem (device, operator size and batch layout, column count,
precision) if the cache holds one, and otherwise runs the library's autotuner (``ResolventOp.tune``) and stores
its choice.  The cache is a JSON file: ``$RESOLVENT_PLAN_CACHE`` if set, else
``~/.cache/resolvent/stepper_plans.json``.  Plans only change how the march is laid out on the device; results
are bit for bit the same under every plan.
"""
import json
import os


def cache_path():
    return os.environ.get("RESOLVENT_PLAN_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "resolvent",
                                                                  "stepper_plans.json")


def problem_key(device, op, k):
    offsets = list(getattr(op, "offsets", [0, op.n]))
    sizes = sorted({int(b) - int(a) for a, b in zip(offsets[:-1], offsets[1:])})
    return "%s|N=%d|inst=%d|sizes=%s|k=%d|%s" % (device, op.n, len(offsets) - 1, ",".join(map(str, sizes)), k,
                                                 op.precision)


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


def tuned(op, k, steps=2048, device=None, path=None, retune=False):
    """Apply the cached plan for (op, k) or tune and cache one; returns (plan, us per step or None if cached)."""
    if device is None:
        import torch
        device = torch.cuda.get_device_name()
    key = problem_key(device, op, k)
    entries = load(path)
    if not retune and key in entries:
        return op.set_plan(entries[key]["plan"]), None
    plan, us = op.tune(k, steps)
    entries[key] = {"plan": list(plan), "us_per_step": us, "steps": steps}
    save(entries, path)
    return plan, us
