"""The C ABI under AddressSanitizer and UndefinedBehaviorSanitizer on the host code.

`paper_2008_10904_amd/build.py` (`build_abi_check`, run by `__graft_entry__.build()`) compiles the runtime and the
driver `tests/host_sanitize/abi_check.cpp` with both sanitizers on the host side only and links them with the
device objects of the library build.  The host part (argument checking, error strings, the FIR design) runs here;
the GPU part runs every entry point once on small operators of each kind and precision (tridiagonal, weighted,
2-D and 3-D grids; FP64 and mixed).  A sanitizer report or an unexpected status fails the test.  Leaks inside the
HIP and HSA runtimes' own state are suppressed (`tests/host_sanitize/lsan.supp`); leaks anywhere else are
reported.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SUPP = os.path.join(HERE, "host_sanitize", "lsan.supp")


def driver():
    from paper_2008_10904_amd import build as B
    if not os.path.exists(B.ABI_CHECK):
        if not all(os.path.exists(os.path.join(B.OBJ, s + ".o")) for s in B.SOURCES):
            B.build(verbose=False)
        B.build_abi_check(verbose=False)
    return B.ABI_CHECK


def run(args, timeout):
    env = dict(os.environ, LSAN_OPTIONS="suppressions=" + SUPP, ASAN_OPTIONS="halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver()] + args, capture_output=True, text=True, timeout=timeout, env=env, cwd=ROOT)
    out = r.stdout + r.stderr
    print(out[-4000:])
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out
    assert "runtime error:" not in out  # UBSan
    assert r.returncode == 0, out[-2000:]
    return out


def test_host_part_under_sanitizers():
    out = run([], 120)
    assert "host part: 0 failure(s)" in out


@pytest.mark.gpu
def test_every_entry_point_under_host_sanitizers():
    """The driver runs in a process of its own beside this one, which may already hold device memory and the
    device's cooperative-launch resources from earlier tests: the library then marches without persistent
    launches (it falls back to a relaunch at every exchange when the device refuses one)."""
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()
    print("case: sanitized ABI driver, GPU part", flush=True)
    out = run(["--gpu"], 300)
    assert "host and GPU parts: 0 failure(s)" in out
