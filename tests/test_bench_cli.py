"""The bench's command-line contract on the CPU: refusals that must happen before any GPU work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = run("--gpus", "2")
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_options_tied_to_one_workload_are_refused_elsewhere():
    p = run("--weighted", "--workload", "adr2d_1024x512")
    assert p.returncode == 2 and "--weighted" in p.stderr
    p = run("--algorithm", "trm")
    assert p.returncode == 2 and "gl_paper_n200" in p.stderr
    p = run("--algorithm", "krylov", "--workload", "gl_paper_n200")
    assert p.returncode == 2 and "gl_periodic_n2000" in p.stderr
