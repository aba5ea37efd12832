"""Builds libresolvent.so (HIP for gfx950) in-tree with hipcc.  Usage: python -m paper_2008_10904_amd.build"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libresolvent.so")
SOURCES = ["step1d.hip", "step1d_m2.hip", "step1d_m4.hip", "stencil.hip", "phase_gemm.hip", "qr.hip", "krylov.hip", "adjoint.hip",
           "trm.hip", "noalloc.hip", "runtime.cpp", "runs.cpp", "iterations.cpp", "backward.cpp", "trm_host.cpp"]
HOST_SOURCES = [s for s in SOURCES if s.endswith(".cpp")]  # the host runtime
EXPORTS = os.path.join(CSRC, "exports.map")  # the library exports the C ABI only
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("RESOLVENT_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# hand-written kernels never rely on packed FP32 instructions
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    cmd = [HIPCC] + COMMON + DEVICE + ["-c", path, "-o", obj]
    if src.endswith(".cpp"):  # host-only code: one device target keeps hipcc from building the default one
        cmd = [HIPCC] + COMMON + ["--offload-arch=" + ARCH, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=True):
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-Wl,--version-script=" + EXPORTS, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Host sanitizer build: the runtime and the ABI driver of tests/host_sanitize with AddressSanitizer and
# UndefinedBehaviorSanitizer on the host code only (device code is never sanitized), linked with the device objects
# of the last build().
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-gpu-sanitize",
            "-fno-sanitize-recover=undefined"]
ABI_CHECK_SRC = os.path.join(ROOT, "tests", "host_sanitize", "abi_check.cpp")
ABI_CHECK = os.path.join(HERE, "abi_check_asan")  # beside the library (the object folder stays on this host)


def build_abi_check(verbose=True):
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    for src in [os.path.join(CSRC, h) for h in HOST_SOURCES] + [ABI_CHECK_SRC]:
        obj = os.path.join(OBJ, os.path.basename(src) + ".asan.o")
        cmd = [HIPCC, "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
               "--offload-arch=" + ARCH] + SANITIZE + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
        objs.append(obj)
    kernels = [os.path.join(OBJ, s + ".o") for s in SOURCES if s.endswith(".hip")]
    missing = [k for k in kernels if not os.path.exists(k)]
    if missing:
        raise RuntimeError("run build() first: missing %s" % ", ".join(missing))
    cmd = [HIPCC, "--offload-arch=" + ARCH] + SANITIZE + ["-o", ABI_CHECK] + objs + kernels
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    if verbose:
        print("built", ABI_CHECK)
    return ABI_CHECK


if __name__ == "__main__":
    build()
    if "--abi-check" in sys.argv:
        build_abi_check()
    sys.exit(0)
