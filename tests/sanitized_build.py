"""Builds of the oracle and of the library's host code with AddressSanitizer
and UndefinedBehaviorSanitizer, for the CPU check in test_sanitizers.py.

Only host code is instrumented: the oracle (plain C, gcc) and the host side
of the HIP translation units that validate arguments and manage handles
(api, batch, surrogate, probe; hipcc with each sanitizer flag behind
-Xarch_host, so device code is compiled as usual).  The step kernels' objects
of the regular build (_build/) are linked in unchanged.  GPU code is never
built with a sanitizer."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1606_06107_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitized")
HOST_TUS = ("api", "batch", "surrogate", "probe")
SAN = ["address", "undefined"]


def gcc_runtime():
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def clang_runtime():
    clang = "/opt/rocm/llvm/bin/clang"
    return subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()


def build_oracle():
    os.makedirs(OUT, exist_ok=True)
    out = os.path.join(OUT, "liboracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c99", "-fPIC", "-shared", "-fopenmp"]
    cmd += [f"-fsanitize={s}" for s in SAN]
    cmd += [os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-o", out, "-lm"]
    subprocess.check_call(cmd)
    return out


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _host_flags():
    flags = []
    for s in SAN:
        flags += ["-Xarch_host", f"-fsanitize={s}"]
    return flags


def build_library():
    """liblbmx with sanitized host code; needs the regular build's objects."""
    os.makedirs(OUT, exist_ok=True)
    reg = os.path.join(ROOT, "_build")
    base = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=on",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC] + _host_flags()

    def comp(tu):
        obj = os.path.join(OUT, tu + ".o")
        r = subprocess.run([_hipcc(), *base, "-c", os.path.join(CSRC, tu + ".hip"), "-o", obj],
                           capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(r.stderr[-4000:])
        return obj

    with cf.ThreadPoolExecutor(len(HOST_TUS)) as ex:
        objs = list(ex.map(comp, HOST_TUS))
    others = [o for o in sorted(glob.glob(os.path.join(reg, "*.hip.o")))
              if os.path.basename(o)[:-len(".hip.o")] not in HOST_TUS]
    if not others:
        raise RuntimeError("the regular build's objects are missing (run the library build first)")
    out = os.path.join(OUT, "liblbmx_san.so")
    r = subprocess.run([_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *_host_flags(), *others, *objs,
                        "-o", out], capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr[-4000:])
    return out
