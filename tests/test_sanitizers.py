"""The oracle and the library's host code (argument validation, handles,
workspace carving) under AddressSanitizer and UndefinedBehaviorSanitizer:
the oracle's pins and the C-ABI tests run in subprocesses that load
sanitizer builds (tests/sanitized_build.py), and any report fails the test
(halt_on_error).  CPU only."""
import os
import subprocess
import sys

import pytest

import sanitized_build as SB

ROOT = SB.ROOT
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(env_extra, args):
    env = dict(os.environ)
    env.update(ENV_SAN)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider", *args],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:] + r.stderr[-3000:])
    assert "runtime error" not in r.stdout + r.stderr and "ERROR: AddressSanitizer" not in r.stdout + r.stderr


def test_oracle_under_sanitizers():
    lib = SB.build_oracle()
    _run({"LBMX_ORACLE_LIB": lib, "LD_PRELOAD": SB.gcc_runtime(), "OMP_NUM_THREADS": "2"},
         ["tests/test_oracle_lattice.py", "tests/test_oracle_equilibrium.py", "tests/test_oracle_step.py",
          "tests/test_oracle_fd.py", "-k", "not slow"])


def test_library_host_code_under_sanitizers():
    if not os.path.exists(os.path.join(ROOT, "paper_1606_06107_amd", "liblbmx.so")):
        pytest.skip("liblbmx.so not built")
    lib = SB.build_library()
    _run({"LBMX_LIB": lib, "LD_PRELOAD": SB.clang_runtime()},
         ["tests/test_abi.py", "-k", "not rollout_refuses"])
