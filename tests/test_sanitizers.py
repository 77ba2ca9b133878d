"""The CPU suites that exercise compiled host code, rerun against builds
with AddressSanitizer and UndefinedBehaviorSanitizer:

- the library's host code (planner, schedule strings, plan description,
  argument validation, gate lists and pass plans, tridiagonal routines;
  tests/test_host_logic.py) built with clang's sanitizers on the host side
  and linked with the regular device objects;
- the oracle's C core (tests/test_oracle.py, without the slow test) built
  with gcc's sanitizers.

Each suite runs in a child process with the matching runtime preloaded; any
sanitizer report aborts it.  No GPU is touched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(env_extra, args):
    env = dict(os.environ)
    env.update(ENV_SAN)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *args],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail


def test_host_library_under_asan_ubsan():
    from paper_2108_13410_amd import build as b
    if not all(os.path.exists(os.path.join(b.BUILD, os.path.splitext(s)[0] + ".o")) for s in b.DEVICE_SOURCES):
        b.build()
    lib = b.build_sanitized()
    _run({"LD_PRELOAD": b.sanitizer_runtime(), "Z2H_LIB": lib},
         ["tests/test_host_logic.py", "-m", "not gpu"])


def test_oracle_core_under_asan_ubsan():
    from oracle import build as ob
    out_dir = os.path.join(ROOT, "_build", "sanitize")
    os.makedirs(out_dir, exist_ok=True)
    lib = ob.build(sanitize=True, out=os.path.join(out_dir, "liboracle.so"))
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    asan = r.stdout.strip()
    if not os.path.isabs(asan):
        pytest.fail("gcc's libasan.so not found")
    _run({"LD_PRELOAD": asan, "Z2H_ORACLE_LIB": lib, "OMP_NUM_THREADS": "4"},
         ["tests/test_oracle.py", "-m", "not slow"])
