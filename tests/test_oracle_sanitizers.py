"""The FP64 oracle under the host AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_check.c builds a 3-level tree of a small synthetic cloud and
runs the E-step and registration of the adaptive descent, the single-level
mixture and the soft multi-path descent with every optional output requested.
Compiled here with gcc, ``-fsanitize=address,undefined`` and no recovery, any
out-of-bounds access, leak or undefined behaviour in the oracle's C code ends
the run with a non-zero status.  CPU only; skipped when gcc or the sanitizer
runtimes are missing.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "sanitize_check")
    cmd = [gcc, "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", ORACLE, os.path.join(ORACLE, "sanitize_check.c"),
           os.path.join(ORACLE, "hgmm_oracle.c"), "-lm", "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0:
        if "asan" in build.stderr.lower() or "ubsan" in build.stderr.lower() or "sanitize" in build.stderr.lower():
            pytest.skip("sanitizer runtimes not available: " + build.stderr.strip()[-200:])
        raise AssertionError(build.stderr)
    # verify_asan_link_order=0: the sanitizer runtime need not come first
    # among the libraries the environment preloads
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "sanitize_check: ok" in run.stdout
