"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): a small C
driver (tests/sanitize/oracle_driver.c) compiles the oracle source in and calls every entry
point on ragged lattices, periodic and with walls (force, moving and wetting walls), in the
three collision modes.  Any sanitizer report aborts the program."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    src = os.path.join(HERE, "sanitize", "oracle_driver.c")
    subprocess.run([gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-static-libasan", "-std=c11", "-Wall", src, "-lm", "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle driver: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
