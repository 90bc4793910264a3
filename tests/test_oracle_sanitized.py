"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host only).

Compiles ``oracle/gotoh.c`` with a small driver (``tests/sanitize_oracle.c``)
that calls every oracle entry point on seeded random DNA and protein inputs
(threads, odd stripe and chunk sizes, empty sequences, invalid arguments), and
runs it: any out-of-bounds access, use after free, leak or
undefined arithmetic ends the run with a sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-O1", "-g", "-std=c11", "-pthread", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    build = subprocess.run(["gcc", *flags, "-o", exe, os.path.join(ROOT, "oracle", "gotoh.c"),
                            os.path.join(HERE, "sanitize_oracle.c")], capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtime not installed")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "clean" in run.stdout
