"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): every exported routine runs on small grids with solids, walls, a
pressure axis, a force, all velocity sets, collisions and closures, and no
sanitizer report may appear."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_address_and_ub_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitize")
        cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer", "-Wno-unknown-pragmas",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               os.path.join(HERE, "oracle_sanitize.c"), "-o", exe, "-lm"]
        b = subprocess.run(cmd, capture_output=True, text=True)
        if b.returncode != 0 and "asan" in b.stderr.lower():
            pytest.skip("sanitizer runtime not installed")
        assert b.returncode == 0, b.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
        env.pop("LD_PRELOAD", None)
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-4000:])
        assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
