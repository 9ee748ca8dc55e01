"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc) and run on small seeded volumes through every entry point: it must exit
cleanly (no out-of-bounds access, leak, overflow or other undefined
behaviour is reported)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    srcs = [os.path.join(HERE, "oracle_sanitize.c"), os.path.join(ROOT, "oracle", "lsrvt_oracle.c"),
            os.path.join(ROOT, "oracle", "los_oracle.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe, *srcs, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in (r.stderr or ""):
        pytest.skip(f"sanitizer runtime unavailable: {r.stderr.strip()[:200]}")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "oracle sanitizer run ok" in run.stdout
    assert "runtime error" not in run.stderr
