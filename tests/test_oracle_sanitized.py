"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): a driver runs every oracle entry point on small problems,
an empty column, an empty matrix, one row and one live column."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    flags = ["-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run(["gcc"] + flags + ["-o", str(exe), os.path.join(ROOT, "oracle", "sanitize_main.c"),
                                      "-lm"], check=True, cwd=os.path.join(ROOT, "oracle"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout, r.stderr[-4000:])
    assert r.stdout.strip().endswith("ok")
