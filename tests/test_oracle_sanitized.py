"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc) and driven through a short discharge that reaches every branch of the
step (walls with reflection and emission, all collision processes, births,
sorts, time averages, electrode histograms, field solvers, the profile
loader): any out-of-bounds access, use after free, signed overflow or
other undefined behaviour aborts the run."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    src = [os.path.join(HERE, "csrc", "oracle_sanitize_main.c"),
           os.path.join(ROOT, "oracle", "philox.c"), os.path.join(ROOT, "oracle", "warm_oracle.c")]
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", str(exe), *src, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtimes not installed")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
    fields = run.stdout.split()
    vals = dict(zip(fields[::2], (int(v) for v in fields[1::2])))
    assert vals["steps"] == 60 and vals["hits"] > 0 and vals["collisions"] > 0 and vals["ionizations"] > 0
