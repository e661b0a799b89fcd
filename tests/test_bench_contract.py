"""bench.py's contract on the CPU: a request for several GPUs stops with a
message before anything touches a GPU, and the HBM-traffic constants the
roofline line carries are the figures the committed rocprofv3 summaries
state (so that neither can change without the other)."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_several_gpus_are_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _bold_bytes(name):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    m = re.search(r"\*\*([0-9.]+) bytes per electron particle-step\*\*", text)
    assert m, name
    return float(m.group(1)), text


def test_traffic_constants_match_the_profiles():
    b = _bench_module()
    first, _ = _bold_bytes("particle_pass_c3_first_steps_hbm_traffic.md")
    cycles, text = _bold_bytes("particle_pass_c3_large_lowp_hbm_traffic.md")
    assert b.PASS_TRAFFIC_BYTES_PER_PARTICLE == first
    assert abs(cycles - first) <= 0.2
    assert f"{b.PASS_TRAFFIC_BYTES_UNPIPELINED} bytes per electron particle-step" in " ".join(text.split())
    # the label names the profiles the constant comes from
    assert "particle_pass_c3_first_steps_hbm_traffic.md" in b.PASS_TRAFFIC_SOURCE


def test_profiles_name_only_committed_commands():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert "_work" not in text, name
        for cmd in re.findall(r"^    (rocprofv3 .*|python3? .*)$", text, re.M):
            assert "_work" not in cmd
