"""The served form's host scheduler core (csrc/sfsched.cpp) on the CPU:
queued admission under a tight HBM budget with small rings, claim classes,
resident block keys (continue, write back, fetch, release) and the error
cases, against a simulated device (tests/sched_sim.cpp) that predicts every
result exactly and checks arena exclusivity, ring-slot reuse and
publication order at each step.  Built with g++ and the host sanitizers."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_21438_amd", "csrc")


def test_scheduler_core_against_simulated_device(tmp_path):
    exe = str(tmp_path / "sched_sim")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I" + CSRC, os.path.join(ROOT, "tests", "sched_sim.cpp"),
                           os.path.join(CSRC, "sfsched.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    print(r.stderr)
    assert r.returncode == 0, r.stderr
    assert "ALL PASS" in r.stdout
