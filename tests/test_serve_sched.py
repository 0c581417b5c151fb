"""The serving loop's admission and batching policy, on the CPU: the policy
header is compiled with g++ into a small check program (tests/native/)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_scheduler_policy(tmp_path):
    exe = str(tmp_path / "sched_check")
    src = os.path.join(HERE, "native", "sched_check.cpp")
    inc = os.path.join(ROOT, "paper_2506_19693_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", inc, src, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
