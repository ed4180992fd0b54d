"""The serving loop's admission policy (admit_decide, a pure host function)
checked on the CPU: workspace reuse, release of idle workspaces, waiting for
running solves, and random request streams that must always drain within the
HBM budget."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1011_3318_amd", "csrc")


def test_admission_policy(tmp_path):
    exe = str(tmp_path / "admit_driver")
    r = subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", f"-I{CSRC}", "-o", exe,
                        os.path.join(HERE, "admit_driver.cpp")], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stdout + r.stderr)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    for name in ("no-idle-slot", "reuse", "keep", "idle-release", "wait-for-running", "random-streams"):
        assert f"ok {name}" in out.stdout
