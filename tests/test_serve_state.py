"""The gridding server's job state transitions, on the CPU: a running job
completes, stays running while its event is not ready, and fails (releasing
its footprint, counted once) when the device reports an error for its work.
Builds tests/serve_state_check.cpp with g++ against the server's host-only
state header and runs it."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_serve_state_transitions(tmp_path):
    exe = tmp_path / "serve_state_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2111_04141_amd", "csrc"),
                    os.path.join(ROOT, "tests", "serve_state_check.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "serve_state ok" in r.stdout
