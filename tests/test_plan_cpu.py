"""Workspace planner checked on the host (no device): builds tests/cpp/plan_check.cpp
against the host runtime with stub kernel launchers, under AddressSanitizer."""
import os
import subprocess

import pytest

from tests.conftest import ROOT

CSRC = os.path.join(ROOT, "paper_2406_06488_amd", "csrc")


def test_workspace_plan_invariants(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = ["/opt/rocm/bin/hipcc", "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "cpp", "plan_check.cpp"), os.path.join(CSRC, "runtime.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("build failed:\n" + r.stderr[-4000:])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stdout[-4000:] + out.stderr[-4000:]
    assert out.stdout.strip().startswith("ok")
