"""Host-side logic that needs no GPU: the serving loop's arena allocator, staging packer and
admission / step-launch policy, built with g++ (and with the address and
undefined-behaviour sanitizers when available)."""
import shutil
import subprocess
from pathlib import Path

import pytest

HERE = Path(__file__).resolve().parent


@pytest.mark.parametrize("sanitize", [False, True])
def test_arena_allocator(tmp_path, sanitize):
    exe = tmp_path / "arena_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", str(HERE / "cpp" / "arena_check.cpp"), "-o", str(exe)]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and sanitize:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "arena ok" in out.stdout


@pytest.mark.parametrize("sanitize", [False, True])
def test_stage_group_packing(tmp_path, sanitize):
    """The serving loop's staging packer puts every message byte of a group at its arena
    position, across alignment gaps, empty messages, requests without payload and any
    piece size, and never writes past a piece."""
    exe = tmp_path / "stage_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", str(HERE / "cpp" / "stage_check.cpp"), "-o", str(exe)]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and sanitize:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "stage ok" in out.stdout


@pytest.mark.parametrize("sanitize", [False, True])
def test_serving_policy(tmp_path, sanitize):
    """The serving loop's admission (arrival order, budget, slots) and step-launch
    decisions (per class, one step per class, cross-class takeover only when that class's
    streams are all busy), under a simulated clock with simulated streams: every decision
    keeps the rules and every request of random open-loop workloads completes."""
    exe = tmp_path / "policy_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", str(HERE / "cpp" / "policy_check.cpp"), "-o", str(exe)]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and sanitize:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "policy ok" in out.stdout
