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


@pytest.mark.parametrize("sanitize", [False, True])
def test_plan_long_chain_regions(tmp_path, sanitize):
    """Host model of the batched plan's long-chain scratch assignment, using the plan's own
    sizing rules (hb_plan_rules.hpp): with block-count keys saturated above about 1.05 MB,
    a wave's region must come from its longest lane, not its first.  The model shows the
    first-lane rule reading past its region on a 1.5 MiB message ordered ahead of a 3 MiB
    one, and that the rule in use never does over random bucketed orders."""
    exe = tmp_path / "plan_region_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", str(HERE / "cpp" / "plan_region_check.cpp"), "-o", str(exe)]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and sanitize:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "plan region ok" in out.stdout


@pytest.mark.parametrize("sanitize", [False, True])
def test_resident_item_formation(tmp_path, sanitize):
    """The resident serving mode's slot layout and work items (hb_items.hpp) over 3,000
    random requests (0 to 12,000 messages, log-normal lengths around 256 B, 8 KiB and 40 KB,
    some up to 16 MiB, one or mixed algorithms), in both formations: slots a permutation
    ordered by algorithm and block-count class; items covering every slot once with their
    longest message's block count; the latency formation taking exactly each algorithm's
    two longest classes of >= 128 blocks into items of at most four, evenly sized."""
    exe = tmp_path / "items_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", str(HERE / "cpp" / "items_check.cpp"), "-o", str(exe)]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and sanitize:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "items ok" in out.stdout


@pytest.mark.parametrize("sanitize", [False, True])
def test_request_failure_text_reaches_the_caller(tmp_path, sanitize):
    """A serving request failed on a staging thread or the loop carries its explanation to
    the thread that waits for it (hb_outcome.hpp, used by hb_server_wait / hb_server_poll):
    the waiter's per-thread error text is the failure's, other threads' are untouched, and
    the first failure wins."""
    exe = tmp_path / "outcome_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", str(HERE / "cpp" / "outcome_check.cpp"), "-o", str(exe)]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and sanitize:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "outcome ok" in out.stdout


@pytest.mark.parametrize("sanitize", [False, True])
def test_host_hashing_code_under_sanitizers(tmp_path, sanitize):
    """The CPU oracle (oracle/hash_oracle.c) and the library's host share of a CPU + GPU
    split (csrc/hb_cpu.cpp) built with the address and undefined-behaviour sanitizers:
    every length 0..300 and 1 MiB-class messages, each in an exact-size heap buffer, all
    three algorithms, with the two codes agreeing on every digest."""
    root = HERE.parent
    flags = ["-O1", "-g"] + (["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                              "-fno-sanitize-recover=undefined"] if sanitize else [])
    obj = tmp_path / "hash_oracle.o"
    r = subprocess.run(["gcc", "-std=c11", *flags, "-c", str(root / "oracle" / "hash_oracle.c"), "-o", str(obj)],
                       capture_output=True, text=True)
    if r.returncode != 0 and sanitize:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    exe = tmp_path / "hash_sanitize_check"
    cmd = ["g++", "-std=c++17", *flags, "-pthread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           str(HERE / "cpp" / "hash_sanitize_check.cpp"), str(root / "paper_2407_09333_amd" / "csrc" / "hb_cpu.cpp"),
           str(obj), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "sanitized hashing ok" in out.stdout


CLANG = Path("/opt/rocm/llvm/bin/clang++")


@pytest.fixture(scope="module")
def server_check_exe(tmp_path_factory):
    """The serving-loop check built once per sanitizer (see the test below)."""
    if not CLANG.exists():
        pytest.skip("clang++ with sanitizer runtimes not found")
    built = {}

    def get(sanitize):
        if sanitize not in built:
            exe = tmp_path_factory.mktemp("server_check") / "server_check"
            cpp = HERE / "cpp"
            cmd = [str(CLANG), "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}", "-fno-omit-frame-pointer",
                   "-I", str(cpp / "fakehip"), "-I", str(HERE.parent / "include"), str(cpp / "server_check.cpp"),
                   str(cpp / "fakehip" / "fake_hip.cpp"),
                   str(HERE.parent / "paper_2407_09333_amd" / "csrc" / "hb_server.cpp"), "-o", str(exe), "-lpthread"]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr
            built[sanitize] = exe
        return built[sanitize]

    return get


@pytest.mark.parametrize("env", [{}, {"GPU_MAX_HW_QUEUES": "8"}, {"HB_SERVER_COPY": "kernel"},
                                 {"HB_SERVER_STAGERS": "1"}, {"HB_SERVER_MODE": "resident"},
                                 {"HB_SERVER_MODE": "resident", "GPU_MAX_HW_QUEUES": "8"}],
                         ids=["default", "8queues", "kernelcopy", "1stager", "resident", "resident8queues"])
@pytest.mark.parametrize("sanitize", ["thread", "address,undefined"], ids=["tsan", "asan"])
def test_serving_loop_on_host_stand_in(server_check_exe, sanitize, env):
    """The serving loop itself (csrc/hb_server.cpp, compiled unchanged) on the CPU against a
    host-only stand-in for the HIP runtime (tests/cpp/fakehip: in-order streams on host
    threads, events, stream waits, copies) and for the plan's hashing (a per-message
    fingerprint), under ThreadSanitizer and under AddressSanitizer + UBSan: three client
    threads submit, cancel and wait on 180 requests against a 2 MiB budget, with device steps
    or (resident mode) the resident serving kernel's item protocol emulated on a host
    thread; every request's
    slots hold its own messages' fingerprints, and no event is destroyed or recorded again
    while in flight, no stream waits on an event never recorded, no destroyed stream or
    event is used, and every event created is destroyed.  Clang's sanitizers are used:
    GCC 11's ThreadSanitizer does not follow condition-variable waits on the steady clock."""
    import os

    exe = server_check_exe(sanitize)
    run_env = dict(os.environ, **env, TSAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    out = subprocess.run([str(exe), "60"], capture_output=True, text=True, timeout=300, env=run_env)
    assert out.returncode == 0, out.stdout + out.stderr[-4000:]
    assert "server ok" in out.stdout
    assert "WARNING: ThreadSanitizer" not in out.stderr, out.stderr[-4000:]
