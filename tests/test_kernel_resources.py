"""The plain kernels' register budgets, read from the gfx950 code object's metadata that
hipcc emits for hb_kernels.hip: no spills or private memory, and the LDS-staged kernels
within the register count that gives them the occupancy they are built for (MD5 five waves
per SIMD, SHA-1 five, SM3 four; the per-lane SHA-1 kernel eight).  A change that pushed a
kernel past its budget would slow it silently; this catches it on the CPU."""
import re
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# kernel symbol -> largest VGPR count that keeps its occupancy (512 VGPRs per SIMD lane,
# allocated in granules of 8)
BUDGETS = {
    "_ZN2hb11k_plain_ldsILi0EEEvPKhmmPh": 96,   # MD5: five waves per SIMD
    "_ZN2hb11k_plain_ldsILi1EEEvPKhmmPh": 96,   # SHA-1: five (the LDS holds five waves)
    "_ZN2hb11k_plain_ldsILi2EEEvPKhmmPh": 128,  # SM3: four
    "_ZN2hb7k_plainILi1ELb1EEEvPKhPKmS4_mmPhjS2_": 64,  # SHA-1 per lane: eight
}


@pytest.fixture(scope="module")
def metadata():
    if not Path(HIPCC).exists():
        pytest.skip("hipcc not available")
    cmd = [HIPCC, "-O3", "-std=c++17", f"-I{ROOT / 'include'}", "--offload-arch=gfx950", "--offload-device-only",
           "-S", "-x", "hip", str(ROOT / "paper_2407_09333_amd" / "csrc" / "hb_kernels.hip"), "-o", "-",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels = {}
    for block in re.split(r"\n  - \.", r.stdout)[1:]:  # one kernel per item of .amdhsa.kernels
        m = re.search(r"^    \.name:\s+(\S+)", block, re.M)  # the kernel's own fields: four spaces in
        if not m:
            continue
        fields = dict(re.findall(r"^    \.(vgpr_count|vgpr_spill_count|sgpr_spill_count|private_segment_fixed_size):\s+(\d+)",
                                 block, re.M))
        kernels[m.group(1)] = {k: int(v) for k, v in fields.items()}
    return kernels


def test_plain_kernels_within_register_budgets(metadata):
    for sym, budget in BUDGETS.items():
        k = metadata.get(sym)
        assert k is not None, f"{sym} not in the code object"
        assert k.get("vgpr_spill_count", 0) == 0 and k.get("sgpr_spill_count", 0) == 0, (sym, k)
        assert k.get("private_segment_fixed_size", 0) == 0, (sym, k)
        assert k["vgpr_count"] <= budget, (sym, k, budget)


def test_no_plain_kernel_spills(metadata):
    for sym, k in metadata.items():
        if "k_plain" in sym or "k_digits9" in sym:
            assert k.get("vgpr_spill_count", 0) == 0 and k.get("private_segment_fixed_size", 0) == 0, (sym, k)
