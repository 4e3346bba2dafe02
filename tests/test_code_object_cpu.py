"""Resource checks on the built gfx950 code object (no GPU needed): no kernel
uses scratch memory, and the default scoring kernels (not the cell-counting
variants, which run once to measure work) fit four wavefronts per SIMD (at
most 128 VGPRs).  Either regression costs a large share of the
scoring speed without changing any result, so the parity tests would not
notice it.  Skipped when the library or the ROCm LLVM tools are absent."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1508_06561_amd", "libhs.so")
LLVM = "/opt/rocm/llvm/bin"


def kernel_metadata(tmp_path):
    tools = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not os.path.exists(LIB) or not all(os.path.exists(t) for t in tools):
        pytest.skip("library or ROCm LLVM tools not available")
    objcopy, bundler, readelf = tools
    fat = str(tmp_path / "fatbin.bin")
    co = str(tmp_path / "gfx950.co")
    subprocess.run([objcopy, f"--dump-section=.hip_fatbin={fat}", LIB, str(tmp_path / "host.o")],
                   check=True, capture_output=True)
    subprocess.run([bundler, "--unbundle", "--type=o", f"--input={fat}",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"],
                   check=True, capture_output=True)
    notes = subprocess.run([readelf, "--notes", co], check=True, capture_output=True, text=True).stdout
    kernels = {}
    cur = {}
    for line in notes.splitlines():
        m = re.match(r"\s*-?\s*\.(\w+):\s+(\S+)", line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "agpr_count" and line.lstrip().startswith("-"):
            cur = {}
        cur[key] = val
        if "name" in cur and "private_segment_fixed_size" in cur and "vgpr_count" in cur:
            kernels[cur["name"]] = (int(cur["private_segment_fixed_size"]), int(cur["vgpr_count"]))
    return kernels


def test_no_scratch_and_default_occupancy(tmp_path):
    kernels = kernel_metadata(tmp_path)
    scoring = {n: v for n, v in kernels.items() if re.search(r"k_score_(sched|batch)", n)}
    # 12 one-query kernels, 8 batch kernels with full wavefront records and
    # 12 with the smaller records of workgroups of up to 16 wavefronts
    assert len(scoring) == 32, sorted(kernels)
    assert any("k_trace_sched" in n for n in kernels) and any("k_trace_batch" in n for n in kernels)
    for name, (scratch, vgprs) in kernels.items():
        assert scratch == 0, f"{name} uses {scratch} bytes of scratch per lane"
    for name, (scratch, vgprs) in scoring.items():
        copies, count, ilp = re.search(r"ILi(\d)ELb(\d)ELb(\d)E", name).groups()
        big_groups = re.search(r"k_score_batchILi\dELb\dELb\dELi[12]E", name) is not None
        if (ilp == "0" and count == "0") or big_groups:
            assert vgprs <= 128, f"{name}: {vgprs} VGPRs (more than four wavefronts per SIMD allow)"
