"""Hot kernels of the built library use no scratch (private) memory.

Scratch accesses go through the memory hierarchy and are easy to introduce
without noticing: a copy of a local struct the compiler cannot keep in
registers once cost the kick 1.8 us of its 14.4 us per launch.  This test
reads the kernel descriptors of the gfx950 code objects the build produced
(per-source objects under paper_2001_03180_amd/_build, unbundled with the
ROCm LLVM tools) and checks `.private_segment_fixed_size` of the kernels on
the GBS step, force and adjoint paths.  CPU only: it inspects the build, it
runs nothing on a GPU.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_2001_03180_amd", "_build")
LLVM = "/opt/rocm/llvm/bin"

# (object file, kernel name pattern) pairs that must not use scratch
HOT = [
    ("kernels_step.o", r"k_kick"),
    ("kernels_step.o", r"k_drift"),
    ("kernels_force.o", r"k_force_mut"),
    ("kernels_force.o", r"k_forceILi1E"),          # the pairwise kernel as built for use (one i-body per lane)
    ("kernels_adjoint.o", r"k_adj_(fwd|rev|combine)"),
]


def _tool(name):
    path = os.path.join(LLVM, name)
    return path if os.path.exists(path) else shutil.which(name)


def _private_sizes(obj, tmp):
    objcopy, bundler, readelf = _tool("llvm-objcopy"), _tool("clang-offload-bundler"), _tool("llvm-readelf")
    if not (objcopy and bundler and readelf):
        pytest.skip("ROCm LLVM tools not found")
    fb = os.path.join(tmp, os.path.basename(obj) + ".fatbin")
    co = os.path.join(tmp, os.path.basename(obj) + ".gfx950.o")
    subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fb}", obj, os.path.join(tmp, "host.o")], check=True,
                   capture_output=True)
    subprocess.run([bundler, "--unbundle", "--type=o", f"--input={fb}", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                    f"--output={co}"], check=True, capture_output=True)
    notes = subprocess.run([readelf, "--notes", co], check=True, capture_output=True, text=True).stdout
    sizes, name = {}, None
    for line in notes.splitlines():   # metadata keys are sorted: .name precedes .private_segment_fixed_size
        m = re.match(r"\s+\.name:\s+(\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.match(r"\s+\.private_segment_fixed_size:\s+(\d+)", line)
        if m and name:
            sizes[name] = int(m.group(1))
            name = None
    return sizes


@pytest.mark.parametrize("obj,pattern", HOT)
def test_hot_kernels_use_no_scratch(obj, pattern, tmp_path):
    path = os.path.join(BUILD, obj)
    if not os.path.exists(path):
        pytest.skip("library not built (run __graft_entry__.build())")
    sizes = _private_sizes(path, str(tmp_path))
    hit = {k: v for k, v in sizes.items() if re.search(pattern, k)}
    assert hit, (obj, pattern, sorted(sizes)[:5])
    bad = {k: v for k, v in hit.items() if v != 0}
    assert not bad, bad
