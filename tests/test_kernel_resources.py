"""The hot-path kernels of the built library use no scratch memory (CPU only).

Reads the kernel metadata of the gfx950 code objects compiled from this repository's sources (the
objects under _build/ that paper_1809_05608_amd.build links into libtm.so).  A kernel whose register
arrays spill, or whose unrolled loops end up indexed at run time, gets a private segment; on this
method that has cost several times the kernel's own time (the coupled factor kernel ran 7.5 times
slower, the adjoint's VJP kernel 9 times), so it is checked here rather than found in a profile.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build")
LLVM = "/opt/rocm/llvm/bin"
SOURCES = ["tm_residual", "tm_factor", "tm_factor_geo", "tm_factor_q", "tm_ye", "tm_energy"]

# kernels that may use scratch: the debug Jacobian output and the per-zone temperature update, neither
# on a timed path
ALLOWED = [r"k_blocks", r"k_ye_temperature"]


def _kernel_scratch(obj, tmp):
    fb, co = os.path.join(tmp, "fatbin"), os.path.join(tmp, "code.o")
    subprocess.run([f"{LLVM}/llvm-objcopy", f"--dump-section=.hip_fatbin={fb}", obj, os.path.join(tmp, "x.o")],
                   check=True, capture_output=True)
    subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--input={fb}",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"], check=True, capture_output=True)
    notes = subprocess.run([f"{LLVM}/llvm-readelf", "--notes", co], check=True, capture_output=True,
                           text=True).stdout
    names = re.findall(r"^\s+\.name:\s+(\S+)", notes, flags=re.M)
    sizes = [int(v) for v in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", notes)]
    assert len(names) == len(sizes) and names, obj
    return dict(zip(names, sizes))


@pytest.mark.parametrize("src", SOURCES)
def test_hot_path_kernels_use_no_scratch(src, tmp_path):
    obj = os.path.join(BUILD, src + ".o")
    if not os.path.exists(obj) or not all(os.path.exists(f"{LLVM}/{t}") for t in
                                          ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")):
        pytest.skip("library objects or ROCm LLVM tools not present (run the build first)")
    scratch = _kernel_scratch(obj, str(tmp_path))
    bad = {k: v for k, v in scratch.items() if v and not any(re.search(a, k) for a in ALLOWED)}
    assert not bad, f"kernels with scratch: {bad}"
    shutil.rmtree(tmp_path, ignore_errors=True)
