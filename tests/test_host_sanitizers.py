"""Host code of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tm_api.hip is compiled again with the sanitizers on its host pass only (each -fsanitize= follows
-Xarch_host; the device code is built as usual) and linked with the library's other objects and the
checks of tests/host/abi_host_checks.c: argument validation, workspace formulas, status strings and NULL
contexts, the paths a caller reaches before any device work.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

from paper_1809_05608_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def test_abi_host_code_is_clean_under_sanitizers(tmp_path):
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    objs = {s: os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o") for s in B.SOURCES}
    def stale(s):
        o = objs[s]
        return not os.path.exists(o) or os.path.getmtime(o) < os.path.getmtime(os.path.join(B.CSRC, s))
    if any(stale(s) for s in B.SOURCES):
        B.build()
    api = str(tmp_path / "tm_api_san.o")
    cmd = [hipcc, *B.flags(), *SAN, "-g", "-c", os.path.join(B.CSRC, "tm_api.hip"), "-o", api]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    drv = str(tmp_path / "abi_host_checks.o")
    subprocess.run([shutil.which("gcc") or "cc", "-g", "-fsanitize=address,undefined", "-I",
                    os.path.join(ROOT, "include"), "-c", os.path.join(HOST, "abi_host_checks.c"), "-o", drv],
                   check=True, capture_output=True, text=True)
    exe = str(tmp_path / "abi_host_checks")
    others = [o for s, o in objs.items() if s != "tm_api.hip"]
    link = [hipcc, f"--offload-arch={B.ARCH}", "-fsanitize=address,undefined", drv, api, *others, "-o", exe]
    subprocess.run(link, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
    assert "abi host checks passed" in out
