"""The C-ABI library loads, exports what include/tm.h declares, and validates arguments
on the host before any device work (CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

import paper_1809_05608_amd.tm as tm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tm.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = tm.load_library()
    declared = _declared_functions()
    assert set(declared) == set(tm.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(tmp_path):
    """ctypes structures have the sizes and field offsets a C compiler gives include/tm.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"tm_problem": tm.Problem, "tm_inputs": tm.Inputs, "tm_stats": tm.Stats,
               "tm_ye_inputs": tm.YeInputs, "tm_ye_stats": tm.YeStats, "tm_eadv_inputs": tm.EadvInputs}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                     check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(out[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def test_status_strings():
    lib = tm.load_library()
    for code, name in tm.STATUS_NAMES.items():
        assert lib.tm_status_string(code).decode() == name


def _prob(**kw):
    base = dict(S=1, R=4, I=16, N=12, c_dt=3e4)
    base.update({k: v for k, v in kw.items() if k in base})
    extra = {k: v for k, v in kw.items() if k not in base}
    return tm.make_problem(base["S"], base["R"], base["I"], base["N"], base["c_dt"], **extra)


@pytest.mark.parametrize("bad", [dict(N=0), dict(N=33), dict(I=0), dict(R=0), dict(S=0), dict(c_dt=0.0),
                                 dict(c_dt=float("nan")), dict(outer_bc=7), dict(outer_bc=3), dict(terms=8), dict(limiter=3),
                                 dict(psi_floor=0.0), dict(precision=3)])
def test_invalid_problem_rejected_before_device_work(bad):
    lib = tm.load_library()
    p = _prob(**bad)
    h = ctypes.c_void_p()
    assert lib.tm_create(ctypes.byref(p), None, ctypes.byref(h)) == 1      # TM_ERR_INVALID_ARG
    assert not h.value
    assert lib.tm_workspace_bytes(ctypes.byref(p), 0) == 0


def test_workspace_bytes_formula():
    lib = tm.load_library()
    p = _prob(S=4, R=10, I=540, N=20)
    per64 = 540 * 20 * 21 * 8          # I * NT * (NT + 1) * 8, NT = 20
    pad = 15                           # spare slots of a last partial wave group
    assert lib.tm_workspace_bytes(ctypes.byref(p), 0) == (40 + pad) * per64
    assert lib.tm_workspace_bytes(ctypes.byref(p), 3) == (3 + pad) * per64
    pm = _prob(S=4, R=10, I=540, N=13, precision=tm.PREC_MIXED)
    assert lib.tm_workspace_bytes(ctypes.byref(pm), 1) == (1 + pad) * 540 * 16 * 17 * 4   # padded to 16, float32
    assert lib.tm_workspace_bytes(ctypes.byref(p), -1) == 0


def test_null_context_is_an_error():
    lib = tm.load_library()
    assert lib.tm_destroy(None) == 1
    assert lib.tm_last_error(None).decode() == "context is NULL"


def test_ye_workspace_bytes_formula():
    """The coupled step keeps, per ray and zone, C [2NT][2NT+1] and y [2NT+1] in float64, padded by one
    double to an even count (16-byte aligned slots)."""
    lib = tm.load_library()
    p = _prob(S=4, R=10, I=540, N=20)
    per = 540 * (41 * 41 + 1) * 8
    assert lib.tm_ye_workspace_bytes(ctypes.byref(p), 0) == 10 * per
    assert lib.tm_ye_workspace_bytes(ctypes.byref(p), 3) == 3 * per
    p13 = _prob(S=2, R=10, I=7, N=13)                  # padded to 16 groups: blocks of 33
    assert lib.tm_ye_workspace_bytes(ctypes.byref(p13), 1) == 7 * (33 * 33 + 1) * 8
    assert lib.tm_ye_workspace_bytes(ctypes.byref(_prob(N=29)), 0) == 0     # 2 NT + 1 rows exceed a wavefront
    assert lib.tm_ye_workspace_bytes(ctypes.byref(p), -1) == 0


def test_ye_entry_points_reject_a_null_context():
    lib = tm.load_library()
    assert lib.tm_ye_newton_step(None, None, None, None, None, None, 1, 0.0, None) == 1
    assert lib.tm_temperature_update(None, None, None, None, None, None, None, None, None, None) == 1


def test_energy_advect_rejects_a_null_context():
    lib = tm.load_library()
    assert lib.tm_energy_advect(None, None, None, None, None, None) == 1


def test_kernel_timing_rejects_a_null_context():
    lib = tm.load_library()
    ms = ctypes.c_double(0.0)
    assert lib.tm_set_kernel_timing(None, 1) == 1
    assert lib.tm_kernel_time_ms(None, ctypes.byref(ms)) == 1
