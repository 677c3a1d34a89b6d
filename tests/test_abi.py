"""CPU checks of the C ABI: the library loads, exports every function that
include/pint.h declares, and rejects invalid arguments before touching a
device (no compute calls are made here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "pint.h")).read()
    return sorted(set(re.findall(r"\b(pint_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    from paper_2306_09497_amd import pint
    assert header_functions() == sorted(pint.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2306_09497_amd import pint
    lib = pint.load()
    for name in header_functions():
        assert getattr(lib, name) is not None


@pytest.mark.parametrize("cfg,msg", [
    ((0, 64, 32), "need M >= 1"),
    ((21, 64, 31), "even nlat"),
    ((21, 40, 32), "2M+2 <= nlon"),
    ((21, 66, 34), "no compiled ring FFT"),
])
def test_plan_create_rejects(cfg, msg):
    from paper_2306_09497_amd import pint
    lib = pint.load()
    c = pint.Config(cfg[0], cfg[1], cfg[2], 6.37122e6, 7.292e-5, 9.80616, 3e4, 4)
    h = ctypes.c_void_p()
    st = lib.pint_plan_create(ctypes.byref(c), None, ctypes.byref(h))
    assert st == -1 and h.value is None
    assert msg in lib.pint_last_error().decode()


def test_null_arguments():
    from paper_2306_09497_amd import pint
    lib = pint.load()
    assert lib.pint_plan_destroy(None) == -1
    assert b"null plan" in lib.pint_last_error()
    assert lib.pint_plan_create(None, None, None) == -1


def test_server_and_diagnostics_argument_checks():
    """Entry points added for serving and diagnostics refuse bad arguments
    before touching a device."""
    from paper_2306_09497_amd import pint
    lib = pint.load()
    h = ctypes.c_void_p()
    assert lib.pint_server_create(None, None, ctypes.byref(h)) == -1
    cfg = pint.ServerConfig(0, None, 1 << 20, 1, 1)
    assert lib.pint_server_create(ctypes.byref(cfg), None, ctypes.byref(h)) == -1
    assert b"n_plans >= 1" in lib.pint_last_error()
    arr = (ctypes.c_void_p * 1)(None)
    cfg = pint.ServerConfig(1, ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), 1 << 20, 1, 1)
    assert lib.pint_server_create(ctypes.byref(cfg), None, ctypes.byref(h)) == -1
    assert b"plan 0 is null" in lib.pint_last_error()
    assert lib.pint_server_destroy(None) == -1
    assert lib.pint_server_tick(None, None) == -1
    st = pint.RequestStatus()
    assert lib.pint_server_status(None, 1, ctypes.byref(st)) == -1
    assert lib.pint_ke_spectrum(None, None, None, 1, None) == -1
    assert lib.pint_spectral_errors(None, None, None, None, 1, None) == -1
    assert lib.pint_grid_l2_errors(None, None, None, None, 1, None) == -1


def test_sl_entry_points_reject_a_null_plan():
    from paper_2306_09497_amd import pint
    lib = pint.load()
    st = pint.sl_stepper(900.0)
    assert lib.pint_sl_steps(None, ctypes.byref(st), None, None, None, None, 1, 1, None) == -1
    assert b"null plan" in lib.pint_last_error()
    fine = pint.stepper(60.0)
    assert lib.pint_parareal_sl(None, ctypes.byref(fine), 4, None, ctypes.byref(st), 1, 4, 1, 2,
                                0, None, None, None) == -1
    assert b"null plan" in lib.pint_last_error()


def test_struct_layouts_match_the_header():
    """The ctypes mirrors have the sizes the C structs have under the x86-64
    ABI (double 8, int 4, natural alignment)."""
    from paper_2306_09497_amd import pint
    assert ctypes.sizeof(pint.Stepper) == 32          # double, int (+4), double, unsigned (+4)
    assert ctypes.sizeof(pint.SlStepper) == 24        # double, int, int, double
    assert pint.SlStepper.traj_iters.offset == 8 and pint.SlStepper.visc_nu.offset == 16


def test_struct_layouts_match_a_c_compiler(tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal those the host C
    compiler gives the structs of include/pint.h."""
    import shutil
    import subprocess
    from paper_2306_09497_amd import pint
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"pint_config": pint.Config, "pint_stepper": pint.Stepper,
               "pint_sl_stepper": pint.SlStepper, "pint_info": pint.Info,
               "pint_pint_params": pint.PintParams, "pint_report": pint.Report,
               "pint_server_config": pint.ServerConfig, "pint_request": pint.Request,
               "pint_request_status": pint.RequestStatus, "pint_prof_entry": pint.ProfEntry,
               "pint_stability_cfg": pint.StabilityCfg}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pint.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        cname, what, val = line.split()
        cls = mirrors[cname]
        got = ctypes.sizeof(cls) if what == "size" else getattr(cls, what).offset
        assert got == int(val), (cname, what, got, val)


def test_workspace_query_rejects_bad_arguments():
    from paper_2306_09497_amd import pint
    lib = pint.load()
    n = ctypes.c_size_t()
    assert lib.pint_plan_workspace_bytes(None, None, None, ctypes.byref(n)) == -1
    assert b"null plan" in lib.pint_last_error()
    assert lib.pint_plan_reserve(None, None, None, None) == -1


def test_binding_refuses_undersized_and_host_arrays():
    """The binding checks an array's size (and that it is a contiguous
    float64 device tensor) before the library sees its pointer, so an
    undersized tensor raises instead of being read or written out of bounds."""
    import torch
    from paper_2306_09497_amd import pint
    with pytest.raises(ValueError, match="holds 10 doubles, the call needs 12"):
        pint._ptr(torch.zeros(10, dtype=torch.float64), 12)
    with pytest.raises(ValueError, match="contiguous float64"):
        pint._ptr(torch.zeros(12, dtype=torch.float64), 12)       # host memory
    with pytest.raises(ValueError, match="contiguous float64"):
        pint._ptr(torch.zeros(12, dtype=torch.float32), 12)
    assert pint._ptr(None, 12) is None
