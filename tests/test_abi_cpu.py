"""CPU-only checks of the C-ABI library: it loads and exports every symbol
declared in include/sft.h (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sft.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sft_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("sft_create", "sft_add_grid", "sft_add_realizations", "sft_set_state",
                     "sft_get_state", "sft_advance", "sft_assimilate", "sft_diagnostics", "sft_time",
                     "sft_destroy", "sft_status_string", "sft_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2501_06377_amd import _abi
    L = _abi.load()
    names = declared_symbols()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(_abi.SIGNATURES), set(names) ^ set(_abi.SIGNATURES)


def test_host_only_entry_points():
    from paper_2501_06377_amd import _abi, make_options
    L = _abi.load()
    o = make_options()
    assert o.precision == _abi.SFT_FP64 and o.cfl_safety == 0.9 and o.diag_every_call == 1
    assert L.sft_status_string(_abi.SFT_ERR_NOT_FINITE) == b"field holds NaN or Inf"
    assert L.sft_options_default(None) == _abi.SFT_ERR_ARG
    assert L.sft_advance(None, 1.0) == _abi.SFT_ERR_ARG
    ctx = ctypes.c_void_p()
    for kw in ({"cfl_safety": 1.5}, {"rfe_model": 3, "rfe_phi_hr": 1e23},
               {"rfe_model": 2, "rfe_phi_hr": 0.0}, {"rfe_model": 1, "rfe_phi_hr": 1e23, "rfe_lifetime_h": -1.0},
               {"rfe_model": 2, "rfe_phi_hr": float("inf")}, {"strang": 2}, {"dt_min": -1.0},
               {"dt_min": float("nan")}, {"att_cfl": 2}):
        bad = make_options(**kw)
        assert L.sft_create(ctypes.byref(ctx), ctypes.byref(bad), None) == _abi.SFT_ERR_ARG, kw
    assert L.sft_last_error(None) == b""
    # the per-step attenuated CFL limit is not combined with flux emergence
    both = make_options(att_cfl=1, rfe_model=2, rfe_phi_hr=1e23)
    assert L.sft_create(ctypes.byref(ctx), ctypes.byref(both), None) == _abi.SFT_ERR_UNSUPPORTED


def test_struct_layouts_match_header(tmp_path):
    """ctypes structures have the sizes and field offsets the C compiler gives."""
    import subprocess
    from paper_2501_06377_amd import _abi
    fields = {"sft_options": ["cfl_safety", "use_graphs", "diag_every_call", "strang", "rfe_model", "lanes",
                              "rfe_seed", "rfe_phi_hr", "rfe_lifetime_h", "dt_min", "att_cfl"],
              "sft_params": ["nu_km2_s", "lat_lim_deg", "flux_balance", "att_b0", "nu_grid_alpha"],
              "sft_diag": ["steps", "phi_pos", "nonfinite", "surr_accept"]}
    lines = ['#include "sft.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("%zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = []
    for st, fs in fields.items():
        cls = getattr(_abi, st)
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f).offset for f in fs]
    assert got == want


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before torch must not map a second HIP runtime:
    torch's device pointers and streams are only valid in its own runtime."""
    import subprocess
    import sys
    code = (
        "import paper_2501_06377_amd._abi as a\n"
        "a.load()\n"
        "import torch\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "libs = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
        "print(len(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=__import__("os").path.dirname(__import__("os").path.dirname(__file__)))
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
